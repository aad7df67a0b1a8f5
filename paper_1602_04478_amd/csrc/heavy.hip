// Grouped path: B sources (<= 64) and T colourings per launch.
//
// The frontier of a cycle program is organised by path length: the entries of
// depth d are the (vertex, source) pairs that a high-starting walk of d edges
// reaches (every register of that depth has a row per entry, whatever its
// annotations, since reachability does not depend on colours or tables).
// Dense groups -- the sources with the widest reach -- keep a row for every
// (v, b) with v < n_lim, and a per-vertex mask per register of the rows that
// may be nonzero.  Sparse groups list their entries: a level is a per-vertex
// 64-bit mark word (bit b: source b reaches v) built with atomic ORs, then a
// deterministic compaction numbers the marks in (vertex, source) order, so the
// entry of (v, b) is base[v] + popcount of the marks of v below b.
//
// EdgeJoin is a pull.  The main kernel is vertex-major: one wavefront owns an
// output vertex w and all sources of the group at once (lane = (source,
// trial)), reads w's neighbour list once with each neighbour's per-vertex
// source bits, and every lane adds the input row (v, b) of its own source into
// its own LDS column, slot by slot to the output slot it becomes (data edge:
// the signature gains chi(v) -- Section 5.1, DB Procedure 1) or to every
// output slot through the products with the edge table (annotated edge:
// EdgeJoin of Section 5.2).  Rows wider than an LDS column per lane allows
// take an entry-major kernel (a wavefront per output entry).  NodeJoin, AXPY
// and the merges are flat: one thread per output slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "kernels.h"
#include "slot_math.h"

namespace cc {

namespace {

using namespace dev;

constexpr int CPER = 4;            // vertices per thread in a compaction chunk
constexpr int CH = BLK * CPER;     // vertices per compaction chunk

__device__ __forceinline__ int64_t nentries(const GroupDev &g, const LevelDev &L) {
  return g.dense ? g.n_lim * (int64_t)g.B : (int64_t)(*L.cnt);
}
__device__ __forceinline__ void entry_vb(const GroupDev &g, const LevelDev &L, int64_t e, int64_t &v, int &b) {
  if (g.dense) {
    v = e / g.B;
    b = (int)(e - v * g.B);
  } else {
    int64_t x = L.list[e];
    v = x >> 6;
    b = (int)(x & 63);
  }
}
__device__ __forceinline__ int64_t sparse_entry(const LevelDev &L, int64_t v, int b) {
  const ulonglong2 p = ((const ulonglong2 *)L.mb)[v];  // marks and base in one load
  const uint64_t mm = p.x;
  const int64_t bs = (int64_t)p.y;
  return ((mm >> b) & 1ull) ? bs + __popcll(mm & ((1ull << b) - 1ull)) : (int64_t)-1;
}
__device__ __forceinline__ int64_t entry_of(const GroupDev &g, const LevelDev &L, int64_t v, int b) {
  if (g.dense) return v < g.n_lim ? v * g.B + b : -1;
  return sparse_entry(L, v, b);
}
// row of register r for (v, b), or -1 when it has none (sparse) or is known
// to be zero (dense: its activity bit is clear)
__device__ __forceinline__ int64_t row_of(const GroupDev &g, const LevelDev &L, const RegDev &r, int64_t v, int b) {
  if (g.dense) return (v < g.n_lim && ((r.mask[v] >> b) & 1ull)) ? v * g.B + b : -1;
  return sparse_entry(L, v, b);
}
__device__ __forceinline__ bool live(const GroupDev &g, const RegDev &r, int64_t v, int b) {
  return !g.dense || ((r.mask[v] >> b) & 1ull);
}
// Every later path vertex must lie below this bound: the source itself
// (degree order, Section 5.1), or no bound at all when the group runs with
// the filter off (path splitting: every vertex may follow).
constexpr int VBIG = 0x7fffffff;
__device__ __forceinline__ int64_t vbound(const GroupDev &g, int64_t u) { return g.nofilter ? (int64_t)VBIG : u; }

__device__ __forceinline__ void mark(uint64_t *m, int64_t v, int b) {
  const uint64_t bit = 1ull << b;
  if (!(m[v] & bit)) atomicOr((unsigned long long *)&m[v], (unsigned long long)bit);
}

// Work counters of a launch (profiling only; prof null otherwise): each wave
// adds its three per-thread counts into one of PROF_LANES triples (no hot
// address).  Every thread of the workgroup calls it.
__device__ __forceinline__ void prof_flush(uint64_t *prof, uint64_t c0, uint64_t c1, uint64_t c2) {
  if (!prof) return;
  for (int o = 32; o > 0; o >>= 1) {
    c0 += __shfl_xor(c0, o);
    c1 += __shfl_xor(c1, o);
    c2 += __shfl_xor(c2, o);
  }
  if ((threadIdx.x & 63) == 0) {
    uint64_t *pc = prof + 3 * ((blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) % PROF_LANES);
    if (c0) atomicAdd((unsigned long long *)&pc[0], (unsigned long long)c0);
    if (c1) atomicAdd((unsigned long long *)&pc[1], (unsigned long long)c1);
    if (c2) atomicAdd((unsigned long long *)&pc[2], (unsigned long long)c2);
  }
}

// Lanes of one wavefront see each other's LDS writes after this (the
// wavefront's LDS operations have completed and are ordered before the reads).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ levels (sparse groups)
// depth 1: the lower neighbours of each source
__global__ void k_mark_init(GraphDev g, GroupDev grp, const int32_t *lowcnt, int max_low, LevelDev L) {
  const int64_t N = (int64_t)grp.B * max_low;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / max_low), j = (int)(i - (int64_t)b * max_low);
    const int64_t u = grp.src[b];
    if (j >= lowcnt[u]) continue;
    mark(L.mb, 2 * (int64_t)g.col[g.rp[u] + j], b);
  }
}

// depth d+1 from depth d: every lower neighbour w < u_b of an entry (v, b).
// A team of lanes takes a vertex v with all its entries (the marks m of v):
// neighbour w (ascending) gets the sources b of m with w < u_b in one atomic
// OR; below the smallest such u_b that is all of m.
__global__ void k_mark_next(GraphDev g, GroupDev grp, LevelDev Lin, LevelDev Lout) {
  constexpr int TEAM = 16;
  __shared__ int32_t s_u[64];  // per source: the bound below which its walks continue
  for (int i = threadIdx.x; i < 64; i += BLK) s_u[i] = i < grp.B ? (int32_t)vbound(grp, grp.src[i]) : 0;
  __syncthreads();
  const int teams = BLK / TEAM, team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  uint64_t prd = 0, pwr = 0;  // profiling: bytes read, written
  const int64_t nvin = Lin.cnt[1];  // the input level's marked vertices (listed in order)
  for (int64_t i = (int64_t)blockIdx.x * teams + team; i < nvin; i += (int64_t)gridDim.x * teams) {
    const int64_t v = Lin.vlist[i];
    const uint64_t m = Lin.mb[2 * v];
    prd += lane == 0 ? 28 : 0;
    int umin = 0x7fffffff, umax = 0;
    for (uint64_t r = m; r; r &= r - 1) {
      const int u = s_u[__builtin_ctzll(r)];
      umin = min(umin, u);
      umax = max(umax, u);
    }
    for (int64_t ee = g.rp[v] + lane; ee < g.rp[v + 1]; ee += TEAM) {
      const int64_t w = g.col[ee];
      if (w >= umax) break;
      uint64_t mask = m;
      if (w >= umin) {
        mask = 0;
        for (uint64_t r = m; r; r &= r - 1) {
          const int b = __builtin_ctzll(r);
          if (w < s_u[b]) mask |= 1ull << b;
        }
      }
      prd += 12;
      // no read first: an atomic OR whose result is not used does not wait
      atomicOr((unsigned long long *)&Lout.mb[2 * w], (unsigned long long)mask);
      pwr += 8;
    }
  }
  prof_flush(grp.prof, prd, pwr, 0);
}

// exclusive prefix sum over the workgroup (BLK threads, all calling); the
// total in tot.  Wavefront scans by shuffles, then the wavefronts' totals
// through s (at least BLK / 64 words).
__device__ __forceinline__ uint32_t block_scan(uint32_t x, uint32_t *s, uint32_t &tot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s[wv] = inc;
  __syncthreads();
  uint32_t base = 0, t = 0;
  for (int i = 0; i < BLK / 64; i++) {
    const uint32_t c = s[i];
    base += i < wv ? c : 0u;
    t += c;
  }
  tot = t;
  __syncthreads();  // s is reused by the next call
  return base + inc - x;
}

// marks and marked vertices per chunk (thread t reads vertices lo + i * BLK + t:
// coalesced); bcnt[chunk] and bcnt[chunks + chunk]
__global__ void k_cmp_count(const uint64_t *mb, int64_t nv, uint32_t *bcnt, uint64_t *prof) {
  __shared__ uint32_t s[BLK], sv[BLK];
  const int64_t lo = (int64_t)blockIdx.x * CH;
  uint32_t c = 0, cv = 0;
  for (int i = 0; i < CPER; i++) {
    const int64_t v = lo + (int64_t)i * BLK + threadIdx.x;
    if (v < nv) {
      const uint64_t m = mb[2 * v];
      c += __popcll(m);
      cv += m != 0;
    }
  }
  s[threadIdx.x] = c;
  sv[threadIdx.x] = cv;
  __syncthreads();
  for (int o = BLK / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s[threadIdx.x] += s[threadIdx.x + o];
      sv[threadIdx.x] += sv[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bcnt[blockIdx.x] = s[0];
    bcnt[gridDim.x + blockIdx.x] = sv[0];
  }
  prof_flush(prof, threadIdx.x == 0 ? 8 * (uint64_t)max((int64_t)0, min((int64_t)CH, nv - lo)) : 0, 0, 0);
}

// exclusive scans of the chunk counts (one workgroup): entries into bcnt[0..nb)
// and cnt[0], marked vertices into bcnt[nb..2nb) and cnt[1]
__global__ void k_cmp_scan(uint32_t *bcnt, int nb, uint32_t *cnt) {
  __shared__ uint32_t s[BLK];
  const int per = (nb + BLK - 1) / BLK;
  const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, lo + per);
  for (int part = 0; part < 2; part++) {
    uint32_t *b = bcnt + part * nb;
    uint32_t sum = 0;
    for (int i = lo; i < hi; i++) sum += b[i];
    uint32_t tot;
    uint32_t run = block_scan(sum, s, tot);
    for (int i = lo; i < hi; i++) {
      const uint32_t x = b[i];
      b[i] = run;
      run += x;
    }
    if (threadIdx.x == 0) cnt[part] = tot;
  }
}

// number the marks: base[v] and the entry list, in (v, b) order, and the list
// of marked vertices in order
__global__ void k_cmp_emit(uint64_t *mb, int64_t nv, const uint32_t *boff, int64_t *list, int32_t *vlist,
                           uint64_t *prof) {
  __shared__ uint32_t s[BLK];
  const int64_t lo = (int64_t)blockIdx.x * CH;
  uint32_t run = boff[blockIdx.x], vrun = boff[gridDim.x + blockIdx.x];
  uint64_t prd = 0, pwr = 0;
  for (int i = 0; i < CPER; i++) {
    const int64_t v = lo + (int64_t)i * BLK + threadIdx.x;
    const uint64_t mm = v < nv ? mb[2 * v] : 0;
    // one scan of both counts: entries in the high 16 bits (at most 256 * 64
    // per step), marked vertices in the low 16 bits (at most 256)
    uint32_t tot;
    const uint32_t pk = block_scan(((uint32_t)__popcll(mm) << 16) | (mm != 0 ? 1u : 0u), s, tot);
    const uint32_t id0 = run + (pk >> 16), vid = vrun + (pk & 0xffffu);
    if (v < nv) {
      uint32_t id = id0;
      if (mm) {  // the base of an unmarked vertex is never read (its marks are zero)
        mb[2 * v + 1] = id0;
        for (uint64_t r = mm; r; r &= r - 1) list[id++] = v * 64 + __builtin_ctzll(r);
        vlist[vid] = (int32_t)v;
      }
      prd += 8;
      pwr += mm ? 8 + 8 * (uint64_t)__popcll(mm) + 4 : 0;
    }
    run += tot >> 16;
    vrun += tot & 0xffffu;
  }
  prof_flush(prof, prd, pwr, 0);
}

// ------------------------------------------------------------------ INIT
// dst[(x, b)] for x in the lower prefix of u_b's row:
//   value over rest R (subset of K \ {chi u, chi x}, size s-2) =
//   sum over splits R = Ra + Re of A_h[u][Ra] * E(u,x)[Re]
// (A_h absent: identity {chi u}; E absent: the data edge {chi u, chi x} -> 1).
__global__ void k_init(GraphDev g, GroupDev grp, const int32_t *lowcnt, int max_low, const uint8_t *colr, LevelDev L,
                       RegDev dst, TabDev et, int e_src_first, TabDev nt, uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int C = dst.C, T = grp.T;
  const int64_t per = (int64_t)T * C;
  const int64_t N = (int64_t)grp.B * max_low * per;
  const int sa = nt.val ? nt.s : 1;
  uint64_t ofm = 0, prd = 0, pwr = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t en = i / per;
    const int r = (int)(i - en * per), t = r / C, c = r - t * C;
    const int b = (int)(en / max_low), j = (int)(en - (int64_t)b * max_low);
    const int64_t u = grp.src[b];
    if (j >= lowcnt[u]) continue;
    const int64_t es = g.rp[u] + j;
    const int64_t x = g.col[es];
    const int64_t e = entry_of(grp, L, x, b);
    const int cu = colr[(int64_t)t * g.n + u], cx = colr[(int64_t)t * g.n + x];
    const int64_t tslot = e_src_first ? es : g.rev[es];
    uint64_t acc = 0;
    bool of = false;
    if (cu != cx) {
      const uint32_t R = spread2(unrank(lut, dst.s - 2, c), cu, cx);
      uint32_t sub = R;
      for (;;) {
        if (__popc(sub) == sa - 1) {
          const uint32_t Re = R & ~sub;
          uint64_t va = nt.val ? nt.val[(u * T + t) * nt.C + s_rank[squeeze1(sub, cu)]] : 1;
          uint64_t ve = et.val ? et.val[(tslot * T + t) * et.C + s_rank[squeeze2(Re, cu, cx)]] : (Re ? 0 : 1);
          if (va && ve) add_ck(acc, mul_ck(va, ve, of), of);
        }
        if (sub == 0) break;
        sub = (sub - 1) & R;
      }
    }
    dst.val[e * per + r] = acc;
    if (grp.dense && r == 0) atomicOr((unsigned long long *)&dst.mask[x], 1ull << b);
    if (of) ofm |= 1ull << t;
    pwr += 8;
    if (c == 0) prd += 4 + 2 + 8 * ((nt.val ? nt.C : 0) + (et.val ? et.C : 0));
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

// ------------------------------------------------------------------ EdgeJoin
// dst[(w,b)][R'] = sum over v in N(w), v < u_b, (v,b) an entry of the lower
// level, of sum over splits R' \ {chi v} = R + Re of a[(v,b)][R] * E(v,w)[Re].
constexpr int WAVE = 64;
constexpr int VNONE = 0x7fffffff;  // no vertex (ids are below 2^31)
constexpr int VMAX_C = 96;  // slots up to which the vertex-major EdgeJoin keeps an LDS column per lane
// wavefronts per SIMD the vertex-major EdgeJoin asks of the register
// allocator (with slot maps and no epilogue): at most 96 registers, five
#ifndef EJ_MINW_SPARSE
#define EJ_MINW_SPARSE 5
#endif
#ifndef EJ_MINW_DENSE
#define EJ_MINW_DENSE 5
#endif
#ifndef EJ_PACK_SW
#define EJ_PACK_SW 16  // lanes per output vertex in sparse groups with packed pairs
#endif
#ifndef EJ_UNROLL_P
#define EJ_UNROLL_P 8  // slots of a row loaded before they are added (pairs packed over the lanes)
#endif
#ifndef EJ_UNROLL_PD
#define EJ_UNROLL_PD 12  // the same in dense groups, at four wavefronts per SIMD (EJ_MINW_PD)
#endif
#ifndef EJ_MINW_PD
#define EJ_MINW_PD 4
#endif
#ifndef EJ_UNROLL_S
#define EJ_UNROLL_S 8  // slots of a row loaded before they are added (one-neighbour steps)
#endif
#ifndef EJ_UNROLL
#define EJ_UNROLL 4  // slots of both rows loaded before they are added (two-neighbour steps)
#endif
constexpr int EJ_BLK = 256;  // four wavefronts per workgroup share the rank tables (narrow rows)

// One wavefront per output entry (w, b); per trial, w's neighbours below u_b
// are taken 64 at a time in two phases:
//   gather: lane j looks up neighbour j (its row in the input register and its
//           colour) and the usable ones are packed into LDS by a ballot;
//   relax:  the wave walks the packed (neighbour, slot) pairs, lane i taking
//           pairs i, i + 64, ..., loading four input values before it adds
//           them, so rows are read contiguously and many loads are in flight.
// Data edge: input slot c goes to the output slot with chi(v) added (Section
// 5.1).  Annotated edge: lanes take (neighbour, output slot) pairs and sum the
// products over the splits of the output signature (EdgeJoin of Section 5.2).
// Accumulation in LDS in split 32-bit halves (non-returning adds that cannot
// overflow), joined and checked when the row is written.
template <bool ANN>
__global__ __launch_bounds__(WAVE) void k_ej(GraphDev g, GroupDev grp, const uint8_t *colr, LevelDev Lin,
                                             LevelDev Lout, RegDev a, RegDev dst, TabDev et, int e_src_first,
                                             uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint32_t s_um[256];  // unranked slots: input (data edge) or output (annotated)
  __shared__ int64_t s_id[WAVE];  // packed neighbours: input row
  __shared__ int64_t s_ts[WAVE];  //   annotated edge's table slot
  __shared__ uint8_t s_cv[WAVE];  //   colour
  extern __shared__ uint64_t acc[];  // [T][C][2]
  load_rank(s_rank, lut);
  const int T = grp.T, C = dst.C, Ca = a.C;
  const int TC = T * C;
  const int ra = a.s - 2, ro = dst.s - 2;
  const int W = ANN ? C : Ca;  // pairs per neighbour
  for (int c = threadIdx.x; c < W; c += WAVE) s_um[c] = unrank(lut, ANN ? ro : ra, c);
  // i / W == (i * magic) >> 32 for i < 64 * 256 (magic = ceil(2^32 / W); 2^32 when W = 1)
  const uint64_t magic = (0x100000000ull + W - 1) / W;
  const int lane = threadIdx.x;
  const uint64_t lt = (1ull << lane) - 1ull;
  const int64_t N = nentries(grp, Lout);
  uint64_t ofm = 0;
  // work counters (profiling): (entry, trial, lower neighbour) pairs scanned,
  // input rows read, output rows written
  uint64_t n_scan = 0, n_rows = 0, n_ent = 0;
  for (int64_t e = blockIdx.x; e < N; e += gridDim.x) {
    __syncthreads();
    for (int q = lane; q < 2 * TC; q += WAVE) acc[q] = 0;
    int64_t w;
    int b;
    entry_vb(grp, Lout, e, w, b);
    const int64_t u = grp.src[b], ub = vbound(grp, u);
    if (w < ub) {
      const int64_t r0 = g.rp[w], r1 = g.rp[w + 1];
      for (int t = 0; t < T; t++) {
        const int cu = colr[(int64_t)t * g.n + u], cw = colr[(int64_t)t * g.n + w];
        if (cu == cw) continue;
        uint64_t *at_acc = acc + 2 * t * C;
        const uint64_t *abase = a.val + (int64_t)t * Ca;
        for (int64_t j0 = r0; j0 < r1; j0 += WAVE) {
          // gather
          const int64_t ee = j0 + lane;
          const int64_t v = ee < r1 ? g.col[ee] : INT64_MAX;
          const bool in = v < ub;
          bool ok = false;
          int64_t id = -1;
          int cv = 0;
          if (in) {
            id = row_of(grp, Lin, a, v, b);
            if (id >= 0) {
              cv = colr[(int64_t)t * g.n + v];
              ok = cv != cu && cv != cw;
            }
          }
          n_scan += id >= 0;  // a key of source b at v below u_b
          n_rows += ok;
          const uint64_t okm = __ballot(ok);
          const bool stop = __ballot(!in) != 0;
          __syncthreads();  // the previous chunk's relax phase is done with the packed lists
          if (ok) {
            const int pos = __popcll(okm & lt);
            s_id[pos] = id;
            s_cv[pos] = (uint8_t)cv;
            if (ANN) s_ts[pos] = e_src_first ? g.rev[ee] : ee;
          }
          __syncthreads();
          // relax
          const int items = __popcll(okm) * W;
          if (!ANN) {
            for (int i0 = lane; i0 < items; i0 += 4 * WAVE) {
              uint64_t x[4];
              int jn[4], c[4];
#pragma unroll
              for (int q = 0; q < 4; q++) {
                const int i = i0 + q * WAVE;
                jn[q] = (int)(((uint64_t)(uint32_t)i * magic) >> 32);
                c[q] = i - jn[q] * W;
                x[q] = i < items ? abase[s_id[jn[q]] * T * Ca + c[q]] : 0;
              }
#pragma unroll
              for (int q = 0; q < 4; q++) {
                if (!x[q]) continue;
                const int cvq = s_cv[jn[q]];
                const uint32_t R = spread2(s_um[c[q]], cu, cvq);
                if ((R >> cw) & 1u) continue;
                const int o = s_rank[squeeze2(R | (1u << cvq), cu, cw)];
                atomicAdd((unsigned long long *)&at_acc[2 * o], (unsigned long long)(x[q] & 0xffffffffull));
                atomicAdd((unsigned long long *)&at_acc[2 * o + 1], (unsigned long long)(x[q] >> 32));
              }
            }
          } else {
            for (int i = lane; i < items; i += WAVE) {
              const int jn = (int)(((uint64_t)(uint32_t)i * magic) >> 32);
              const int co = i - jn * W;
              const int cvq = s_cv[jn];
              const uint32_t Rp = spread2(s_um[co], cu, cw);
              if (!((Rp >> cvq) & 1u)) continue;
              const uint32_t R = Rp & ~(1u << cvq);
              const uint64_t *at = abase + s_id[jn] * T * Ca;
              const uint64_t *er = et.val + (s_ts[jn] * T + t) * et.C;
              uint64_t sum = 0;
              bool of = false;
              uint32_t s1 = R;
              for (;;) {
                if (__popc(s1) == ra) {
                  const uint64_t xa = at[s_rank[squeeze2(s1, cu, cvq)]];
                  if (xa) {
                    const uint64_t y = er[s_rank[squeeze2(R & ~s1, cvq, cw)]];
                    if (y) add_ck(sum, mul_ck(xa, y, of), of);
                  }
                }
                if (s1 == 0) break;
                s1 = (s1 - 1) & R;
              }
              if (sum) {
                atomicAdd((unsigned long long *)&at_acc[2 * co], (unsigned long long)(sum & 0xffffffffull));
                atomicAdd((unsigned long long *)&at_acc[2 * co + 1], (unsigned long long)(sum >> 32));
              }
              if (of) ofm |= 1ull << t;
            }
          }
          if (stop) break;
        }
      }
    }
    __syncthreads();
    uint64_t *drow = dst.val + e * (int64_t)TC;
    bool nz = false;
    for (int q = lane; q < TC; q += WAVE) {
      const uint64_t lo = acc[2 * q], hi = acc[2 * q + 1];
      // value = hi * 2^32 + lo, both halves sums of 32-bit parts
      const uint64_t hs = hi + (lo >> 32);
      if (hs >> 32) ofm |= 1ull << (q / C);
      const uint64_t v = (hs << 32) | (lo & 0xffffffffull);
      drow[q] = v;
      nz |= v != 0;
    }
    if (grp.dense) {
      // the activity words were cleared before the launch (every bit of
      // them, also the bits of sources this group does not have)
      const bool any = __any(nz);
      if (lane == 0) {
        if (any) atomicOr((unsigned long long *)&dst.mask[w], 1ull << b);
        n_ent += any;
      }
    } else if (lane == 0) {
      n_ent++;
    }
  }
  flag_trials(ovf, ofm);
  if (grp.prof) {
    for (int o = 32; o > 0; o >>= 1) {
      n_scan += __shfl_xor(n_scan, o);
      n_rows += __shfl_xor(n_rows, o);
      n_ent += __shfl_xor(n_ent, o);
    }
    if (lane == 0) {
      uint64_t *pc = grp.prof + 3 * (blockIdx.x % PROF_LANES);  // spread over lanes: no hot address
      atomicAdd((unsigned long long *)&pc[0], (unsigned long long)n_scan);
      atomicAdd((unsigned long long *)&pc[1], (unsigned long long)n_rows);
      atomicAdd((unsigned long long *)&pc[2], (unsigned long long)n_ent);
    }
  }
}

// Vertex-major EdgeJoin.  A group of SW lanes (a whole wavefront, or a
// quarter of one when few sources meet at a vertex) owns an output vertex w,
// lane = (source b, trial t).  All sources of the group share w's neighbour
// list, so each neighbour v is read once with its per-vertex bits (which
// sources have an input row at v), and every lane then relaxes its own row
// (v, b) for its trial into its own LDS column: no atomics, checked 64-bit
// adds.  A pass takes the next SW / T sources among w's output bits.  Groups
// talk only through ballots and shuffles inside the group, so groups of one
// wavefront may follow different vertices.
__device__ __forceinline__ int nth_set_bit(uint64_t m, int k) {  // k < popcount(m)
  int pos = 0;
  for (int sh = 32; sh; sh >>= 1) {
    const uint64_t lo = m & ((1ull << sh) - 1ull);
    const int c = __popcll(lo);
    if (k >= c) {
      k -= c;
      m >>= sh;
      pos += sh;
    } else {
      m = lo;
    }
  }
  return pos;
}

// dynamic LDS of k_ejv: lane-owned columns, then (with an epilogue) the
// operands' rows, the unrank lists and the root-merge sums
__host__ __device__ constexpr size_t ejv_lds(int ncols, int nregs, bool epi, int nb) {
  return (size_t)ncols * nb * 8 + (epi ? (size_t)nregs * nb * 8 + (LUT_SIZE - LUT_UNRANK) * 2 + 2 * WAVE * 8 : 0);
}
constexpr size_t EJV_LDS_MAX = 56 * 1024;

// With MAP, the slot arithmetic of a relaxation (the input row's slot c, the
// source's colour cu, the neighbour's colour cv and the output vertex's colour
// cw give the output slot, or none when cw is already used) is read from a
// table [cu][cv][cw][c] of bytes (0xff: none), four slots per LDS word.
//
// With PACK (one trial, slot maps, no epilogue) the lanes of a group do
// not each wait for their own source's rows: the (neighbour, source) pairs of
// a step of SW neighbours that relax a row are numbered by an exclusive scan
// of their counts, and each lane takes one pair a round, adding into the
// source's column with LDS atomics (checked through the returned old value).
//
// With DUAL (packed only) the launch also runs a second EdgeJoin whose input
// register epi.in2 lies at the same level as a: both share the neighbour scan
// (the lists, the activity words or marks, the colours), a pair names its
// input, and the second output is epi.regs[1] in the LDS columns after the
// first's.  The profile counts slots instead of rows.
template <bool ANN, int SW, bool EPI, int NB, bool MAP, bool PACK = false, bool DUAL = false>
__global__ __launch_bounds__(NB, MAP && !EPI ? (SW == 16 ? EJ_MINW_SPARSE : PACK ? EJ_MINW_PD : EJ_MINW_DENSE) : 1) void k_ejv(GraphDev g, GroupDev grp, const uint8_t *colr, LevelDev Lin, RegDev a,
                                              const Epilogue epi, TabDev et, int e_src_first, uint32_t *ovf,
                                              AccDev accd, const uint16_t *lut, const uint32_t *emap, int emap_w,
                                              int emap_cp) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint32_t s_um[256];  // unranked slots: input (data edge) or output (annotated)
  __shared__ int32_t s_src[WAVE];
  __shared__ int32_t s_bnd[WAVE];  // per source: its walks' bound (itself, or none with the filter off)
  __shared__ uint64_t s_live[EPI_MAX_REGS * (NB / SW)];  // dense: per written register and group, live rows
  extern __shared__ uint64_t accs[];  // [columns][64]: lane-owned columns, EdgeJoin output first
  int64_t *const s_rid = (int64_t *)(accs + (size_t)epi.ncols * NB);  // [regs][64] operands' rows
  uint16_t *const s_unr = (uint16_t *)(s_rid + (size_t)epi.nregs * NB);  // unrank lists and offsets
  uint64_t *const s_msum = (uint64_t *)(s_unr + (LUT_SIZE - LUT_UNRANK));  // [64] x (lo, hi)
  load_rank(s_rank, lut);
  const int tid = threadIdx.x;
  if (EPI) {
    if (tid < 2 * WAVE) s_msum[tid] = 0;
    for (int i = tid; i < LUT_SIZE - LUT_UNRANK; i += NB) s_unr[i] = lut[LUT_UNRANK + i];
  }
  // unranked slot idx of rank r from the LDS copy (layout of the global table, shifted)
  auto unr = [&](int r, int idx) -> uint32_t { return s_unr[s_unr[LUT_OFF - LUT_UNRANK + r] + idx]; };
  const LevelDev Lout = epi.regs[0].L;
  const RegDev dst = epi.regs[0].r;
  uint64_t *const acc = accs + (size_t)epi.regs[0].col * NB;
  const int T = grp.T, B = grp.B, C = dst.C, Ca = a.C;
  const int ra = a.s - 2, ro = dst.s - 2;
  const int W = ANN ? C : Ca;
  const int lane = tid % WAVE;
  for (int c = tid; c < W; c += NB) s_um[c] = unrank(lut, ANN ? ro : ra, c);
  if (tid < WAVE) {
    s_src[tid] = tid < B ? grp.src[tid] : -1;
    s_bnd[tid] = tid < B ? (int32_t)vbound(grp, grp.src[tid]) : -1;
  }
  uint32_t *const s_map = (uint32_t *)((char *)accs + ejv_lds(epi.ncols, epi.nregs, EPI, NB));
  if (MAP)
    for (int i = tid; i < emap_w; i += NB) s_map[i] = emap[i];
  uint32_t *const s_map2 = s_map + emap_w;  // DUAL: the second input's map
  if (DUAL)
    for (int i = tid; i < epi.map2_w; i += NB) s_map2[i] = epi.map2[i];
  const int Ca2 = DUAL ? epi.in2.C : 0, col2 = DUAL ? epi.regs[1].col : 0;
  __shared__ uint64_t s_cm[16];  // PACK: the sources of each colour (bit b: source b)
  __shared__ uint8_t s_cu[WAVE];  // PACK: source b's colour
  if (PACK) {
    if (tid < 16) s_cm[tid] = 0;
    __syncthreads();
    if (tid < B) {
      const int c = colr[grp.src[tid]];
      s_cu[tid] = (uint8_t)c;
      atomicOr((unsigned long long *)&s_cm[c], 1ull << tid);
    }
  }
  __syncthreads();
  constexpr int NG = WAVE / SW;  // groups per wavefront
  const int gl = lane % SW, gbase = lane - gl;
  const uint64_t gmask = SW == 64 ? ~0ull : ((1ull << SW) - 1ull);
  auto gballot = [&](bool p) -> uint64_t { return ((uint64_t)__ballot(p) >> gbase) & gmask; };
  const int Bc = SW / T;                 // sources per pass
  const int lt = gl % T, lb = gl / T;    // lane's trial, its source's slot in the pass
  const int64_t n = g.n;
  const uint32_t Kmask = (1u << grp.k) - 1u;
  uint64_t ofm = 0;
  uint32_t n_scan = 0, n_rows = 0, n_ent = 0;  // profile counts of this lane (each below 2^32 per launch)
  uint64_t mlo = 0, mhi = 0;  // this lane's root-merge sum (its trial)
  constexpr int WPB = NB / WAVE;  // wavefronts per workgroup
  // Work items.  Dense groups with a hub schedule: first the chunks of the
  // hubs' neighbour lists (a wavefront each, partial rows added atomically
  // into rows cleared before the launch), then the other vertices from the
  // highest down.  Otherwise one item per output vertex, ascending.
  // Vertex ids fit 31 bits (the graph's limit), so they travel as int.
  const bool hsplit = !EPI && grp.dense && grp.nh > 0;
  const uint32_t nh = hsplit ? (uint32_t)grp.nh : 0u;
  const uint32_t nlight = (uint32_t)(hsplit ? min(grp.n_lim, grp.split_lo) : grp.n_lim);
  // sparse groups: only the vertices the output level marks (listed in order)
  const uint32_t nitems = grp.dense ? nh + nlight : Lout.cnt[1], wstride = gridDim.x * WPB * NG;
  for (uint32_t wl = (blockIdx.x * WPB + tid / WAVE) * NG + lane / SW; wl < nitems; wl += wstride) {
    int w;
    int64_t r0, r1;  // the item's neighbour range
    bool split = false, first_chunk = true;
    if (wl < nh) {
      w = grp.hitems[2 * wl];
      const int off = grp.hitems[2 * wl + 1];
      const int64_t a1 = g.rp[w + 1];
      r0 = g.rp[w] + off;
      r1 = min(a1, r0 + (int64_t)grp.split_chunk);
      split = true;
      first_chunk = off == 0;
    } else {
      w = !grp.dense ? Lout.vlist[wl] : hsplit ? (int)(nlight - 1u - (wl - nh)) : (int)wl;
      // w's edge range is loaded with its marks, not after them (one step
      // less on the chain of dependent loads)
      r0 = g.rp[w];
      r1 = g.rp[w + 1];
    }
    // output rows at w: dense -- every source above w; sparse -- the marks
    uint64_t ob = 0;
    if (grp.dense) {
      for (int i = 0; i < B; i += SW) ob |= gballot(i + gl < B && s_bnd[i + gl] > w) << i;
    } else {
      ob = Lout.mb[2 * (int64_t)w];
    }
    if (!ob) {
      if (grp.dense && gl == 0 && !split)
        for (int j = 0; j < epi.nregs; j++)
          if (epi.regs[j].write) epi.regs[j].r.mask[w] = 0;
      continue;
    }
    if (grp.dense && gl == 0)
      for (int j = 0; j < epi.nregs; j++) s_live[j * (NB / SW) + tid / SW] = 0;
    uint64_t rest = ob;
    while (rest) {
      // this pass: the first Bc sources of rest
      const int nr = __popcll(rest);
      const int np = nr < Bc ? nr : Bc;
      const int last = nth_set_bit(rest, np - 1);
      const uint64_t pass = last == 63 ? rest : rest & ((1ull << (last + 1)) - 1ull);
      rest &= ~pass;
      const int b = lb < np ? nth_set_bit(pass, lb) : -1;
      const int u = b >= 0 ? s_src[b] : 0;
      const int ub = b >= 0 ? s_bnd[b] : 0;
      int umax = ub;  // the neighbours below the pass's largest bound
      for (int o = SW / 2; o > 0; o >>= 1) umax = max(umax, __shfl_xor(umax, o, SW));
      int cu = 0, cw = 0;
      bool act = false;
      if (b >= 0) {
        cu = colr[(int64_t)lt * n + u];
        cw = colr[(int64_t)lt * n + w];
        act = cu != cw;
      }
      for (int o = 0; o < epi.ncols; o++) accs[o * NB + tid] = 0;
      bool of = false;
      for (int64_t j0 = r0; j0 < r1; j0 += SW) {
        const int64_t ee = j0 + gl;
        int vj = ee < r1 ? g.col[ee] : VNONE;
        if (vj >= umax) vj = VNONE;
        uint64_t inb = 0, mfull = 0, inb2 = 0;
        int64_t bj = 0;
        if (vj != VNONE) {
          if (grp.dense) {
            inb = a.mask[vj];
            if (DUAL) inb2 = epi.in2.mask[vj] & pass;
          } else {
            const ulonglong2 p = ((const ulonglong2 *)Lin.mb)[vj];
            mfull = p.x;
            bj = (int64_t)p.y;
            inb = mfull;
            if (DUAL) inb2 = mfull & pass;
          }
          inb &= pass;
        }
        if (grp.prof) {
          // (key, trial, lower neighbour) triples: the pass's sources b with an
          // input row at v = vj (bit set in inb), v below u_b, and a trial in
          // which b is not idle at w (its colour differs from w's)
          for (uint64_t r = inb | inb2; r; r &= r - 1) {
            const int uq = s_src[__builtin_ctzll(r)];
            if (vj < s_bnd[__builtin_ctzll(r)])
              for (int t = 0; t < T; t++) n_scan += colr[(int64_t)t * n + uq] != colr[(int64_t)t * n + w] ? 1u : 0u;
          }
        }
        uint64_t todo = gballot(inb != 0);
        const bool stop = gballot(vj == VNONE) != 0;
        // one trial: the neighbour's colour travels with it (loaded by its own lane)
        const int cvj = (T == 1 && (inb | inb2)) ? colr[vj] : 0;
        if (PACK) {
          // sources that relax a row from neighbour j: bit set in inb, colour
          // neither the neighbour's nor w's (w's colour: the source is idle at w)
          const int cwv = colr[w];
          const uint64_t valid = (inb && cvj != cwv) ? inb & ~s_cm[cvj] & ~s_cm[cwv] : 0ull;
          const uint64_t valid2 = (DUAL && inb2 && cvj != cwv) ? inb2 & ~s_cm[cvj] & ~s_cm[cwv] : 0ull;
          const int own = __popcll(valid) + (DUAL ? __popcll(valid2) : 0);
          int incl = own;
          for (int o = 1; o < SW; o <<= 1) {
            const int y = __shfl_up(incl, o, SW);
            if (gl >= o) incl += y;
          }
          const int excl = incl - own, P = __shfl(incl, SW - 1, SW);
          for (int p0 = 0; p0 < P; p0 += SW) {
            const int pp = p0 + gl;
            int jl = 0;  // the last neighbour whose first pair is at or before pp
            for (int st = SW / 2; st > 0; st >>= 1)
              if (__shfl(excl, jl + st, SW) <= pp) jl += st;
            const int kth = pp - __shfl(excl, jl, SW);
            const int vA = __shfl(vj, jl, SW), cA = __shfl(cvj, jl, SW);
            const uint64_t vm = __shfl(valid, jl, SW);
            const uint64_t vm2 = DUAL ? __shfl(valid2, jl, SW) : 0ull;
            // (packed launches: whole wavefronts for dense groups, quarters for sparse ones)
            constexpr bool PD = SW == WAVE;
            const uint64_t mfA = PD ? 0 : __shfl(mfull, jl, SW);
            const int64_t bA = PD ? 0 : __shfl(bj, jl, SW);
            if (pp >= P) continue;
            // the pair's input: the first register's pairs of a neighbour come first
            const int n1 = DUAL ? __popcll(vm) : 0;
            const bool sec = DUAL && kth >= n1;
            const int bb = sec ? nth_set_bit(vm2, kth - n1) : nth_set_bit(vm, kth);
            if (vA >= s_bnd[bb]) continue;
            const int Cq = sec ? Ca2 : Ca;
            n_rows += DUAL ? (uint32_t)Cq : 1u;
            const uint64_t below_bb = (1ull << bb) - 1ull;
            const int colw = (tid - gl) + __popcll(pass & below_bb) + (sec ? col2 * NB : 0);  // source bb's column
            const int64_t rid = PD ? (int64_t)vA * B + bb : bA + __popcll(mfA & below_bb);
            const uint64_t *row = sec ? epi.in2.val + rid * Ca2 : a.val + rid * Ca;
            const uint32_t *mA = sec ? s_map2 + ((s_cu[bb] * grp.k + cA) * grp.k + cwv) * (epi.map2_cp >> 2)
                                     : s_map + ((s_cu[bb] * grp.k + cA) * grp.k + cwv) * (emap_cp >> 2);
            constexpr int UP = PD ? EJ_UNROLL_PD : EJ_UNROLL_P;
            for (int c0 = 0; c0 < Cq; c0 += UP) {
              uint64_t xa[UP];
#pragma unroll
              for (int q = 0; q < UP; q++) xa[q] = c0 + q < Cq ? row[c0 + q] : 0;
#pragma unroll
              for (int q = 0; q < UP; q++) {
                if (!xa[q]) continue;
                const uint32_t o = (mA[(c0 + q) >> 2] >> (8 * (q & 3))) & 0xffu;
                if (o == 0xffu) continue;
                const uint64_t old = atomicAdd((unsigned long long *)&accs[o * NB + colw], (unsigned long long)xa[q]);
                of |= old + xa[q] < old;
              }
            }
          }
        } else if (!ANN && SW < 64) {
          // quarter wavefronts: one neighbour per step, few registers (more
          // wavefronts in flight hide the per-vertex load chains)
          while (todo) {
            const int jA = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int vA = __shfl(vj, jA, SW);
            const uint64_t ibA = __shfl(inb, jA, SW);
            const uint64_t mfA = grp.dense ? 0 : __shfl(mfull, jA, SW);
            const int64_t bA = grp.dense ? 0 : __shfl(bj, jA, SW);
            int cA = __shfl(cvj, jA, SW);
            bool okA = act && vA < ub && ((ibA >> b) & 1ull);
            if (T > 1 && okA) cA = colr[(int64_t)lt * n + vA];
            okA = okA && cA != cu && cA != cw;
            if (!okA) continue;
            n_rows++;
            const uint64_t *rowA =
                a.val + ((grp.dense ? (int64_t)vA * B + b : bA + __popcll(mfA & ((1ull << b) - 1ull))) * T + lt) * Ca;
            const uint32_t *mA = s_map + ((cu * grp.k + cA) * grp.k + cw) * (emap_cp >> 2);
            for (int c0 = 0; c0 < Ca; c0 += EJ_UNROLL_S) {
              uint64_t xa[EJ_UNROLL_S];
#pragma unroll
              for (int q = 0; q < EJ_UNROLL_S; q++) xa[q] = c0 + q < Ca ? rowA[c0 + q] : 0;
#pragma unroll
              for (int q = 0; q < EJ_UNROLL_S; q++) {
                if (!xa[q]) continue;
                if (MAP) {
                  const uint32_t o = (mA[(c0 + q) >> 2] >> (8 * (q & 3))) & 0xffu;
                  if (o != 0xffu) add_ck(acc[o * NB + tid], xa[q], of);
                } else {
                  const uint32_t R = spread2(s_um[c0 + q], cu, cA);
                  if (!((R >> cw) & 1u)) add_ck(acc[s_rank[squeeze2(R | (1u << cA), cu, cw)] * NB + tid], xa[q], of);
                }
              }
            }
          }
        } else if (!ANN) {
          // two neighbours per step, both rows' loads in flight together
          while (todo) {
            const int jA = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int jB = todo ? __builtin_ctzll(todo) : jA;
            if (todo) todo &= todo - 1;
            const bool hasB = jB != jA;
            // every lane of the group takes part in the cross-lane reads
            const int vA = __shfl(vj, jA, SW), vB = __shfl(vj, jB, SW);
            const uint64_t ibA = __shfl(inb, jA, SW), ibB = __shfl(inb, jB, SW);
            const uint64_t mfA = grp.dense ? 0 : __shfl(mfull, jA, SW), mfB = grp.dense ? 0 : __shfl(mfull, jB, SW);
            const int64_t bA = grp.dense ? 0 : __shfl(bj, jA, SW), bB = grp.dense ? 0 : __shfl(bj, jB, SW);
            int cA = __shfl(cvj, jA, SW), cB = __shfl(cvj, jB, SW);
            bool okA = act && vA < ub && ((ibA >> b) & 1ull);
            bool okB = act && hasB && vB < ub && ((ibB >> b) & 1ull);
            if (T > 1) {
              if (okA) cA = colr[(int64_t)lt * n + vA];
              if (okB) cB = colr[(int64_t)lt * n + vB];
            }
            okA = okA && cA != cu && cA != cw;
            okB = okB && cB != cu && cB != cw;
            if (!okA && !okB) continue;
            n_rows += (uint32_t)okA + (uint32_t)okB;
            const uint64_t lowb = (1ull << b) - 1ull;
            const uint64_t *rowA =
                a.val + ((grp.dense ? (int64_t)vA * B + b : bA + __popcll(mfA & lowb)) * T + lt) * Ca;
            const uint64_t *rowB =
                a.val + ((grp.dense ? (int64_t)vB * B + b : bB + __popcll(mfB & lowb)) * T + lt) * Ca;
            const uint32_t *mA = s_map + ((cu * grp.k + cA) * grp.k + cw) * (emap_cp >> 2);
            const uint32_t *mB = s_map + ((cu * grp.k + cB) * grp.k + cw) * (emap_cp >> 2);
            for (int c0 = 0; c0 < Ca; c0 += EJ_UNROLL) {
              uint64_t xa[EJ_UNROLL], xb[EJ_UNROLL];
#pragma unroll
              for (int q = 0; q < EJ_UNROLL; q++) {
                xa[q] = okA && c0 + q < Ca ? rowA[c0 + q] : 0;
                xb[q] = okB && c0 + q < Ca ? rowB[c0 + q] : 0;
              }
              static_assert(EJ_UNROLL % 4 == 0, "map words hold four slots");
#pragma unroll
              for (int q = 0; q < EJ_UNROLL; q++) {
                if (MAP) {
                  const uint32_t oA = (mA[(c0 + q) >> 2] >> (8 * (q & 3))) & 0xffu;
                  const uint32_t oB = (mB[(c0 + q) >> 2] >> (8 * (q & 3))) & 0xffu;
                  if (xa[q] && oA != 0xffu) add_ck(acc[oA * NB + tid], xa[q], of);
                  if (xb[q] && oB != 0xffu) add_ck(acc[oB * NB + tid], xb[q], of);
                  continue;
                }
                if (xa[q]) {
                  const uint32_t R = spread2(s_um[c0 + q], cu, cA);
                  if (!((R >> cw) & 1u)) add_ck(acc[s_rank[squeeze2(R | (1u << cA), cu, cw)] * NB + tid], xa[q], of);
                }
                if (xb[q]) {
                  const uint32_t R = spread2(s_um[c0 + q], cu, cB);
                  if (!((R >> cw) & 1u)) add_ck(acc[s_rank[squeeze2(R | (1u << cB), cu, cw)] * NB + tid], xb[q], of);
                }
              }
            }
          }
        } else if (ANN && T == 1 && epi.ann_lanes) {
          // annotated, one trial: the output slots of a (neighbour, source)
          // pair spread over the lanes (lane = (pair of the round, slot); rows
          // wider than the group: one pair a round, SW slots a step), so a
          // neighbour that relaxes few sources still keeps the lanes busy.
          // Each (source, slot) column has one writer per round: plain adds.
          const int NY = C <= SW ? SW / C : 1;  // pairs per round
          const int py = C <= SW ? gl / C : 0, co0 = C <= SW ? gl - py * C : gl, cstep = C <= SW ? C : SW;
          const bool lane_on = py < NY;
          const int cwq = colr[w];  // w's colour (cw is set only on lanes that hold a source)
          while (todo) {
            const int jj = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int v = __shfl(vj, jj, SW);
            const uint64_t ib = __shfl(inb, jj, SW);
            const uint64_t mf = grp.dense ? 0 : __shfl(mfull, jj, SW);
            const int64_t vb = grp.dense ? 0 : __shfl(bj, jj, SW);
            const int cv = __shfl(cvj, jj, SW);
            // the group's lanes whose sources relax a row from v
            uint64_t M = gballot(act && v < ub && ((ib >> b) & 1ull) && cv != cu && cv != cw);
            if (!M) continue;
            const int64_t es = j0 + jj;
            const int64_t tslot = e_src_first ? g.rev[es] : es;
            const uint64_t *er = et.val + tslot * et.C;
            while (M) {
              const int nm = __popcll(M);
              const int lpos = lane_on && py < nm ? nth_set_bit(M, py) : -1;  // this lane's pair: its source's lane
              if (nm <= NY) M = 0;
              else M &= ~((2ull << nth_set_bit(M, NY - 1)) - 1ull);  // the bit is below 63: more follow it
              const int bq = __shfl(b, lpos < 0 ? 0 : lpos, SW), cuq = __shfl(cu, lpos < 0 ? 0 : lpos, SW);
              if (lpos < 0) continue;
              const int64_t id = grp.dense ? (int64_t)v * B + bq : vb + __popcll(mf & ((1ull << bq) - 1ull));
              if (co0 == 0) n_rows++;
              const uint64_t *row = a.val + id * Ca;
              for (int co = co0; co < C; co += cstep) {
                const uint32_t Rp = spread2(s_um[co], cuq, cwq);
                if (!((Rp >> cv) & 1u)) continue;
                const uint32_t R = Rp & ~(1u << cv);
                const int nR = __popc(R);
                if (ra > nR) continue;
                uint64_t sum = 0;
                // the subsets of R of size ra (the input row's colours)
                for (uint32_t cm = (1u << ra) - 1u; cm < (1u << nR); cm = ra ? next_comb(cm) : (1u << nR)) {
                  const uint32_t s1 = deposit(cm, R);
                  const uint64_t xa = row[s_rank[squeeze2(s1, cuq, cv)]];
                  if (xa) {
                    const uint64_t y = er[s_rank[squeeze2(R & ~s1, cv, cwq)]];
                    if (y) add_ck(sum, mul_ck(xa, y, of), of);
                  }
                }
                if (sum) add_ck(acc[co * NB + (tid - gl) + lpos], sum, of);
              }
            }
          }
        } else {
          while (todo) {
            const int jj = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int v = __shfl(vj, jj, SW);
            const uint64_t ib = __shfl(inb, jj, SW);
            const uint64_t mf = grp.dense ? 0 : __shfl(mfull, jj, SW);
            const int64_t vb = grp.dense ? 0 : __shfl(bj, jj, SW);
            const int cvs = __shfl(cvj, jj, SW);
            if (!act || v >= ub || !((ib >> b) & 1ull)) continue;
            const int cv = T == 1 ? cvs : colr[(int64_t)lt * n + v];
            if (cv == cu || cv == cw) continue;
            const int64_t id = grp.dense ? (int64_t)v * B + b : vb + __popcll(mf & ((1ull << b) - 1ull));
            n_rows++;
            const uint64_t *row = a.val + (id * T + lt) * Ca;
            const int64_t es = j0 + jj;
            const int64_t tslot = e_src_first ? g.rev[es] : es;
            const uint64_t *er = et.val + (tslot * T + lt) * et.C;
            for (int co = 0; co < C; co++) {
              const uint32_t Rp = spread2(s_um[co], cu, cw);
              if (!((Rp >> cv) & 1u)) continue;
              const uint32_t R = Rp & ~(1u << cv);
              const int nR = __popc(R);
              if (ra > nR) continue;
              uint64_t sum = 0;
              // the subsets of R of size ra (the input row's colours)
              for (uint32_t cm = (1u << ra) - 1u; cm < (1u << nR); cm = ra ? next_comb(cm) : (1u << nR)) {
                const uint32_t s1 = deposit(cm, R);
                const uint64_t xa = row[s_rank[squeeze2(s1, cu, cv)]];
                if (xa) {
                  const uint64_t y = er[s_rank[squeeze2(R & ~s1, cv, cw)]];
                  if (y) add_ck(sum, mul_ck(xa, y, of), of);
                }
              }
              if (sum) add_ck(acc[co * NB + tid], sum, of);
            }
          }
        }
        if (stop) break;
      }
      // other lanes' adds into this lane's columns are done
      if (PACK || (ANN && T == 1 && epi.ann_lanes)) __threadfence_block();
      // epilogue: row-local ops on the rows of w, operands in LDS or read
      // from global memory at their own level
      if (EPI && b >= 0 && epi.nops) {
        for (int j = 0; j < epi.nregs; j++) {
          const EpiReg &R = epi.regs[j];
          int64_t id = -1;
          if (R.col < 0) {
            if (grp.dense) id = ((R.r.mask[w] >> b) & 1ull) ? (int64_t)w * B + b : -1;
            else id = sparse_entry(R.L, w, b);
          }
          s_rid[j * NB + tid] = id;
        }
        auto val = [&](int j, int slot) -> uint64_t {
          const EpiReg &R = epi.regs[j];
          if (R.col >= 0) return accs[(R.col + slot) * NB + tid];
          const int64_t id = s_rid[j * NB + tid];
          return id < 0 ? 0 : R.r.val[(id * T + lt) * R.r.C + slot];
        };
        for (int oi = 0; oi < epi.nops; oi++) {
          const EpiOp &op = epi.ops[oi];
          if (op.kind == EPI_NJ) {
            // dst[R'] = sum over splits R' = R + Ra of a[R] * A[w][Ra]  (NodeJoin at w)
            const EpiReg &D = epi.regs[op.dst];
            const int rA = op.nt.s - 1;
            for (int c = 0; c < D.r.C; c++) {
              uint64_t v = 0;
              if (cu != cw) {
                const uint32_t Rp = spread2(unr(D.r.s - 2, c), cu, cw);
                const uint64_t *nr = op.nt.val + ((int64_t)w * T + lt) * op.nt.C;
                uint32_t sA = Rp;
                for (;;) {
                  if (__popc(sA) == rA) {
                    const uint64_t y = nr[s_rank[squeeze1(sA, cw)]];
                    if (y) {
                      const uint64_t x = val(op.a, s_rank[squeeze2(Rp & ~sA, cu, cw)]);
                      if (x) add_ck(v, mul_ck(x, y, of), of);
                    }
                  }
                  if (sA == 0) break;
                  sA = (sA - 1) & Rp;
                }
              }
              accs[(D.col + c) * NB + tid] = v;
            }
          } else if (op.kind == EPI_AXPY) {
            const EpiReg &D = epi.regs[op.dst];
            for (int c = 0; c < D.r.C; c++) {
              uint64_t y = op.first ? 0 : accs[(D.col + c) * NB + tid];
              const uint64_t x = val(op.a, c);
              if (x) add_ck(y, mul_ck(op.w, x, of), of);
              accs[(D.col + c) * NB + tid] = y;
            }
          } else if (cu != cw) {  // EPI_MROOT: the cycle closes at w
            const EpiReg &A = epi.regs[op.a];
            for (int c = 0; c < A.r.C; c++) {
              const uint64_t x = val(op.a, c);
              if (!x) continue;
              const uint32_t R1 = spread2(unr(A.r.s - 2, c), cu, cw);
              const uint32_t R2 = Kmask & ~R1 & ~(1u << cu) & ~(1u << cw);
              const uint64_t y = val(op.b, s_rank[squeeze2(R2, cu, cw)]);
              if (!y) continue;
              uint64_t pl, ph;
    mul_wide(x, y, pl, ph);
              if (op.w != 1) {
                const uint64_t l2 = pl * op.w, c2 = __umul64hi(pl, op.w);
                const uint64_t h2 = ph * op.w + c2;
                if (__umul64hi(ph, op.w) != 0 || h2 < c2) of = true;
                pl = l2;
                ph = h2;
              }
              if (accd.per_src) atomic_add128(&accd.per_src[2 * ((int64_t)u * T + lt)], pl, ph);
              const uint64_t sl = mlo + pl;
              mhi += ph + (sl < pl ? 1u : 0u);
              mlo = sl;
            }
          }
        }
      }
      if (of) ofm |= 1ull << lt;
      // write the registers that leave the vertex, the lane's row (w, b) for
      // trial lt: sparse -- every marked row; dense -- the rows nonzero in some
      // trial (the others stay dead)
      for (int j = 0; j < epi.nregs; j++) {
        const EpiReg &R = epi.regs[j];
        if (!R.write) continue;
        const int Cj = R.r.C;
        uint64_t mine = 0;
        if (grp.dense && b >= 0) {
          bool nz = false;
          for (int o = 0; o < Cj; o++) nz |= accs[(R.col + o) * NB + tid] != 0;
          mine = nz ? 1ull << b : 0;
        }
        if (grp.dense)
          for (int o = SW / 2; o > 0; o >>= 1) mine |= (uint64_t)__shfl_xor(mine, o, SW);
        if (grp.dense && gl == 0) s_live[j * (NB / SW) + tid / SW] |= mine;
        const bool wr = b >= 0 && (!grp.dense || ((mine >> b) & 1ull));
        if (wr) {
          const int64_t id = grp.dense ? (int64_t)w * B + b : sparse_entry(R.L, w, b);
          uint64_t *drow = R.r.val + (id * T + lt) * Cj;
          if (split) {  // a chunk of a hub: add the partial row (checked through the old value)
            for (int o = 0; o < Cj; o++) {
              const uint64_t x = accs[(R.col + o) * NB + tid];
              if (!x) continue;
              const uint64_t old = atomicAdd((unsigned long long *)&drow[o], (unsigned long long)x);
              if (old + x < old) ofm |= 1ull << lt;
            }
          } else {
            for (int o = 0; o < Cj; o++) drow[o] = accs[(R.col + o) * NB + tid];
          }
        }
        // rows (w, b) written, all their trials (a hub's rows once, by its first chunk)
        if (b >= 0 && lt == 0 && (split ? first_chunk : wr)) n_ent += DUAL ? (uint32_t)Cj : 1u;
      }
    }
    if (gl == 0 && grp.dense)
      for (int j = 0; j < epi.nregs; j++) {
        if (!epi.regs[j].write) continue;
        const uint64_t lv = s_live[j * (NB / SW) + tid / SW];
        if (!split) epi.regs[j].r.mask[w] = lv;
        else if (lv) atomicOr((unsigned long long *)&epi.regs[j].r.mask[w], (unsigned long long)lv);
      }
  }
  flag_trials(ovf, ofm);
  if (EPI) {
    if (mlo | mhi) atomic_add128(&s_msum[2 * lt], mlo, mhi);
    __syncthreads();
    if (tid < T && (s_msum[2 * tid] | s_msum[2 * tid + 1]))
      atomic_add128(&accd.sum[2 * tid], s_msum[2 * tid], s_msum[2 * tid + 1]);
  }
  if (grp.prof) {
    uint64_t c0 = n_scan, c1 = n_rows, c2 = n_ent;
    for (int o = 32; o > 0; o >>= 1) {
      c0 += __shfl_xor(c0, o);
      c1 += __shfl_xor(c1, o);
      c2 += __shfl_xor(c2, o);
    }
    if (lane == 0) {
      uint64_t *pc = grp.prof + 3 * ((blockIdx.x * WPB + tid / WAVE) % PROF_LANES);  // spread over lanes: no hot address
      atomicAdd((unsigned long long *)&pc[0], (unsigned long long)c0);
      atomicAdd((unsigned long long *)&pc[1], (unsigned long long)c1);
      atomicAdd((unsigned long long *)&pc[2], (unsigned long long)c2);
    }
  }
}

// The group's source ranks and their colours per trial in LDS, for kernels
// that need them per slot: one LDS read instead of two dependent global loads.
__device__ __forceinline__ void load_sources(const GroupDev &grp, const uint8_t *colr, int64_t n, int32_t *s_u,
                                             uint8_t *s_cu) {
  for (int i = threadIdx.x; i < WAVE; i += blockDim.x) s_u[i] = i < grp.B ? grp.src[i] : 0;
  for (int i = threadIdx.x; i < grp.T * WAVE; i += blockDim.x) {
    const int t = i / WAVE, b = i - t * WAVE;
    s_cu[i] = b < grp.B ? colr[(int64_t)t * n + grp.src[b]] : 0;
  }
}

// ------------------------------------------------------------------ NodeJoin
// dst[(v,b)][R'] = sum over splits R' = R + Ra of a[(v,b)][R] * A[v][Ra]
__global__ __launch_bounds__(BLK) void k_nj(GroupDev grp, int64_t n, const uint8_t *colr, LevelDev L, RegDev a,
                                            RegDev dst, TabDev nt, uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int T = grp.T, C = dst.C, Ca = a.C;
  const int rA = nt.s - 1;
  const int64_t per = (int64_t)T * C;
  const int64_t N = nentries(grp, L) * per;
  uint64_t ofm = 0, prd = 0, pwr = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t e = i / per;
    const int r = (int)(i - e * per), t = r / C, c = r - t * C;
    int64_t v;
    int b;
    entry_vb(grp, L, e, v, b);
    if (!live(grp, a, v, b)) continue;
    pwr += 8;
    const int64_t u = grp.src[b];
    uint64_t acc = 0;
    bool of = false;
    if (v < vbound(grp, u)) {
      const int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
      if (cu != cv) {
        if (c == 0) prd += 8 * (uint64_t)(Ca + nt.C);
        const uint32_t Rp = spread2(unrank(lut, dst.s - 2, c), cu, cv);
        const uint64_t *ar = a.val + (e * T + t) * Ca;
        const uint64_t *nr = nt.val + (v * T + t) * nt.C;
        uint32_t sA = Rp;
        for (;;) {
          if (__popc(sA) == rA) {
            uint64_t y = nr[s_rank[squeeze1(sA, cv)]];
            if (y) {
              uint64_t x = ar[s_rank[squeeze2(Rp & ~sA, cu, cv)]];
              if (x) add_ck(acc, mul_ck(x, y, of), of);
            }
          }
          if (sA == 0) break;
          sA = (sA - 1) & Rp;
        }
      }
    }
    dst.val[i] = acc;
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

// ------------------------------------------------------------------ AXPY
// dst = (first ? 0 : dst) + w * a, slot by slot (same level, same rows)
__global__ __launch_bounds__(BLK) void k_axpy(GroupDev grp, LevelDev L, RegDev a, RegDev dst, uint64_t w, int first,
                                              uint32_t *ovf) {
  const int T = grp.T, C = dst.C;
  const int64_t N = nentries(grp, L) * T * C;
  uint64_t ofm = 0, prd = 0, pwr = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    bool of = false;
    bool on = true, dlive = true;
    if (grp.dense) {
      // dense registers are pooled: a row whose activity bit is clear holds
      // whatever an earlier group left there and counts as zero
      const int64_t row = i / ((int64_t)T * C);
      on = (a.mask[row / grp.B] >> (row % grp.B)) & 1ull;
      dlive = !first && ((dst.mask[row / grp.B] >> (row % grp.B)) & 1ull);
      if (!on && !first) continue;
    }
    uint64_t y = (first || !dlive) ? 0 : dst.val[i];
    if (on) add_ck(y, mul_ck(w, a.val[i], of), of);
    dst.val[i] = y;
    if (of) ofm |= 1ull << ((i / C) % T);
    prd += 8 * ((on ? 1 : 0) + (!first && dlive ? 1 : 0));
    pwr += 8;
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

// dst = sum of w_i * a_i over up to four terms (an AXPY chain in one pass)
// A term is a register, or the NodeJoin of a register with a node table
// (then the NodeJoin's output is never stored: its slot is computed here).
struct AxpyTerms {
  RegDev a[4];
  uint64_t w[4];
  TabDev nt[4];          // nt[q].val: term q is NodeJoin(a[q], nt[q])
  const uint32_t *jm[4];  // NodeJoin split map of term q (or null), jmw[q] words, jns[q] splits per slot
  int jmw[4], jns[4];
  int n;
};

// NodeJoin splits from a map.  For output slot c (colour set S of dst, cu and
// cv squeezed out) the splits are the subsets S_j of S of nt's size; the map
// word of split j holds the slot of S_j in nt's row in its low 16 bits (only
// the position of cu among the k - 1 colours other than cv matters: cu' = cu -
// [cv < cu]) and the slot of S minus S_j in a in its high 16 bits (it does not
// depend on the colours).  Words of (cu', c) start at (cu' * C + c) * ns.
__device__ __forceinline__ const uint32_t *split_words(const uint32_t *jm, int cup, int C, int c, int ns) {
  return jm + (cup * C + c) * ns;
}
__device__ __forceinline__ uint64_t nj_slot_map(const uint64_t *ar, const uint64_t *nr, const uint32_t *sp, int ns,
                                                bool &of) {
  uint64_t acc = 0;
  for (int j = 0; j < ns; j++) {
    const uint32_t w = sp[j];
    const uint64_t y = nr[w & 0xffffu];
    if (!y) continue;
    const uint64_t x = ar[w >> 16];
    if (x) add_ck(acc, mul_ck(x, y, of), of);
  }
  return acc;
}
// LDS copies of the split maps of the terms, one after another
__device__ __forceinline__ void load_jmaps(const AxpyTerms &tm, uint32_t *s_jm) {
  int off = 0;
  for (int q = 0; q < tm.n; q++) {
    for (int i = threadIdx.x; i < tm.jmw[q]; i += blockDim.x) s_jm[off + i] = tm.jm[q][i];
    off += tm.jmw[q];
  }
}
__device__ __forceinline__ const uint32_t *jmap_at(const AxpyTerms &tm, const uint32_t *s_jm, int q) {
  int off = 0;
  for (int p = 0; p < q; p++) off += tm.jmw[p];
  return s_jm + off;
}

// slot c (of dst's signature size s) of NodeJoin(a, nt) at row (v, b), trial t
__device__ __forceinline__ uint64_t nj_slot(const RegDev &a, const TabDev &nt, int64_t row, int64_t v, int t, int T,
                                            int cu, int cv, uint32_t Rp_unranked, const uint16_t *s_rank, bool &of) {
  const uint32_t Rp = spread2(Rp_unranked, cu, cv);
  const uint64_t *ar = a.val + (row * T + t) * a.C;
  const uint64_t *nr = nt.val + (v * T + t) * nt.C;
  const int rA = nt.s - 1;
  uint64_t acc = 0;
  uint32_t sA = Rp;
  for (;;) {
    if (__popc(sA) == rA) {
      const uint64_t y = nr[s_rank[squeeze1(sA, cv)]];
      if (y) {
        const uint64_t x = ar[s_rank[squeeze2(Rp & ~sA, cu, cv)]];
        if (x) add_ck(acc, mul_ck(x, y, of), of);
      }
    }
    if (sA == 0) break;
    sA = (sA - 1) & Rp;
  }
  return acc;
}

__global__ __launch_bounds__(BLK) void k_axpyn(GroupDev grp, int64_t n, const uint8_t *colr, LevelDev L, AxpyTerms tm,
                                               RegDev dst, uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint32_t s_uo[256];  // unranked slots of dst
  extern __shared__ uint32_t s_jm[];
  __shared__ int32_t s_u[WAVE];
  __shared__ uint8_t s_cu[WAVE * WAVE];
  load_sources(grp, colr, n, s_u, s_cu);
  load_jmaps(tm, s_jm);
  load_rank(s_rank, lut);
  const int T = grp.T, C = dst.C;
  for (int c = threadIdx.x; c < C; c += BLK) s_uo[c] = unrank(lut, dst.s - 2, c);
  __syncthreads();
  const int64_t per = (int64_t)T * C;
  const int64_t N = nentries(grp, L) * per;
  uint64_t ofm = 0, prd = 0, pwr = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    bool of = false;
    uint64_t y = 0;
    const int64_t row = i / per;
    const int r = (int)(i - row * per), t = r / C, c = r - t * C;
    pwr += 8;
    for (int q = 0; q < tm.n; q++) {
      if (grp.dense && !((tm.a[q].mask[row / grp.B] >> (row % grp.B)) & 1ull)) continue;
      uint64_t x;
      if (tm.nt[q].val) {
        int64_t v;
        int b;
        entry_vb(grp, L, row, v, b);
        const int64_t u = s_u[b];
        const int cu = s_cu[t * WAVE + b], cv = colr[(int64_t)t * n + v];
        x = 0;
        if (v < vbound(grp, u) && cu != cv) {
          if (c == 0) prd += 8 * (uint64_t)(tm.a[q].C + tm.nt[q].C);
          if (tm.jmw[q]) {
            const int ns = tm.jns[q];
            const uint32_t *sp = split_words(jmap_at(tm, s_jm, q), cu - (cv < cu), C, c, ns);
            x = nj_slot_map(tm.a[q].val + (row * T + t) * tm.a[q].C, tm.nt[q].val + (v * T + t) * tm.nt[q].C, sp,
                            ns, of);
          } else {
            x = nj_slot(tm.a[q], tm.nt[q], row, v, t, T, cu, cv, s_uo[c], s_rank, of);
          }
        }
      } else {
        x = tm.a[q].val[i];
        prd += 8;
      }
      if (x) add_ck(y, mul_ck(tm.w[q], x, of), of);
    }
    dst.val[i] = y;
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}
__global__ void k_mask_orn(AxpyTerms tm, uint64_t *dm, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t m = 0;
    for (int q = 0; q < tm.n; q++) m |= tm.a[q].mask[i];
    dm[i] = m;
  }
}

// dst.mask = (first ? 0 : dst.mask) | a.mask
__global__ void k_mask_or(const uint64_t *am, uint64_t *dm, int64_t n, int first) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dm[i] = first ? am[i] : (dm[i] | am[i]);
}
__global__ void k_fill_v(uint64_t *p, int64_t n, uint64_t x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = x;
}

// ------------------------------------------------------------------ dense groups: live rows only
// A wavefront per vertex v walks the live rows (set bits of v's activity
// word) times their slots; a vertex with no live row costs one load.
__device__ __forceinline__ int nth_bit(uint64_t m, int k) {  // k < popcount(m)
  int pos = 0;
  for (int sh = 32; sh; sh >>= 1) {
    const uint64_t lo = m & ((1ull << sh) - 1ull);
    const int c = __popcll(lo);
    if (k >= c) {
      k -= c;
      m >>= sh;
      pos += sh;
    } else {
      m = lo;
    }
  }
  return pos;
}

__global__ __launch_bounds__(BLK) void k_nj_dense(GroupDev grp, int64_t n, const uint8_t *colr, RegDev a, RegDev dst,
                                                  TabDev nt, uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint32_t s_uo[256];
  load_rank(s_rank, lut);
  const int T = grp.T, C = dst.C, Ca = a.C, B = grp.B;
  for (int c = threadIdx.x; c < C; c += BLK) s_uo[c] = unrank(lut, dst.s - 2, c);
  __syncthreads();
  const int rA = nt.s - 1;
  const int per = T * C;
  const int lane = threadIdx.x % 64;
  const int64_t wave = (int64_t)blockIdx.x * (BLK / 64) + threadIdx.x / 64, nwave = (int64_t)gridDim.x * (BLK / 64);
  uint64_t ofm = 0, prd = 0, pwr = 0;
  const uint64_t bmask = B >= 64 ? ~0ull : (1ull << B) - 1ull;  // the group's sources
  for (int64_t v = wave; v < grp.n_lim; v += nwave) {
    const uint64_t m = a.mask[v] & bmask;
    prd += lane == 0 ? 8 : 0;
    if (!m) continue;
    const int items = __popcll(m) * per;
    for (int it = lane; it < items; it += 64) {
      const int q = it / per, r = it - q * per, t = r / C, c = r - t * C;
      const int b = nth_bit(m, q);
      const int64_t e = v * B + b;
      const int64_t u = grp.src[b];
      uint64_t acc = 0;
      bool of = false;
      if (v < vbound(grp, u)) {
        const int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
        if (cu != cv) {
          if (c == 0) prd += 8 * (uint64_t)(Ca + nt.C);
          const uint32_t Rp = spread2(s_uo[c], cu, cv);
          const uint64_t *ar = a.val + (e * T + t) * Ca;
          const uint64_t *nr = nt.val + (v * T + t) * nt.C;
          uint32_t sA = Rp;
          for (;;) {
            if (__popc(sA) == rA) {
              const uint64_t y = nr[s_rank[squeeze1(sA, cv)]];
              if (y) {
                const uint64_t x = ar[s_rank[squeeze2(Rp & ~sA, cu, cv)]];
                if (x) add_ck(acc, mul_ck(x, y, of), of);
              }
            }
            if (sA == 0) break;
            sA = (sA - 1) & Rp;
          }
        }
      }
      dst.val[e * per + r] = acc;
      if (of) ofm |= 1ull << t;
      pwr += 8;
    }
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

// JM: every NodeJoin term has a split map (the subset walk is not compiled in)
template <bool JM>
__global__ __launch_bounds__(BLK) void k_axpyn_dense(GroupDev grp, int64_t n, const uint8_t *colr, AxpyTerms tm,
                                                     RegDev dst, uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint32_t s_uo[256];  // unranked slots of dst
  extern __shared__ uint32_t s_jm[];
  __shared__ int32_t s_u[WAVE];
  __shared__ uint8_t s_cu[WAVE * WAVE];
  load_sources(grp, colr, n, s_u, s_cu);
  load_jmaps(tm, s_jm);
  load_rank(s_rank, lut);
  const int T = grp.T, C = dst.C, B = grp.B;
  for (int c = threadIdx.x; c < C; c += BLK) s_uo[c] = unrank(lut, dst.s - 2, c);
  __syncthreads();
  const int per = T * C;
  const int lane = threadIdx.x % 64;
  const int64_t wave = (int64_t)blockIdx.x * (BLK / 64) + threadIdx.x / 64, nwave = (int64_t)gridDim.x * (BLK / 64);
  uint64_t ofm = 0, prd = 0, pwr = 0;
  const uint64_t bmask = B >= 64 ? ~0ull : (1ull << B) - 1ull;  // the group's sources
  for (int64_t v = wave; v < grp.n_lim; v += nwave) {
    uint64_t mt[4] = {0, 0, 0, 0};
    if (lane == 0) {
      prd += 8 * (uint64_t)tm.n;
      pwr += 8;
    }
    uint64_t m = 0;
#pragma unroll
    for (int q = 0; q < 4; q++)
      if (q < tm.n) {
        mt[q] = tm.a[q].mask[v] & bmask;
        m |= mt[q];
      }
    if (lane == 0) dst.mask[v] = m;
    if (!m) continue;
    const int cv1 = T == 1 ? colr[v] : 0;  // one trial: v's colour, loaded once for all its items
    const int items = __popcll(m) * per;
    for (int it = lane; it < items; it += 64) {
      const int q0 = it / per, r = it - q0 * per, t = r / C, c = r - t * C;
      const int b = nth_bit(m, q0);
      const int64_t row = v * B + b;
      const int64_t i = row * per + r;
      bool of = false;
      uint64_t y = 0;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        if (q >= tm.n || !((mt[q] >> b) & 1ull)) continue;
        uint64_t x;
        if (tm.nt[q].val) {
          const int64_t u = s_u[b];
          const int cu = s_cu[t * WAVE + b], cv = T == 1 ? cv1 : colr[(int64_t)t * n + v];
          x = 0;
          if (v < vbound(grp, u) && cu != cv) {
            if (c == 0) prd += 8 * (uint64_t)(tm.a[q].C + tm.nt[q].C);
            if (JM || tm.jmw[q]) {
              const int ns = tm.jns[q];
              const uint32_t *sp = split_words(jmap_at(tm, s_jm, q), cu - (cv < cu), C, c, ns);
              x = nj_slot_map(tm.a[q].val + (row * T + t) * tm.a[q].C, tm.nt[q].val + (v * T + t) * tm.nt[q].C, sp,
                              ns, of);
            } else {
              x = nj_slot(tm.a[q], tm.nt[q], row, v, t, T, cu, cv, s_uo[c], s_rank, of);
            }
          }
        } else {
          x = tm.a[q].val[i];
          prd += 8;
        }
        if (x) add_ck(y, mul_ck(tm.w[q], x, of), of);
      }
      dst.val[i] = y;
      if (of) ofm |= 1ull << (r / C);
      pwr += 8;
    }
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

// One colouring: the AXPY chain by chunks of rows, like the root merge below
// (a wavefront takes R = 64 / C rows, lane = (row of the chunk, slot); the
// plain terms' slots are loaded by their lanes, the NodeJoin terms' input rows
// and node-table rows are staged in the wavefront's LDS; every load of a chunk
// is issued before any is used).  Dense groups write the activity word of
// dst and its live rows; sparse groups every entry.  NT: the number of terms.
template <bool DENSE, int NT>
__global__ __launch_bounds__(BLK) void k_axpyn_rows(GroupDev grp, int64_t n, const uint8_t *colr, LevelDev L,
                                                    AxpyTerms tm, RegDev dst, uint32_t *ovf, int jm_words,
                                                    int stage_words) {
  __shared__ int32_t s_u[WAVE];
  __shared__ uint8_t s_cu[WAVE];
  extern __shared__ uint64_t s_dyn[];  // split maps, then the stages
  uint32_t *s_jm = (uint32_t *)s_dyn;
  for (int i = threadIdx.x; i < WAVE; i += blockDim.x) {
    s_u[i] = i < grp.B ? grp.src[i] : 0;
    s_cu[i] = i < grp.B ? colr[grp.src[i]] : 0;
  }
  load_jmaps(tm, s_jm);
  __syncthreads();
  const int B = grp.B, C = dst.C;
  const int lane = threadIdx.x % 64;
  uint64_t *stg = s_dyn + (jm_words + 1) / 2 + (size_t)(threadIdx.x / 64) * stage_words;
  const int R = 64 / C;
  const int jr = lane / C, c = lane - jr * C;  // this lane's row of the chunk and slot
  int off_a[NT], off_n[NT];
  {
    int off = 0;
#pragma unroll
    for (int q = 0; q < NT; q++) {
      off_a[q] = off_n[q] = 0;
      if (!tm.nt[q].val) continue;
      off_a[q] = off;
      off += R * tm.a[q].C;
      off_n[q] = off;
      off += (DENSE ? 1 : R) * tm.nt[q].C;
    }
  }
  // the lane's first staged node-table element (sparse groups stage one row per
  // entry): its entry of the chunk and slot
  int nr0[NT], nc0[NT];
#pragma unroll
  for (int q = 0; q < NT; q++) {
    const int Cn = tm.nt[q].val ? tm.nt[q].C : 1;
    nr0[q] = min(lane / Cn, R - 1);
    nc0[q] = lane - (lane / Cn) * Cn;
  }
  const uint64_t bmask = B >= 64 ? ~0ull : (1ull << B) - 1ull;
  uint64_t prd = 0, pwr = 0;
  bool of = false;
  // the lane's slot of the chain once its loads have landed
  auto slot = [&](int b, int64_t v, uint32_t on, const uint64_t *xp, int cv) -> uint64_t {
    const int cu = s_cu[b];
    const bool njok = v < vbound(grp, s_u[b]) && cu != cv;
    const int cup = cu - (cv < cu);
    uint64_t y = 0;
#pragma unroll
    for (int q = 0; q < NT; q++) {
      if (!((on >> q) & 1u)) continue;
      uint64_t xq = 0;
      if (tm.nt[q].val) {
        if (!njok) continue;
        if (c == 0) prd += 8 * (uint64_t)(tm.a[q].C + tm.nt[q].C);
        const int ns = tm.jns[q];
        const uint32_t *jm = jmap_at(tm, s_jm, q);
        const uint32_t *sp = split_words(jm, cup, C, c, ns);
        const uint64_t *ar = stg + off_a[q] + jr * tm.a[q].C;
        const uint64_t *nr = stg + off_n[q] + (DENSE ? 0 : jr * tm.nt[q].C);
        for (int j = 0; j < ns; j++) {
          const uint32_t w = sp[j];
          const uint64_t z = nr[w & 0xffffu];
          if (!z) continue;
          const uint64_t xa = ar[w >> 16];
          if (xa) add_ck(xq, mul_ck(xa, z, of), of);
        }
      } else {
        xq = xp[q];
        prd += 8;
      }
      if (xq) add_ck(y, tm.w[q] == 1 ? xq : mul_ck(tm.w[q], xq, of), of);
    }
    return y;
  };
  const int64_t wave = (int64_t)blockIdx.x * (BLK / 64) + threadIdx.x / 64, nwave = (int64_t)gridDim.x * (BLK / 64);
  if (DENSE) {
    for (int64_t v = wave; v < grp.n_lim; v += nwave) {
      uint64_t mt[NT], m = 0;
#pragma unroll
      for (int q = 0; q < NT; q++) {
        mt[q] = tm.a[q].mask[v] & bmask;
        m |= mt[q];
      }
      if (lane == 0) {
        dst.mask[v] = m;
        prd += 8 * (uint64_t)NT;
        pwr += 8;
      }
      if (!m) continue;
      const int cv = colr[v];
      const int nrows = __popcll(m);
      for (int j0 = 0; j0 < nrows; j0 += R) {
        const bool act = jr < R && j0 + jr < nrows;
        const int b = act ? nth_bit(m, j0 + jr) : 0;
        const int64_t row = v * B + b;
        uint32_t on = 0;
        uint64_t xp[NT];
#pragma unroll
        for (int q = 0; q < NT; q++) {
          xp[q] = 0;
          const bool hq = act && ((mt[q] >> b) & 1ull);
          on |= (uint32_t)hq << q;
          if (hq && !tm.nt[q].val) xp[q] = tm.a[q].val[row * C + c];
        }
        if (j0 == 0) {
#pragma unroll
          for (int q = 0; q < NT; q++)
            if (tm.nt[q].val)
              for (int i = lane; i < tm.nt[q].C; i += 64) stg[off_n[q] + i] = tm.nt[q].val[v * tm.nt[q].C + i];
        }
#pragma unroll
        for (int q = 0; q < NT; q++) {
          if (!tm.nt[q].val) continue;
          const int Cq = tm.a[q].C;
          // row r's source comes from the lane that owns row r (lane r * C)
          for (int i0 = 0; i0 < R * Cq; i0 += 64) {
            const int i = i0 + lane;
            const int r = min(i / Cq, R - 1);
            const int br = __shfl(b, r * C);
            if (i < R * Cq && j0 + r < nrows && ((mt[q] >> br) & 1ull))
              stg[off_a[q] + i] = tm.a[q].val[(v * B + br) * Cq + (i - r * Cq)];
          }
        }
        wave_lds_sync();
        if (act) {
          dst.val[row * C + c] = slot(b, v, on, xp, cv);
          pwr += 8;
        }
        wave_lds_sync();  // the stage is read before the next chunk overwrites it
      }
    }
  } else {
    const int64_t N = *L.cnt, nch = (N + R - 1) / R;
    for (int64_t ch = wave; ch < nch; ch += nwave) {
      const int64_t e0 = ch * R;
      const int lim = N - e0 < R ? (int)(N - e0) : R;  // entries of this chunk
      const int64_t e = e0 + jr;
      const bool act = jr < lim;
      int64_t v = 0;
      int b = 0, cv = 0;
      uint64_t xp[NT];
#pragma unroll
      for (int q = 0; q < NT; q++) xp[q] = 0;
      if (act) {
        const int64_t x = L.list[e];
        v = x >> 6;
        b = (int)(x & 63);
        cv = colr[v];
#pragma unroll
        for (int q = 0; q < NT; q++)
          if (!tm.nt[q].val) xp[q] = tm.a[q].val[e * C + c];
      }
#pragma unroll
      for (int q = 0; q < NT; q++) {
        if (!tm.nt[q].val) continue;
        const int Cq = tm.a[q].C, Cn = tm.nt[q].C;
        for (int i = lane; i < lim * Cq; i += 64) stg[off_a[q] + i] = tm.a[q].val[e0 * Cq + i];
        // row r's vertex comes from the lane that owns entry r (lane r * C)
        for (int i0 = 0; i0 < lim * Cn; i0 += 64) {
          const int i = i0 + lane;
          const int r = i0 ? min(i / Cn, R - 1) : nr0[q], cc = i0 ? i - (i / Cn) * Cn : nc0[q];
          const int vr = __shfl((int)v, r * C);
          if (i < lim * Cn) stg[off_n[q] + i] = tm.nt[q].val[(int64_t)vr * Cn + cc];
        }
      }
      wave_lds_sync();
      if (act) {
        dst.val[e * C + c] = slot(b, v, (1u << NT) - 1u, xp, cv);
        pwr += 8;
      }
      wave_lds_sync();
    }
  }
  flag_trials(ovf, of ? 1ull : 0ull);
  prof_flush(grp.prof, prd, pwr, 0);
}

template <bool DENSE>
void launch_axpyn_rows_nt(int nt, dim3 gr, size_t lds, hipStream_t st, const GroupDev &grp, int64_t n,
                          const uint8_t *colr, LevelDev L, const AxpyTerms &tm, RegDev dst, uint32_t *ovf,
                          int jm_words, int words) {
#define CC_AR(NTV)                                                                                                   \
  hipLaunchKernelGGL((k_axpyn_rows<DENSE, NTV>), gr, dim3(BLK), lds, st, grp, n, colr, L, tm, dst, ovf, jm_words, \
                     words)
  switch (nt) {
    case 1: CC_AR(1); break;
    case 2: CC_AR(2); break;
    case 3: CC_AR(3); break;
    default: CC_AR(4); break;
  }
#undef CC_AR
}

// ------------------------------------------------------------------ root merge
// count[t] += w * sum over entries (v, b) of both levels of
//             sum over R of a[(v,b)][R] * b[(v,b)][K \ {chi u, chi v} \ R]
__global__ __launch_bounds__(BLK) void k_mroot(GroupDev grp, int64_t n, const uint8_t *colr, LevelDev La,
                                               LevelDev Lb, RegDev a, RegDev bb, uint64_t w, AccDev acc,
                                               const uint16_t *lut) {
  // The partner slot of a's slot c does not depend on the colours: with cu
  // and cv squeezed out, K minus {cu, cv} minus R is the complement of c's
  // colour set in k - 2 bits.
  __shared__ uint16_t s_yi[256];  // b's slot partnering a's slot c
  __shared__ uint64_t s_acc[2 * 64];
  __shared__ int32_t s_u[WAVE];
  __shared__ uint8_t s_cu[WAVE * WAVE];
  load_sources(grp, colr, n, s_u, s_cu);
  for (int i = threadIdx.x; i < 2 * 64; i += blockDim.x) s_acc[i] = 0;
  const int T = grp.T, Ca = a.C, Cb = bb.C, k = grp.k;
  const uint32_t Kp = (1u << (k - 2)) - 1u;
  for (int c = threadIdx.x; c < Ca; c += BLK) s_yi[c] = lut[LUT_RANK + (Kp & ~unrank(lut, a.s - 2, c))];
  __syncthreads();
  const int64_t N = nentries(grp, La);
  uint64_t tlo = 0, thi = 0, prd = 0;
  for (int64_t e = (int64_t)blockIdx.x * BLK + threadIdx.x; e < N; e += (int64_t)gridDim.x * BLK) {
    int64_t v;
    int b;
    entry_vb(grp, La, e, v, b);
    if (!live(grp, a, v, b)) continue;
    const int64_t eb = row_of(grp, Lb, bb, v, b);
    if (eb < 0) continue;
    const int64_t u = s_u[b];
    for (int t = 0; t < T; t++) {
      const int cu = s_cu[t * WAVE + b], cv = colr[(int64_t)t * n + v];
      if (cu == cv) continue;
      prd += 16 * (uint64_t)Ca;
      const uint64_t *ar = a.val + (e * T + t) * Ca;
      const uint64_t *br = bb.val + (eb * T + t) * Cb;
      uint64_t lo = 0, hi = 0;
      bool of = false;
      for (int c0 = 0; c0 < Ca; c0 += 4) {  // both rows' slots loaded before they are used
        uint64_t xs[4], ys[4];
#pragma unroll
        for (int q = 0; q < 4; q++) xs[q] = c0 + q < Ca ? ar[c0 + q] : 0;
#pragma unroll
        for (int q = 0; q < 4; q++) ys[q] = c0 + q < Ca ? br[s_yi[c0 + q]] : 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const uint64_t x = xs[q], y = ys[q];
          if (!x || !y) continue;
          uint64_t pl, ph;
    mul_wide(x, y, pl, ph);
          if (w != 1) {
            const uint64_t l2 = pl * w, c2 = __umul64hi(pl, w);
            const uint64_t h2 = ph * w + c2;
            if (__umul64hi(ph, w) != 0 || h2 < c2) of = true;
            pl = l2;
            ph = h2;
          }
          const uint64_t sl = lo + pl;
          hi += ph + (sl < pl ? 1u : 0u);
          lo = sl;
        }
      }
      if (of) atomicOr(&acc.ovf[t], 1u);
      if (!(lo | hi)) continue;
      if (acc.per_src) atomic_add128(&acc.per_src[2 * (u * T + t)], lo, hi);
      if (T == 1) {  // one trial: the thread keeps its sum until the end
        const uint64_t sl = tlo + lo;
        thi += hi + (sl < lo ? 1u : 0u);
        tlo = sl;
      } else {
        atomic_add128(&s_acc[2 * t], lo, hi);
      }
    }
  }
  if (tlo | thi) atomic_add128(&s_acc[0], tlo, thi);
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += blockDim.x)
    if (s_acc[2 * t] | s_acc[2 * t + 1]) atomic_add128(&acc.sum[2 * t], s_acc[2 * t], s_acc[2 * t + 1]);
  prof_flush(grp.prof, prd, 0, 0);
}

// Root merge whose first operand is an AXPY chain read by nothing else:
// count[t] += w * sum over rows of sum over R of (sum_q w_q term_q)[R] * b[K \ {chi u, chi v} \ R],
// the chain's slots computed in the pass (a term is a register, or the
// NodeJoin of a register with a node table through its split map) and never
// stored.  By linearity this is the chain's AXPY followed by k_mroot, with the
// same checked arithmetic, without writing and re-reading the chain's rows.
// Slot-parallel like the AXPY chains: dense groups a wavefront per vertex over
// its live (row, trial, slot) items, sparse groups one thread per item; each
// thread keeps its products' 128-bit sum per trial.
__device__ __forceinline__ uint64_t chain_slot(const AxpyTerms &tm, const uint32_t *s_jm, uint32_t on, bool below,
                                               int64_t e, int64_t v, int t, int T, int c, int C, int cup, bool &of) {
  uint64_t x = 0;
  for (int q = 0; q < tm.n; q++) {
    if (!((on >> q) & 1u)) continue;
    uint64_t xq;
    if (tm.nt[q].val) {
      if (!below) continue;
      const int ns = tm.jns[q];
      const uint32_t *jm = jmap_at(tm, s_jm, q);
      xq = nj_slot_map(tm.a[q].val + (e * T + t) * tm.a[q].C, tm.nt[q].val + (v * T + t) * tm.nt[q].C,
                       split_words(jm, cup, C, c, ns), ns, of);
    } else {
      xq = tm.a[q].val[(e * T + t) * C + c];
    }
    if (xq) add_ck(x, mul_ck(tm.w[q], xq, of), of);
  }
  return x;
}

template <bool DENSE>
__global__ __launch_bounds__(BLK) void k_mroot_terms(GroupDev grp, int64_t n, const uint8_t *colr, LevelDev La,
                                                     LevelDev Lb, AxpyTerms tm, int C, int sa, RegDev bb,
                                                     uint64_t w, AccDev acc, const uint16_t *lut) {
  __shared__ uint16_t s_yi[256];
  __shared__ uint64_t s_acc[2 * 64];
  __shared__ int32_t s_u[WAVE];
  __shared__ uint8_t s_cu[WAVE * WAVE];
  extern __shared__ uint32_t s_jm[];
  load_sources(grp, colr, n, s_u, s_cu);
  load_jmaps(tm, s_jm);
  for (int i = threadIdx.x; i < 2 * 64; i += blockDim.x) s_acc[i] = 0;
  const int T = grp.T, Cb = bb.C, k = grp.k, B = grp.B;
  const uint32_t Kp = (1u << (k - 2)) - 1u;
  for (int c = threadIdx.x; c < C; c += BLK) s_yi[c] = lut[LUT_RANK + (Kp & ~unrank(lut, sa - 2, c))];
  __syncthreads();
  const uint64_t bmask = B >= 64 ? ~0ull : (1ull << B) - 1ull;
  const int per = T * C;
  uint64_t tlo = 0, thi = 0, prd = 0;  // this thread's sum (one trial)
  uint32_t ofm = 0;
  // one (row, trial, slot) item: its products into the thread's sum
  // bmv: dense -- the other operand's activity word at v; cv1: v's colour when
  // one trial (both loaded once per vertex)
  auto item = [&](int64_t e, int64_t v, int b, int t, int c, uint32_t on, uint64_t bmv, int cv1) {
    const int cu = s_cu[t * WAVE + b], cv = (DENSE && T == 1) ? cv1 : colr[(int64_t)t * n + v];
    if (cu == cv) return;
    const int64_t eb = DENSE ? ((bmv >> b) & 1ull ? e : -1) : sparse_entry(Lb, v, b);
    if (eb < 0) return;
    bool of = false;
    const uint64_t x = chain_slot(tm, s_jm, on, v < vbound(grp, s_u[b]), e, v, t, T, c, C, cu - (cv < cu), of);
    prd += 8 * (uint64_t)(tm.n + 1);
    if (of) ofm |= 1u << t;
    if (!x) return;
    const uint64_t y = bb.val[(eb * T + t) * Cb + s_yi[c]];
    if (!y) return;
    uint64_t pl, ph;
    mul_wide(x, y, pl, ph);
    if (w != 1) {
      const uint64_t l2 = pl * w, c2 = __umul64hi(pl, w);
      const uint64_t h2 = ph * w + c2;
      if (__umul64hi(ph, w) != 0 || h2 < c2) ofm |= 1u << t;
      pl = l2;
      ph = h2;
    }
    if (acc.per_src) atomic_add128(&acc.per_src[2 * ((int64_t)s_u[b] * T + t)], pl, ph);
    if (T == 1) {
      const uint64_t sl = tlo + pl;
      thi += ph + (sl < pl ? 1u : 0u);
      tlo = sl;
    } else {
      atomic_add128(&s_acc[2 * t], pl, ph);
    }
  };
  if (DENSE) {
    const int lane = threadIdx.x % 64;
    const int64_t wave = (int64_t)blockIdx.x * (BLK / 64) + threadIdx.x / 64, nwave = (int64_t)gridDim.x * (BLK / 64);
    for (int64_t v = wave; v < grp.n_lim; v += nwave) {
      uint64_t mt[4] = {0, 0, 0, 0}, m = 0;
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (q < tm.n) {
          mt[q] = tm.a[q].mask[v] & bmask;
          m |= mt[q];
        }
      const uint64_t bmv = bb.mask[v] & bmask;
      m &= bmv;  // rows without a partner row add nothing
      if (!m) continue;
      const int cv1 = T == 1 ? colr[v] : 0;
      const int items = __popcll(m) * per;
      for (int it = lane; it < items; it += 64) {
        const int q0 = it / per, r = it - q0 * per, t = r / C, c = r - t * C;
        const int b = nth_bit(m, q0);
        uint32_t on = 0;
        for (int q = 0; q < tm.n; q++) on |= (uint32_t)((mt[q] >> b) & 1ull) << q;
        item(v * B + b, v, b, t, c, on, bmv, cv1);
      }
    }
  } else {
    const int64_t N = (int64_t)(*La.cnt) * per;
    for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
      const int64_t e = i / per;
      const int r = (int)(i - e * per), t = r / C, c = r - t * C;
      int64_t v;
      int b;
      entry_vb(grp, La, e, v, b);
      item(e, v, b, t, c, (1u << tm.n) - 1u, 0, 0);
    }
  }
  for (int t = 0; t < T; t++)
    if ((ofm >> t) & 1u) atomicOr(&acc.ovf[t], 1u);
  if (tlo | thi) atomic_add128(&s_acc[0], tlo, thi);
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += blockDim.x)
    if (s_acc[2 * t] | s_acc[2 * t + 1]) atomic_add128(&acc.sum[2 * t], s_acc[2 * t], s_acc[2 * t + 1]);
  prof_flush(grp.prof, prd, 0, 0);
}

// The same merge for one colouring, by chunks of rows: a wavefront takes R =
// IPL * 64 / C rows at a time, each lane IPL of the chunk's (row, slot) items.
// Every global load of a chunk is issued before any is used: each item's slot
// of the plain terms and its partner slot, and the chunk's rows of the
// NodeJoin terms' inputs and node-table rows, which go to the wavefront's LDS
// stage (coalesced: a chunk's rows are adjacent in the register); then every
// item's splits are computed from LDS.  A chunk costs one memory latency
// instead of a chain of dependent gathers per slot.  NT: the number of terms.
// Stage layout per wavefront (64-bit words): for each NodeJoin term q, R rows
// of a[q] (a[q].C words each) and then the node-table rows (one row in dense
// groups, where a chunk shares its vertex; R rows in sparse groups).
template <bool DENSE, int NT, int IPL>
__global__ __launch_bounds__(BLK) void k_mroot_rows(GroupDev grp, int64_t n, const uint8_t *colr, LevelDev La,
                                                    LevelDev Lb, AxpyTerms tm, int C, int sa, RegDev bb,
                                                    uint64_t w, AccDev acc, const uint16_t *lut, int jm_words,
                                                    int stage_words) {
  __shared__ uint16_t s_yi[256];
  __shared__ uint64_t s_acc[2];
  __shared__ int32_t s_u[WAVE];
  __shared__ uint8_t s_cu[WAVE];
  extern __shared__ uint64_t s_dyn[];  // split maps, then the stages
  uint32_t *s_jm = (uint32_t *)s_dyn;
  for (int i = threadIdx.x; i < WAVE; i += blockDim.x) {
    s_u[i] = i < grp.B ? grp.src[i] : 0;
    s_cu[i] = i < grp.B ? colr[grp.src[i]] : 0;
  }
  load_jmaps(tm, s_jm);
  if (threadIdx.x < 2) s_acc[threadIdx.x] = 0;
  const int k = grp.k, B = grp.B, Cb = bb.C;
  const uint32_t Kp = (1u << (k - 2)) - 1u;
  for (int c = threadIdx.x; c < C; c += BLK) s_yi[c] = lut[LUT_RANK + (Kp & ~unrank(lut, sa - 2, c))];
  __syncthreads();
  const int lane = threadIdx.x % 64;
  uint64_t *stg = s_dyn + (jm_words + 1) / 2 + (size_t)(threadIdx.x / 64) * stage_words;
  const int R = IPL * 64 / C;  // rows per chunk
  int jr[IPL], c[IPL];         // the lane's items: row of the chunk, slot
#pragma unroll
  for (int i = 0; i < IPL; i++) {
    jr[i] = (lane + 64 * i) / C;
    c[i] = lane + 64 * i - jr[i] * C;
  }
  // stage offsets of the NodeJoin terms (rows of a[q], then node-table rows)
  int off_a[NT], off_n[NT];
  {
    int off = 0;
#pragma unroll
    for (int q = 0; q < NT; q++) {
      off_a[q] = off_n[q] = 0;
      if (!tm.nt[q].val) continue;
      off_a[q] = off;
      off += R * tm.a[q].C;
      off_n[q] = off;
      off += (DENSE ? 1 : R) * tm.nt[q].C;
    }
  }
  // the lane's first staged node-table element (sparse groups stage one row per
  // entry): its entry of the chunk and slot
  int nr0[NT], nc0[NT];
#pragma unroll
  for (int q = 0; q < NT; q++) {
    const int Cn = tm.nt[q].val ? tm.nt[q].C : 1;
    nr0[q] = min(lane / Cn, R - 1);
    nc0[q] = lane - (lane / Cn) * Cn;
  }
  const uint64_t bmask = B >= 64 ? ~0ull : (1ull << B) - 1ull;
  const bool same_level = La.mb == Lb.mb;  // sparse: the partner row has the same entry
  uint64_t tlo = 0, thi = 0, prd = 0;
  bool of = false;
  // an item once its loads have landed: xp[q] the plain terms' slots, y the
  // partner slot (0: the item adds nothing)
  auto finish = [&](int jri, int ci, int b, int64_t v, uint32_t on, const uint64_t *xp, uint64_t y, int cv) {
    const int cu = s_cu[b];
    if (cu == cv) return;
    const bool below = v < vbound(grp, s_u[b]);
    const int cup = cu - (cv < cu);
    prd += 8 * (uint64_t)(NT + 1);
    if (!y) return;
    uint64_t x = 0;
#pragma unroll
    for (int q = 0; q < NT; q++) {
      if (!((on >> q) & 1u)) continue;
      uint64_t xq = 0;
      if (tm.nt[q].val) {
        if (!below) continue;
        const int ns = tm.jns[q];
        const uint32_t *jm = jmap_at(tm, s_jm, q);
        const uint32_t *sp = split_words(jm, cup, C, ci, ns);
        const uint64_t *ar = stg + off_a[q] + jri * tm.a[q].C;
        const uint64_t *nr = stg + off_n[q] + (DENSE ? 0 : jri * tm.nt[q].C);
        for (int j = 0; j < ns; j++) {
          const uint32_t w = sp[j];
          const uint64_t z = nr[w & 0xffffu];
          if (!z) continue;
          const uint64_t xa = ar[w >> 16];
          if (xa) add_ck(xq, mul_ck(xa, z, of), of);
        }
      } else {
        xq = xp[q];
      }
      if (xq) add_ck(x, tm.w[q] == 1 ? xq : mul_ck(tm.w[q], xq, of), of);
    }
    if (!x) return;
    uint64_t pl, ph;
    mul_wide(x, y, pl, ph);
    if (w != 1) {
      const uint64_t l2 = pl * w, c2 = __umul64hi(pl, w);
      const uint64_t h2 = ph * w + c2;
      if (__umul64hi(ph, w) != 0 || h2 < c2) of = true;
      pl = l2;
      ph = h2;
    }
    if (acc.per_src) atomic_add128(&acc.per_src[2 * (int64_t)s_u[b]], pl, ph);
    const uint64_t sl = tlo + pl;
    thi += ph + (sl < pl ? 1u : 0u);
    tlo = sl;
  };
  const int64_t wave = (int64_t)blockIdx.x * (BLK / 64) + threadIdx.x / 64, nwave = (int64_t)gridDim.x * (BLK / 64);
  if (DENSE) {
    for (int64_t v = wave; v < grp.n_lim; v += nwave) {
      uint64_t mt[NT], m = 0;
#pragma unroll
      for (int q = 0; q < NT; q++) {
        mt[q] = tm.a[q].mask[v] & bmask;
        m |= mt[q];
      }
      m &= bb.mask[v] & bmask;  // rows without a partner row add nothing
      if (!m) continue;
      const int cv = colr[v];
      const int nrows = __popcll(m);
      for (int j0 = 0; j0 < nrows; j0 += R) {
        // issue: the items' plain-term and partner slots, then the stage
        int bi[IPL];
        uint32_t on[IPL];
        uint64_t xp[IPL][NT], y[IPL];
#pragma unroll
        for (int i = 0; i < IPL; i++) {
          const bool act = jr[i] < R && j0 + jr[i] < nrows;
          bi[i] = act ? nth_bit(m, j0 + jr[i]) : -1;
          on[i] = 0;
          y[i] = 0;
#pragma unroll
          for (int q = 0; q < NT; q++) xp[i][q] = 0;
          if (act && s_cu[bi[i]] != cv) {
            const int64_t row = v * B + bi[i];
#pragma unroll
            for (int q = 0; q < NT; q++) {
              const bool hq = (mt[q] >> bi[i]) & 1ull;
              on[i] |= (uint32_t)hq << q;
              if (!tm.nt[q].val && hq) xp[i][q] = tm.a[q].val[row * C + c[i]];
            }
            y[i] = bb.val[row * Cb + s_yi[c[i]]];
          }
        }
        if (j0 == 0) {
#pragma unroll
          for (int q = 0; q < NT; q++)
            if (tm.nt[q].val)
              for (int i = lane; i < tm.nt[q].C; i += 64) stg[off_n[q] + i] = tm.nt[q].val[v * tm.nt[q].C + i];
        }
#pragma unroll
        for (int q = 0; q < NT; q++) {
          if (!tm.nt[q].val) continue;
          const int Cq = tm.a[q].C;
          if (IPL == 1) {  // row r's source comes from the lane that owns row r (lane r * C)
            for (int i0 = 0; i0 < R * Cq; i0 += 64) {
              const int i = i0 + lane;
              const int r = min(i / Cq, R - 1);
              const int br = __shfl(bi[0], r * C);
              if (i < R * Cq && j0 + r < nrows && ((mt[q] >> br) & 1ull))
                stg[off_a[q] + i] = tm.a[q].val[(v * B + br) * Cq + (i - r * Cq)];
            }
          } else {
            for (int i = lane; i < R * Cq; i += 64) {
              const int r = i / Cq;
              if (j0 + r >= nrows) break;
              const int br = nth_bit(m, j0 + r);
              if ((mt[q] >> br) & 1ull) stg[off_a[q] + i] = tm.a[q].val[(v * B + br) * Cq + (i - r * Cq)];
            }
          }
        }
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < IPL; i++)
          if (bi[i] >= 0) finish(jr[i], c[i], bi[i], v, on[i], xp[i], y[i], cv);
        wave_lds_sync();  // the stage is read before the next chunk overwrites it
      }
    }
  } else {
    const int64_t N = *La.cnt, nch = (N + R - 1) / R;
    for (int64_t ch = wave; ch < nch; ch += nwave) {
      const int64_t e0 = ch * R;
      const int lim = N - e0 < R ? (int)(N - e0) : R;  // entries of this chunk
      int64_t v[IPL];
      int bi[IPL], cv[IPL];
      uint64_t xp[IPL][NT], y[IPL];
#pragma unroll
      for (int i = 0; i < IPL; i++) {
        const int64_t e = e0 + jr[i];
        v[i] = 0;
        bi[i] = -1;
        cv[i] = 0;
        y[i] = 0;
#pragma unroll
        for (int q = 0; q < NT; q++) xp[i][q] = 0;
        if (jr[i] < lim) {
          const int64_t x = La.list[e];
          v[i] = x >> 6;
          bi[i] = (int)(x & 63);
          cv[i] = colr[v[i]];
          const int64_t eb = same_level ? e : sparse_entry(Lb, v[i], bi[i]);
          if (eb >= 0 && s_cu[bi[i]] != cv[i]) {
#pragma unroll
            for (int q = 0; q < NT; q++)
              if (!tm.nt[q].val) xp[i][q] = tm.a[q].val[e * C + c[i]];
            y[i] = bb.val[eb * Cb + s_yi[c[i]]];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < NT; q++) {
        if (!tm.nt[q].val) continue;
        const int Cq = tm.a[q].C, Cn = tm.nt[q].C;
        for (int i = lane; i < lim * Cq; i += 64) stg[off_a[q] + i] = tm.a[q].val[e0 * Cq + i];
        if (IPL == 1) {  // row r's vertex comes from the lane that owns entry r (lane r * C)
          for (int i0 = 0; i0 < lim * Cn; i0 += 64) {
            const int i = i0 + lane;
            const int r = i0 ? min(i / Cn, R - 1) : nr0[q], cc = i0 ? i - (i / Cn) * Cn : nc0[q];
            const int vr = __shfl((int)v[0], r * C);
            if (i < lim * Cn) stg[off_n[q] + i] = tm.nt[q].val[(int64_t)vr * Cn + cc];
          }
        } else {
          for (int i = lane; i < lim * Cn; i += 64) {
            const int r = i / Cn;
            const int64_t vr = La.list[e0 + r] >> 6;
            stg[off_n[q] + i] = tm.nt[q].val[vr * Cn + (i - r * Cn)];
          }
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < IPL; i++)
        if (bi[i] >= 0) finish(jr[i], c[i], bi[i], v[i], (1u << NT) - 1u, xp[i], y[i], cv[i]);
      wave_lds_sync();
    }
  }
  if (of) atomicOr(&acc.ovf[0], 1u);
  if (tlo | thi) atomic_add128(&s_acc[0], tlo, thi);
  __syncthreads();
  if (threadIdx.x == 0 && (s_acc[0] | s_acc[1])) atomic_add128(&acc.sum[0], s_acc[0], s_acc[1]);
  prof_flush(grp.prof, prd, 0, 0);
}

template <bool DENSE, int IPL>
void launch_mroot_rows_nt(int nt, dim3 gr, size_t lds, hipStream_t st, const GroupDev &grp, int64_t n,
                          const uint8_t *colr, LevelDev La, LevelDev Lb, const AxpyTerms &tm, int C, int sa, RegDev b,
                          uint64_t w, AccDev acc, const uint16_t *lut, int jm_words, int words) {
#define CC_MR(NTV)                                                                                                   \
  hipLaunchKernelGGL((k_mroot_rows<DENSE, NTV, IPL>), gr, dim3(BLK), lds, st, grp, n, colr, La, Lb, tm, C, sa, b, w, \
                     acc, lut, jm_words, words)
  switch (nt) {
    case 1: CC_MR(1); break;
    case 2: CC_MR(2); break;
    case 3: CC_MR(3); break;
    default: CC_MR(4); break;
  }
#undef CC_MR
}

// ------------------------------------------------------------------ merges into unary tables
// at_u:  out[u_b][R'] += w * sum over splits of R' \ {chi v} of a[(v,b)] * b[(v,b)]
// !at_u: out[v][R']   += w * (same products, R' \ {chi u_b})
__global__ __launch_bounds__(BLK) void k_munary(GroupDev grp, int64_t n, const uint8_t *colr, LevelDev La,
                                                LevelDev Lb, RegDev a, RegDev bb, uint64_t w, int at_u,
                                                uint64_t *out, int s_out, int C_out, uint32_t *ovf,
                                                const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int T = grp.T, Ca = a.C, Cb = bb.C;
  const int ra = a.s - 2;
  const int64_t per = (int64_t)T * C_out;
  const int64_t N = nentries(grp, La) * per;
  uint64_t ofm = 0, prd = 0, pwr = 0;  // profile: bytes read, written
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t e = i / per;
    const int r = (int)(i - e * per), t = r / C_out, c = r - t * C_out;
    int64_t v;
    int b;
    entry_vb(grp, La, e, v, b);
    const int64_t u = grp.src[b];
    if (v >= vbound(grp, u) || !live(grp, a, v, b)) continue;
    const int64_t eb = row_of(grp, Lb, bb, v, b);
    if (eb < 0) continue;
    const int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
    if (cu == cv) continue;
    const int ckey = at_u ? cu : cv, coth = at_u ? cv : cu;
    if (c == 0) prd += 8 * (uint64_t)(Ca + Cb);  // both rows, once per (entry, trial)
    const uint32_t Rq = spread1(unrank(lut, s_out - 1, c), ckey);
    if (!((Rq >> coth) & 1u)) continue;
    const uint32_t R = Rq & ~(1u << coth);
    const uint64_t *ar = a.val + (e * T + t) * Ca;
    const uint64_t *br = bb.val + (eb * T + t) * Cb;
    uint64_t s = 0;
    bool of = false;
    uint32_t s1 = R;
    for (;;) {
      if (__popc(s1) == ra) {
        uint64_t x = ar[s_rank[squeeze2(s1, cu, cv)]];
        if (x) {
          uint64_t y = br[s_rank[squeeze2(R & ~s1, cu, cv)]];
          if (y) add_ck(s, mul_ck(x, y, of), of);
        }
      }
      if (s1 == 0) break;
      s1 = (s1 - 1) & R;
    }
    if (s) {
      atomic_add_ck(&out[((at_u ? u : v) * T + t) * C_out + c], mul_ck(s, w, of), of);
      pwr += 8;
    }
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

// ------------------------------------------------------------------ pair-keyed merges
// P[(u_b, v)][R'] = w * sum over splits R' = R1 + R2 of a[(v,b)][R1] * b[(v,b)][R2]
// (Procedure 2 of Section 5.1: the two paths from u meet at v with colour
// sets overlapping exactly in {chi u, chi v}; R', R1, R2 with those two
// colours squeezed out).  Dense groups: one thread per (row, trial, output
// slot) into a staging register (rows v * B + b) whose activity word marks
// the nonzero rows.
__global__ __launch_bounds__(BLK) void k_mpair(GroupDev grp, int64_t n, const uint8_t *colr, RegDev a, RegDev bb,
                                               uint64_t w, RegDev dst, uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int T = grp.T, Ca = a.C, Cb = bb.C, C = dst.C;
  const int ra = a.s - 2;
  const int64_t per = (int64_t)T * C;
  const int64_t N = grp.n_lim * (int64_t)grp.B * per;
  uint64_t ofm = 0, prd = 0, pwr = 0;  // profile: bytes read, written (every staged slot)
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t row = i / per;
    const int r = (int)(i - row * per), t = r / C, c = r - t * C;
    const int64_t v = row / grp.B;
    const int b = (int)(row - v * grp.B);
    uint64_t sum = 0;
    bool of = false;
    const int64_t u = grp.src[b];
    if (v != u && live(grp, a, v, b) && live(grp, bb, v, b)) {
      const int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
      if (cu != cv) {
        if (c == 0) prd += 8 * (uint64_t)(Ca + Cb);  // both rows, once per (row, trial)
        const uint32_t R = spread2(unrank(lut, dst.s - 2, c), cu, cv);
        const uint64_t *ar = a.val + (row * T + t) * Ca;
        const uint64_t *br = bb.val + (row * T + t) * Cb;
        uint32_t s1 = R;
        for (;;) {
          if (__popc(s1) == ra) {
            const uint64_t x = ar[s_rank[squeeze2(s1, cu, cv)]];
            if (x) {
              const uint64_t y = br[s_rank[squeeze2(R & ~s1, cu, cv)]];
              if (y) add_ck(sum, mul_ck(x, y, of), of);
            }
          }
          if (s1 == 0) break;
          s1 = (s1 - 1) & R;
        }
        if (sum) sum = mul_ck(sum, w, of);
      }
    }
    dst.val[i] = sum;
    pwr += 8;
    if (sum) atomicOr((unsigned long long *)&dst.mask[v], 1ull << b);
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

// Append the nonzero staged rows as pair-table entries: keys (u_b, v),
// values [T][C].  Entries beyond `cap` are counted but not written.
__global__ __launch_bounds__(BLK) void k_pair_emit(GroupDev grp, RegDev st, int32_t *keys, uint64_t *vals,
                                                   uint64_t cap, unsigned long long *cnt) {
  const int64_t per = (int64_t)grp.T * st.C;
  const int64_t N = grp.n_lim * (int64_t)grp.B;
  for (int64_t row = (int64_t)blockIdx.x * BLK + threadIdx.x; row < N; row += (int64_t)gridDim.x * BLK) {
    const int64_t v = row / grp.B;
    const int b = (int)(row - v * grp.B);
    if (!((st.mask[v] >> b) & 1ull)) continue;
    const unsigned long long pos = atomicAdd(cnt, 1ull);
    if (pos >= cap) continue;
    keys[2 * pos] = grp.src[b];
    keys[2 * pos + 1] = (int32_t)v;
    const uint64_t *sr = st.val + row * per;
    uint64_t *dr = vals + (int64_t)pos * per;
    for (int64_t q = 0; q < per; q++) dr[q] = sr[q];
  }
}

// Table rows aligned to the slots of a pair table's graph: slot e takes
// entry idx[e]'s row, or zeros (idx -1).
__global__ void k_pair_gather(const int64_t *idx, int64_t m2, const uint64_t *vals, int64_t per, uint64_t *tab) {
  const int64_t N = m2 * per;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / per;
    const int64_t j = idx[e];
    tab[i] = j >= 0 ? vals[j * per + (i - e * per)] : 0;
  }
}

// ------------------------------------------------------------------ edge merges
// T[x,y][R'] += w * a[(x,b)][R1] * E(x,y)[Re] * b[(y,b)][R2],  R' \ {chi u_b} = R1 + Re + R2
__global__ __launch_bounds__(BLK) void k_medge(GraphDev g, GroupDev grp, const uint8_t *colr, LevelDev La,
                                               LevelDev Lb, RegDev a, RegDev bb, TabDev et, int e_src_first,
                                               int out_first_is_x, uint64_t w, uint64_t *out, int s_out, int C_out,
                                               uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int T = grp.T, Ca = a.C, Cb = bb.C;
  const int ra = a.s - 2, rb = bb.s - 2;
  const int64_t per = (int64_t)T * C_out;
  const int64_t N = nentries(grp, La) * per;
  uint64_t ofm = 0, prd = 0, pwr = 0;  // profile: bytes read, written
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t e = i / per;
    const int r = (int)(i - e * per), t = r / C_out, c = r - t * C_out;
    int64_t x;
    int b;
    entry_vb(grp, La, e, x, b);
    const int64_t u = grp.src[b];
    if (x >= vbound(grp, u) || !live(grp, a, x, b)) continue;
    const int cu = colr[(int64_t)t * g.n + u], cx = colr[(int64_t)t * g.n + x];
    if (cu == cx) continue;
    const uint64_t *ar = a.val + (e * T + t) * Ca;
    if (c == 0) prd += 8 * (uint64_t)Ca;  // a's row, once per (entry, trial)
    bool of = false;
    for (int64_t ee = g.rp[x]; ee < g.rp[x + 1]; ee++) {
      const int64_t y = g.col[ee];
      if (y >= vbound(grp, u)) break;
      if (c == 0) prd += 4;  // the neighbour id
      const int64_t eb = row_of(grp, Lb, bb, y, b);
      if (eb < 0) continue;
      const int cy = colr[(int64_t)t * g.n + y];
      if (cy == cx || cy == cu) continue;
      if (c == 0) prd += 8 * (uint64_t)(Cb + (et.val ? et.C : 0));  // b's row and the edge's
      const uint32_t Rp = spread2(unrank(lut, s_out - 2, c), cx, cy);
      if (!((Rp >> cu) & 1u)) continue;
      const uint32_t R = Rp & ~(1u << cu);
      const uint64_t *br = bb.val + (eb * T + t) * Cb;
      const int64_t tslot = e_src_first ? ee : g.rev[ee];
      const uint64_t *er = et.val ? et.val + (tslot * T + t) * et.C : nullptr;
      uint64_t s = 0;
      uint32_t s1 = R;
      for (;;) {
        if (__popc(s1) == ra) {
          uint64_t xa = ar[s_rank[squeeze2(s1, cu, cx)]];
          if (xa) {
            uint32_t Q = R & ~s1;
            uint32_t s2 = Q;
            for (;;) {
              if (__popc(s2) == rb) {
                uint64_t xb = br[s_rank[squeeze2(s2, cu, cy)]];
                uint32_t Qe = Q & ~s2;
                uint64_t xe = er ? er[s_rank[squeeze2(Qe, cx, cy)]] : (Qe == 0 ? 1u : 0u);
                if (xb && xe) add_ck(s, mul_ck(mul_ck(xa, xb, of), xe, of), of);
              }
              if (s2 == 0) break;
              s2 = (s2 - 1) & Q;
            }
          }
        }
        if (s1 == 0) break;
        s1 = (s1 - 1) & R;
      }
      if (s) {
        const int64_t oslot = out_first_is_x ? ee : g.rev[ee];
        atomic_add_ck(&out[(oslot * T + t) * C_out + c], mul_ck(s, w, of), of);
        pwr += 8;
      }
    }
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

// The same merge vertex-major: a wavefront owns a vertex x with all the
// group's sources that have a row of a at x, reads x's neighbour list once
// with each neighbour's source bits of b, and gives each lane one (neighbour,
// trial, output slot): the lane sums its slot over the sources common to x
// and its neighbour y, then adds the sum to the edge's slot once.  Rows are
// found from the bits (dense: (v, b); sparse: the level's base and the
// marks below b).  Requires T * C_out <= 64.
template <bool DENSE>
__global__ __launch_bounds__(BLK) void k_medge_v(GraphDev g, GroupDev grp, const uint8_t *colr, LevelDev La,
                                                 LevelDev Lb, RegDev a, RegDev bb, TabDev et, int e_src_first,
                                                 int out_first_is_x, uint64_t w, uint64_t *out, int s_out, int C_out,
                                                 uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint32_t s_uo[64];  // unranked output slots
  __shared__ int32_t s_u[WAVE];
  __shared__ int32_t s_bnd[WAVE];
  __shared__ uint8_t s_cu[WAVE * WAVE];
  load_rank(s_rank, lut);
  load_sources(grp, colr, g.n, s_u, s_cu);
  for (int i = threadIdx.x; i < WAVE; i += blockDim.x) s_bnd[i] = i < grp.B ? (int32_t)vbound(grp, grp.src[i]) : -1;
  for (int c = threadIdx.x; c < C_out; c += blockDim.x) s_uo[c] = unrank(lut, s_out - 2, c);
  __syncthreads();
  const int T = grp.T, B = grp.B, Ca = a.C, Cb = bb.C;
  const int ra = a.s - 2, rb = bb.s - 2;
  const int per = T * C_out, NY = 64 / per;  // neighbours per round
  const int lane = threadIdx.x % 64;
  const int yl = lane / per, r = lane - yl * per, t = r / C_out, c = r - t * C_out;
  const bool lane_on = yl < NY;
  const uint64_t bmask = B >= 64 ? ~0ull : (1ull << B) - 1ull;
  const int64_t n = g.n;
  uint64_t ofm = 0, prd = 0, pwr = 0;  // profile: bytes read, written
  const int64_t wave = (int64_t)blockIdx.x * (BLK / 64) + threadIdx.x / 64, nwave = (int64_t)gridDim.x * (BLK / 64);
  const int64_t nitems = DENSE ? grp.n_lim : (int64_t)La.cnt[1];
  for (int64_t it = wave; it < nitems; it += nwave) {
    const int x = DENSE ? (int)it : La.vlist[it];
    uint64_t A;
    int64_t abase = 0;
    if (DENSE) {
      A = a.mask[x] & bmask;
    } else {
      const ulonglong2 p = ((const ulonglong2 *)La.mb)[x];
      A = p.x;
      abase = (int64_t)p.y;
    }
    const uint64_t Aall = A;  // sparse: the entries of x are numbered over all its marks
    // sources whose walks may pass x
    A &= __ballot(lane < B && s_bnd[lane] > x);
    if (!A) continue;
    int umax = 0;
    for (uint64_t q = A; q; q &= q - 1) umax = max(umax, s_bnd[__builtin_ctzll(q)]);
    const int cx = colr[(int64_t)t * n + x];
    const int64_t r0 = g.rp[x], r1 = g.rp[x + 1];
    bool of = false;
    for (int64_t j0 = r0; j0 < r1; j0 += 64) {
      const int64_t ee = j0 + lane;
      int y = ee < r1 ? g.col[ee] : VNONE;
      if (y >= umax || (DENSE && y >= grp.n_lim)) y = VNONE;  // ascending: the later ones too
      if (grp.prof && y != VNONE) prd += 4;  // the neighbour id
      uint64_t Bm = 0;
      int64_t bbase = 0;
      if (y != VNONE) {
        if (DENSE) {
          Bm = bb.mask[y];
        } else {
          const ulonglong2 p = ((const ulonglong2 *)Lb.mb)[y];
          Bm = p.x;
          bbase = (int64_t)p.y;
        }
      }
      const uint64_t Bfull = Bm;
      Bm &= A;
      uint64_t todo = __ballot(Bm != 0);
      const bool stop = __ballot(y == VNONE) != 0;
      while (todo) {
        // this round: the next NY neighbours with common sources
        int jn = -1;
        uint64_t tcur = todo;
        for (int i = 0; i < NY; i++) {
          const int jj = tcur ? __builtin_ctzll(tcur) : -1;
          if (i == yl) jn = jj;
          if (tcur) tcur &= tcur - 1;
        }
        todo = tcur;
        const int yv = __shfl(y, jn < 0 ? 0 : jn);
        const uint64_t Bv = __shfl(Bm, jn < 0 ? 0 : jn), Bf = __shfl(Bfull, jn < 0 ? 0 : jn);
        const int64_t bbv = __shfl(bbase, jn < 0 ? 0 : jn);
        if (!lane_on || jn < 0) continue;
        const int cy = colr[(int64_t)t * n + yv];
        if (cy == cx) continue;
        if (grp.prof && c == 0 && et.val) prd += 8 * (uint64_t)et.C;  // the edge's row
        const uint32_t Rp = spread2(s_uo[c], cx, cy);
        const int64_t es = j0 + jn;
        const int64_t tslot = e_src_first ? es : g.rev[es];
        const uint64_t *er = et.val ? et.val + (tslot * T + t) * et.C : nullptr;
        uint64_t sum = 0;
        for (uint64_t q = Bv; q; q &= q - 1) {
          const int b = __builtin_ctzll(q);
          if (yv >= s_bnd[b]) continue;
          const int cu = s_cu[t * WAVE + b];
          if (cu == cx || cu == cy) continue;
          if (grp.prof && c == 0) prd += 8 * (uint64_t)(Ca + Cb);  // both rows, once per (source, edge, trial)
          if (!((Rp >> cu) & 1u)) continue;
          const uint32_t R = Rp & ~(1u << cu);
          const uint64_t lowb = (1ull << b) - 1ull;
          const int64_t ea = DENSE ? (int64_t)x * B + b : abase + __popcll(Aall & lowb);
          const int64_t eb = DENSE ? (int64_t)yv * B + b : bbv + __popcll(Bf & lowb);
          const uint64_t *ar = a.val + (ea * T + t) * Ca;
          const uint64_t *br = bb.val + (eb * T + t) * Cb;
          // R = s1 + s2 + Qe: the colours of a's row, of b's row and of the edge table's
          const int nR = __popc(R);
          if (ra > nR) continue;
          for (uint32_t cm = (1u << ra) - 1u; cm < (1u << nR); cm = ra ? next_comb(cm) : (1u << nR)) {
            const uint32_t s1 = deposit(cm, R);
            const uint64_t xa = ar[s_rank[squeeze2(s1, cu, cx)]];
            if (!xa) continue;
            const uint32_t Q = R & ~s1;
            const int nQ = nR - ra;
            if (!er) {  // no edge table: b's row takes all of Q
              if (nQ != rb) continue;
              const uint64_t xb = br[s_rank[squeeze2(Q, cu, cy)]];
              if (xb) add_ck(sum, mul_ck(xa, xb, of), of);
              continue;
            }
            if (rb > nQ) continue;
            for (uint32_t cq = (1u << rb) - 1u; cq < (1u << nQ); cq = rb ? next_comb(cq) : (1u << nQ)) {
              const uint32_t s2 = deposit(cq, Q);
              const uint64_t xb = br[s_rank[squeeze2(s2, cu, cy)]];
              if (!xb) continue;
              const uint64_t xe = er[s_rank[squeeze2(Q & ~s2, cx, cy)]];
              if (xe) add_ck(sum, mul_ck(mul_ck(xa, xb, of), xe, of), of);
            }
          }
        }
        if (sum) {
          const int64_t oslot = out_first_is_x ? es : g.rev[es];
          atomic_add_ck(&out[(oslot * T + t) * C_out + c], mul_ck(sum, w, of), of);
          pwr += 8;
        }
      }
      if (stop) break;
    }
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

// T[u,y] += w * A[u][Ra] * E(u,y)[Re] * b[(y,b)][R2] over the lower neighbours y of u_b.
__global__ __launch_bounds__(BLK) void k_medge_t(GraphDev g, GroupDev grp, const uint8_t *colr,
                                                 const int32_t *lowcnt, int max_low, TabDev nt, LevelDev Lb,
                                                 RegDev bb, TabDev et, int e_src_first, int out_first_is_u,
                                                 uint64_t w, uint64_t *out, int s_out, int C_out, uint32_t *ovf,
                                                 const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int T = grp.T, Cb = bb.C;
  const int rA = nt.val ? nt.s - 1 : 0, rb = bb.s - 2;
  const int64_t per = (int64_t)T * C_out;
  const int64_t N = (int64_t)grp.B * max_low * per;
  uint64_t ofm = 0, prd = 0, pwr = 0;  // profile: bytes read, written
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t en = i / per;
    const int r = (int)(i - en * per), t = r / C_out, c = r - t * C_out;
    const int b = (int)(en / max_low), j = (int)(en - (int64_t)b * max_low);
    const int64_t u = grp.src[b];
    if (j >= lowcnt[u]) continue;
    const int64_t es = g.rp[u] + j;
    const int64_t y = g.col[es];
    const int64_t eb = row_of(grp, Lb, bb, y, b);
    if (eb < 0) continue;
    const int cu = colr[(int64_t)t * g.n + u], cy = colr[(int64_t)t * g.n + y];
    if (cu == cy) continue;
    // b's row, the edge's and the node table's, once per (source, edge, trial)
    if (c == 0) prd += 8 * (uint64_t)(Cb + (et.val ? et.C : 0) + (nt.val ? nt.C : 0));
    const uint32_t R = spread2(unrank(lut, s_out - 2, c), cu, cy);
    const uint64_t *br = bb.val + (eb * T + t) * Cb;
    const int64_t tslot = e_src_first ? es : g.rev[es];
    const uint64_t *er = et.val ? et.val + (tslot * T + t) * et.C : nullptr;
    const uint64_t *ar = nt.val ? nt.val + (u * T + t) * nt.C : nullptr;
    uint64_t s = 0;
    bool of = false;
    uint32_t sA = R;
    for (;;) {
      if (__popc(sA) == rA) {
        uint64_t xa = ar ? ar[s_rank[squeeze1(sA, cu)]] : 1u;
        if (xa) {
          uint32_t Q = R & ~sA;
          uint32_t s2 = Q;
          for (;;) {
            if (__popc(s2) == rb) {
              uint64_t xb = br[s_rank[squeeze2(s2, cu, cy)]];
              uint32_t Qe = Q & ~s2;
              uint64_t xe = er ? er[s_rank[squeeze2(Qe, cu, cy)]] : (Qe == 0 ? 1u : 0u);
              if (xb && xe) add_ck(s, mul_ck(mul_ck(xa, xb, of), xe, of), of);
            }
            if (s2 == 0) break;
            s2 = (s2 - 1) & Q;
          }
        }
      }
      if (sA == 0) break;
      sA = (sA - 1) & R;
    }
    if (s) {
      const int64_t oslot = out_first_is_u ? es : g.rev[es];
      atomic_add_ck(&out[(oslot * T + t) * C_out + c], mul_ck(s, w, of), of);
      pwr += 8;
    }
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
  prof_flush(grp.prof, prd, pwr, 0);
}

const uint16_t *cur_lut() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return lut_device(dev);
}

int fgrid(const GroupDev &grp, int64_t per_entry) {
  if (!grp.dense) return 8192;
  int64_t tot = grp.n_lim * (int64_t)grp.B * per_entry;
  return (int)std::max<int64_t>(1, std::min<int64_t>((tot + BLK - 1) / BLK, 65536));
}

}  // namespace

static void compact(const GroupDev &grp, LevelDev L, hipStream_t st) {
  const int64_t nv = grp.n_lim;
  const int nb = (int)((nv + CH - 1) / CH);
  hipLaunchKernelGGL(k_cmp_count, dim3(nb), dim3(BLK), 0, st, L.mb, nv, L.bcnt, grp.prof);
  hipLaunchKernelGGL(k_cmp_scan, dim3(1), dim3(BLK), 0, st, L.bcnt, nb, L.cnt);
  hipLaunchKernelGGL(k_cmp_emit, dim3(nb), dim3(BLK), 0, st, L.mb, nv, L.bcnt, L.list, L.vlist, grp.prof);
}

int64_t level_chunks(int64_t n_lim) { return (n_lim + CH - 1) / CH; }

void launch_level_init(const GraphDev &g, const GroupDev &grp, const int32_t *lowcnt, int max_low, LevelDev L,
                       hipStream_t st) {
  const int64_t N = (int64_t)grp.B * max_low;
  hipLaunchKernelGGL(k_mark_init, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((N + BLK - 1) / BLK, 4096))),
                     dim3(BLK), 0, st, g, grp, lowcnt, max_low, L);
}

void launch_level_next(const GraphDev &g, const GroupDev &grp, LevelDev Lin, LevelDev Lout, hipStream_t st) {
  hipLaunchKernelGGL(k_mark_next, dim3(8192), dim3(BLK), 0, st, g, grp, Lin, Lout);
  compact(grp, Lout, st);
}

void launch_level_compact(const GroupDev &grp, LevelDev L, hipStream_t st) { compact(grp, L, st); }

// clear the marks for the next group (the list, base and count are rewritten by the next compaction)
void launch_level_reset(const GroupDev &grp, LevelDev L, hipStream_t st) {
  launch_fill_u64(L.mb, 2 * grp.n_lim, st);
}

void launch_init(const GraphDev &g, const GroupDev &grp, const int32_t *lowcnt, int max_low, const uint8_t *colr,
                 LevelDev L, RegDev dst, TabDev etab, int e_src_first, TabDev ntab, uint32_t *ovf, hipStream_t st) {
  int64_t N = (int64_t)grp.B * max_low * grp.T * dst.C;
  int gr = (int)std::max<int64_t>(1, std::min<int64_t>((N + BLK - 1) / BLK, 65536));
  hipLaunchKernelGGL(k_init, dim3(gr), dim3(BLK), 0, st, g, grp, lowcnt, max_low, colr, L, dst, etab, e_src_first,
                     ntab, ovf, cur_lut());
}

bool epi_fits(int ncols, int T, int etab_C) {
  return ncols <= VMAX_C && T <= WAVE && etab_C <= 256 && ejv_lds(ncols, EPI_MAX_REGS, true, WAVE) <= EJV_LDS_MAX;
}

// EdgeJoin slot maps: for colours k and input rank ra (slots of the input
// rows: C(k-2, ra)), entry [cu][cv][cw][c] is the output slot of input slot
// c when the path from a source of colour cu steps from a vertex of colour cv
// to one of colour cw -- the rank of (R + cv) with cu and cw squeezed out,
// where R is slot c's colour set spread around cu and cv -- or 0xff when cw is
// in R or the three colours are not distinct.  Rows padded to four slots.
// Built on the host once per device and k, kept in the constant-table pool
// (static device memory) until the process ends.
constexpr size_t EJMAP_MAX = 16384;  // bytes of one map (it is copied into LDS)
namespace {
struct EjMaps {
  uint32_t *d[12] = {};
  int words[12] = {}, cp[12] = {}, ca[12] = {};
};
std::mutex ejm_mu;
std::map<std::pair<int, int>, EjMaps> ejm;

int host_binom(int n, int r) {
  if (r < 0 || r > n) return 0;
  long c = 1;
  for (int i = 1; i <= r; i++) c = c * (n - r + i) / i;
  return (int)c;
}
int host_rank(uint32_t m) {  // colex rank among masks of the same popcount
  int idx = 0, i = 0;
  for (int p = 0; p < 32; p++)
    if ((m >> p) & 1u) idx += host_binom(p, ++i);
  return idx;
}
}  // namespace

static bool njmaps_build(int dev, int k);

bool ejmaps_prepare(int k) {
  if (k < 3 || k > 12) return true;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(ejm_mu);
  if (!njmaps_build(dev, k)) return false;
  if (ejm.count({dev, k})) return true;
  EjMaps M;
  for (int ra = 0; ra <= k - 2; ra++) {
    const int ca = host_binom(k - 2, ra), cp = (ca + 3) & ~3;
    const size_t bytes = (size_t)k * k * k * cp;
    if (bytes > EJMAP_MAX || host_binom(k - 2, ra + 1) > 255) continue;
    std::vector<uint32_t> um(ca);
    for (uint32_t m = 0; m < (1u << (k - 2)); m++)
      if (__builtin_popcount(m) == ra) um[host_rank(m)] = m;
    std::vector<uint8_t> h(bytes, 0xff);
    for (int cu = 0; cu < k; cu++)
      for (int cv = 0; cv < k; cv++)
        for (int cw = 0; cw < k; cw++) {
          if (cu == cv || cu == cw || cv == cw) continue;
          uint8_t *row = &h[(((size_t)cu * k + cv) * k + cw) * cp];
          for (int c = 0; c < ca; c++) {
            const uint32_t R = dev::spread2(um[c], cu, cv);
            if ((R >> cw) & 1u) continue;
            row[c] = (uint8_t)host_rank(dev::squeeze2(R | (1u << cv), cu, cw));
          }
        }
    uint32_t *d = (uint32_t *)table_pool_alloc(bytes);
    if (!d) return false;
    if (!upload_sync(d, h.data(), bytes)) return false;
    M.d[ra] = d;
    M.words[ra] = (int)(bytes / 4);
    M.cp[ra] = cp;
    M.ca[ra] = ca;
  }
  ejm[{dev, k}] = M;
  return true;
}

static bool getenv_flag_off(const char *name) {
  const char *e = std::getenv(name);
  return e && e[0] == '0';
}

// the prepared map for (k, ra) on the current device, if any (allocates nothing)
static bool ejmap_find(int k, int ra, int ca, const uint32_t **p, int *words, int *cp) {
  if (ra < 0 || ra > 11) return false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(ejm_mu);
  auto it = ejm.find({dev, k});
  if (it == ejm.end() || !it->second.d[ra] || it->second.ca[ra] != ca) return false;
  *p = it->second.d[ra];
  *words = it->second.words[ra];
  *cp = it->second.cp[ra];
  return true;
}

// NodeJoin split maps for colours k, output rank ro (dst slots C(k-2, ro)) and
// nt rank rA (nt slots C(k-1, rA), a slots C(k-2, ro-rA)): per output slot c
// and split j, xi[c][j] (bytes; the map's first words) then yi[cu'][c][j]
// (16-bit), as nj_slot_map reads them.  Built with the slot maps above.
constexpr size_t NJMAP_MAX = 16384, NJMAP_LDS_MAX = 32768;
namespace {
struct NjMaps {
  uint32_t *d[12][12] = {};
  int words[12][12] = {}, ns[12][12] = {};
};
std::map<std::pair<int, int>, NjMaps> njm;  // guarded by ejm_mu
}  // namespace

static bool njmaps_build(int dev, int k) {  // ejm_mu held
  if (njm.count({dev, k})) return true;
  NjMaps M;
  for (int ro = 1; ro <= k - 2; ro++)
    for (int rA = 1; rA <= ro; rA++) {
      const int C = host_binom(k - 2, ro), ns = host_binom(ro, rA);
      const size_t bytes = (size_t)(k - 1) * C * ns * 4;  // one 32-bit word per (cu', c, split)
      if (bytes > NJMAP_MAX || host_binom(k - 2, ro - rA) > 65535 || host_binom(k - 1, rA) > 65535) continue;
      std::vector<uint32_t> uo(C);
      for (uint32_t m = 0; m < (1u << (k - 2)); m++)
        if (__builtin_popcount(m) == ro) uo[host_rank(m)] = m;
      std::vector<uint32_t> h((size_t)(k - 1) * C * ns, 0);
      for (int c = 0; c < C; c++) {
        int j = 0;
        for (uint32_t S = uo[c];; S = (S - 1) & uo[c]) {  // subsets of uo[c] of size rA, in a fixed order
          if (__builtin_popcount(S) == rA) {
            const uint32_t xi = (uint32_t)host_rank(uo[c] & ~S);  // the input row's slot
            for (int cu = 0; cu < k - 1; cu++) {
              const uint32_t Sp = (S & ((1u << cu) - 1u)) | ((S >> cu) << (cu + 1));  // zero inserted at cu
              h[((size_t)cu * C + c) * ns + j] = (uint32_t)host_rank(Sp) | (xi << 16);
            }
            j++;
          }
          if (S == 0) break;
        }
      }
      uint32_t *d = (uint32_t *)table_pool_alloc(bytes);
      if (!d) return false;
      if (!upload_sync(d, h.data(), bytes)) return false;
      M.d[ro][rA] = d;
      M.words[ro][rA] = (int)(bytes / 4);
      M.ns[ro][rA] = ns;
    }
  njm[{dev, k}] = M;
  return true;
}

static bool njmap_find(int k, int ro, int rA, int C, int Ca, int Cn, const uint32_t **p, int *words, int *ns) {
  if (ro < 1 || ro > 11 || rA < 1 || rA > ro || k < 3 || k > 12) return false;
  if (C != host_binom(k - 2, ro) || Ca != host_binom(k - 2, ro - rA) || Cn != host_binom(k - 1, rA)) return false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(ejm_mu);
  auto it = njm.find({dev, k});
  if (it == njm.end() || !it->second.d[ro][rA]) return false;
  *p = it->second.d[ro][rA];
  *words = it->second.words[ro][rA];
  *ns = it->second.ns[ro][rA];
  return true;
}

void launch_ej_epi(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev Lin, RegDev a,
                   const Epilogue &epi_in, TabDev etab, int e_src_first, uint32_t *ovf, AccDev acc, hipStream_t st) {
  Epilogue epi = epi_in;
  epi.ann_lanes = getenv_flag_off("CC_EJANNLANES") ? 0 : 1;
  const bool ep = epi.nops > 0;
  if (!ep && grp.dense && grp.nh > 0 && grp.split_lo < grp.n_lim) {
    // the hubs' rows and activity words start at zero: their chunks add into them
    const RegDev &d = epi.regs[0].r;
    const int64_t per = (int64_t)grp.B * grp.T * d.C;
    launch_fill_u64(d.val + grp.split_lo * per, (grp.n_lim - grp.split_lo) * per, st);
    launch_fill_u64(d.mask + grp.split_lo, grp.n_lim - grp.split_lo, st);
  }
  const uint32_t *em = nullptr;
  int emw = 0, emcp = 0;
  const bool mp = !etab.val && !getenv_flag_off("CC_EJMAP") && ejmap_find(grp.k, a.s - 2, a.C, &em, &emw, &emcp);
  const size_t mapb = mp ? (size_t)emw * 4 : 0;
  // four wavefronts per workgroup when their LDS columns fit, else one
  const bool wide = ejv_lds(epi.ncols, epi.nregs, ep, EJ_BLK) + mapb <= EJV_LDS_MAX;
  const int nb = wide ? EJ_BLK : WAVE;
  const size_t lds = ejv_lds(epi.ncols, epi.nregs, ep, nb) + mapb;
  // sparse groups meet few sources per vertex: four vertices per wavefront
  const bool quarter = !grp.dense && grp.T <= 16;
  // one trial: (neighbour, source) pairs packed over the lanes
  const bool pack = grp.T == 1 && grp.k <= 16 && !getenv_flag_off("CC_EJPACK");
  const bool spk = quarter && pack && mp && !ep && !etab.val;  // sparse, packed: EJ_PACK_SW lanes per vertex
  const int vpw = spk ? WAVE / EJ_PACK_SW : quarter ? 4 : 1;  // vertices per wavefront
  const int64_t nw = (grp.n_lim + vpw - 1) / vpw;  // wavefronts' worth of vertices
  const int gr = (int)std::max<int64_t>(1, std::min<int64_t>((nw + nb / WAVE - 1) / (nb / WAVE), 32768 / (nb / WAVE)));
#define CC_EJV(ANN_, SW_, EPI_, NB_, MAP_)                                                                   \
  hipLaunchKernelGGL((k_ejv<ANN_, SW_, EPI_, NB_, MAP_>), dim3(gr), dim3(NB_), lds, st, g, grp, colr, Lin, a, epi, \
                     etab, e_src_first, ovf, acc, cur_lut(), em, emw, emcp)
#define CC_EJV2(ANN_, SW_, EPI_, MAP_) \
  if (wide) CC_EJV(ANN_, SW_, EPI_, EJ_BLK, MAP_); else CC_EJV(ANN_, SW_, EPI_, WAVE, MAP_)
  const int sel = (mp ? 8 : 0) | (etab.val ? 4 : 0) | (quarter ? 2 : 0) | (ep ? 1 : 0);
  switch (sel) {
    case 0: CC_EJV2(false, 64, false, false); break;
    case 1: CC_EJV2(false, 64, true, false); break;
    case 2: CC_EJV2(false, 16, false, false); break;
    case 3: CC_EJV2(false, 16, true, false); break;
    case 4: CC_EJV2(true, 64, false, false); break;
    case 5: CC_EJV2(true, 64, true, false); break;
    case 6: CC_EJV2(true, 16, false, false); break;
    case 7: CC_EJV2(true, 16, true, false); break;
    case 8:
      if (pack) {
        if (wide)
          hipLaunchKernelGGL((k_ejv<false, 64, false, EJ_BLK, true, true>), dim3(gr), dim3(EJ_BLK), lds, st, g, grp,
                             colr, Lin, a, epi, etab, e_src_first, ovf, acc, cur_lut(), em, emw, emcp);
        else
          hipLaunchKernelGGL((k_ejv<false, 64, false, WAVE, true, true>), dim3(gr), dim3(WAVE), lds, st, g, grp, colr,
                             Lin, a, epi, etab, e_src_first, ovf, acc, cur_lut(), em, emw, emcp);
      } else {
        CC_EJV2(false, 64, false, true);
      }
      break;
    case 9: CC_EJV2(false, 64, true, true); break;
    case 10:
      if (pack) {
        if (wide)
          hipLaunchKernelGGL((k_ejv<false, EJ_PACK_SW, false, EJ_BLK, true, true>), dim3(gr), dim3(EJ_BLK), lds, st, g,
                             grp, colr, Lin, a, epi, etab, e_src_first, ovf, acc, cur_lut(), em, emw, emcp);
        else
          hipLaunchKernelGGL((k_ejv<false, EJ_PACK_SW, false, WAVE, true, true>), dim3(gr), dim3(WAVE), lds, st, g, grp,
                             colr, Lin, a, epi, etab, e_src_first, ovf, acc, cur_lut(), em, emw, emcp);
      } else {
        CC_EJV2(false, 16, false, true);
      }
      break;
    default: CC_EJV2(false, 16, true, true); break;
  }
#undef CC_EJV2
#undef CC_EJV
}

void launch_ej(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev Lin, LevelDev Lout, RegDev a,
               RegDev dst, TabDev etab, int e_src_first, uint32_t *ovf, hipStream_t st) {
  if (epi_fits(dst.C, grp.T, etab.val ? etab.C : 0)) {
    Epilogue epi{};
    epi.nops = 0;
    epi.nregs = 1;
    epi.ncols = dst.C;
    epi.regs[0] = EpiReg{dst, Lout, 0, 1};
    launch_ej_epi(g, grp, colr, Lin, a, epi, etab, e_src_first, ovf, AccDev{nullptr, nullptr, nullptr}, st);
    return;
  }
  const int64_t N = grp.dense ? grp.n_lim * grp.B : (int64_t)1 << 62;
  const int gr = (int)std::max<int64_t>(1, std::min<int64_t>(N, 32768));
  const size_t lds = (size_t)2 * grp.T * dst.C * sizeof(uint64_t);
  // dense: the kernel sets the activity bit of each live row (v, b); the
  // words start at zero
  if (grp.dense) launch_fill_u64(dst.mask, grp.n_lim, st);
  if (etab.val)
    hipLaunchKernelGGL(k_ej<true>, dim3(gr), dim3(WAVE), lds, st, g, grp, colr, Lin, Lout, a, dst, etab, e_src_first,
                       ovf, cur_lut());
  else
    hipLaunchKernelGGL(k_ej<false>, dim3(gr), dim3(WAVE), lds, st, g, grp, colr, Lin, Lout, a, dst, etab,
                       e_src_first, ovf, cur_lut());
}

bool launch_ej_dual(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev Lin, LevelDev Lout,
                    RegDev a1, RegDev d1, RegDev a2, RegDev d2, uint32_t *ovf, hipStream_t st) {
  if (grp.T != 1 || grp.k > 16 || getenv_flag_off("CC_EJPACK") || getenv_flag_off("CC_EJMAP") ||
      getenv_flag_off("CC_EJDUAL"))
    return false;
  if (!grp.dense && grp.T > 16) return false;
  const uint32_t *m1 = nullptr, *m2 = nullptr;
  int w1 = 0, cp1 = 0, w2 = 0, cp2 = 0;
  if (!ejmap_find(grp.k, a1.s - 2, a1.C, &m1, &w1, &cp1) || !ejmap_find(grp.k, a2.s - 2, a2.C, &m2, &w2, &cp2))
    return false;
  // the LDS columns of both outputs bound the wavefronts per compute unit: a
  // pair with many output slots runs as two launches (CC_EJDUAL_COLS: the limit)
  static const int max_cols = [] {
    const char *ev = getenv("CC_EJDUAL_COLS");
    return ev ? atoi(ev) : 16;
  }();
  if (d1.C + d2.C > std::min(max_cols, VMAX_C)) return false;
  const size_t lds = ejv_lds(d1.C + d2.C, 2, false, EJ_BLK) + (size_t)(w1 + w2) * 4;
  if (lds > EJV_LDS_MAX) return false;
  Epilogue epi{};
  epi.nops = 0;
  epi.nregs = 2;
  epi.ncols = d1.C + d2.C;
  epi.regs[0] = EpiReg{d1, Lout, 0, 1};
  epi.regs[1] = EpiReg{d2, Lout, d1.C, 1};
  epi.in2 = a2;
  epi.map2 = m2;
  epi.map2_w = w2;
  epi.map2_cp = cp2;
  if (grp.dense && grp.nh > 0 && grp.split_lo < grp.n_lim) {
    // the hubs' rows and activity words start at zero: their chunks add into them
    for (const RegDev *d : {&d1, &d2}) {
      const int64_t per = (int64_t)grp.B * grp.T * d->C;
      launch_fill_u64(d->val + grp.split_lo * per, (grp.n_lim - grp.split_lo) * per, st);
      launch_fill_u64(d->mask + grp.split_lo, grp.n_lim - grp.split_lo, st);
    }
  }
  const int vpw = grp.dense ? 1 : WAVE / EJ_PACK_SW;
  const int64_t nw = (grp.n_lim + vpw - 1) / vpw;
  const int gr = (int)std::max<int64_t>(1, std::min<int64_t>((nw + EJ_BLK / WAVE - 1) / (EJ_BLK / WAVE),
                                                             32768 / (EJ_BLK / WAVE)));
  const AccDev acc{nullptr, nullptr, nullptr};
  if (grp.dense)
    hipLaunchKernelGGL((k_ejv<false, 64, false, EJ_BLK, true, true, true>), dim3(gr), dim3(EJ_BLK), lds, st, g, grp,
                       colr, Lin, a1, epi, TabDev{nullptr, 0, 0}, 0, ovf, acc, cur_lut(), m1, w1, cp1);
  else
    hipLaunchKernelGGL((k_ejv<false, EJ_PACK_SW, false, EJ_BLK, true, true, true>), dim3(gr), dim3(EJ_BLK), lds, st, g,
                       grp, colr, Lin, a1, epi, TabDev{nullptr, 0, 0}, 0, ovf, acc, cur_lut(), m1, w1, cp1);
  return true;
}

void launch_nj(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev L, RegDev a, RegDev dst,
               TabDev ntab, uint32_t *ovf, hipStream_t st) {
  if (grp.dense) {
    const int gr = (int)std::max<int64_t>(1, std::min<int64_t>((grp.n_lim + 3) / 4, 65536));
    hipLaunchKernelGGL(k_nj_dense, dim3(gr), dim3(BLK), 0, st, grp, g.n, colr, a, dst, ntab, ovf, cur_lut());
    return;
  }
  hipLaunchKernelGGL(k_nj, dim3(fgrid(grp, (int64_t)grp.T * dst.C)), dim3(BLK), 0, st, grp, g.n, colr, L, a, dst,
                     ntab, ovf, cur_lut());
}

void launch_axpy(const GroupDev &grp, LevelDev L, RegDev a, RegDev dst, uint64_t w, int first, uint32_t *ovf,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(fgrid(grp, (int64_t)grp.T * dst.C)), dim3(BLK), 0, st, grp, L, a, dst, w, first,
                     ovf);
  if (grp.dense)
    hipLaunchKernelGGL(k_mask_or, dim3((unsigned)std::min<int64_t>((grp.n_lim + BLK - 1) / BLK, 8192)), dim3(BLK), 0,
                       st, a.mask, dst.mask, grp.n_lim, first);
}
void launch_axpyn(const GroupDev &grp, int64_t n, const uint8_t *colr, LevelDev L, const RegDev *a,
                  const TabDev *nt, const uint64_t *w, int nterms, RegDev dst, uint32_t *ovf, hipStream_t st) {
  AxpyTerms tm{};
  tm.n = nterms;
  size_t lds = 0;
  const bool maps = !getenv_flag_off("CC_NJMAP");
  for (int q = 0; q < nterms; q++) {
    tm.a[q] = a[q];
    tm.w[q] = w[q];
    tm.nt[q] = nt ? nt[q] : TabDev{nullptr, 0, 0};
    tm.jm[q] = nullptr;
    tm.jmw[q] = tm.jns[q] = 0;
    if (maps && tm.nt[q].val &&
        njmap_find(grp.k, dst.s - 2, tm.nt[q].s - 1, dst.C, a[q].C, tm.nt[q].C, &tm.jm[q], &tm.jmw[q], &tm.jns[q]))
      lds += (size_t)tm.jmw[q] * 4;
  }
  if (lds > NJMAP_LDS_MAX) {  // keep the LDS of one launch modest: no maps
    lds = 0;
    for (int q = 0; q < nterms; q++) tm.jm[q] = nullptr, tm.jmw[q] = tm.jns[q] = 0;
  }
  // one colouring, every NodeJoin term with its split map: chunks of rows
  // staged in LDS per wavefront (CC_AXPY_ROWS=0: one slot per lane with gathers)
  bool all_maps = true;
  for (int q = 0; q < nterms; q++) all_maps = all_maps && (!tm.nt[q].val || tm.jmw[q]);
  if (grp.T == 1 && dst.C <= 64 && all_maps && !getenv_flag_off("CC_AXPY_ROWS")) {
    const int R = 64 / dst.C;
    int words = 0;
    for (int q = 0; q < nterms; q++)
      if (tm.nt[q].val) words += R * tm.a[q].C + (grp.dense ? 1 : R) * tm.nt[q].C;
    const int jm_words = (int)(lds / 4);
    words = std::max(1, words);
    const size_t lds2 = (size_t)(jm_words + 1) / 2 * 8 + (size_t)(BLK / 64) * words * 8;
    if (words <= 2048 && lds2 <= 64 * 1024) {
      const dim3 gr(grp.dense ? (unsigned)std::max<int64_t>(1, std::min<int64_t>((grp.n_lim + 3) / 4, 65536)) : 8192u);
      if (grp.dense)
        launch_axpyn_rows_nt<true>(nterms, gr, lds2, st, grp, n, colr, L, tm, dst, ovf, jm_words, words);
      else
        launch_axpyn_rows_nt<false>(nterms, gr, lds2, st, grp, n, colr, L, tm, dst, ovf, jm_words, words);
      return;
    }
  }
  if (grp.dense) {  // the activity word of dst is written by the same pass
    const int gr = (int)std::max<int64_t>(1, std::min<int64_t>((grp.n_lim + 3) / 4, 65536));
    bool jm = true;
    for (int q = 0; q < nterms; q++) jm = jm && (!tm.nt[q].val || tm.jmw[q]);
    if (jm)
      hipLaunchKernelGGL(k_axpyn_dense<true>, dim3(gr), dim3(BLK), lds, st, grp, n, colr, tm, dst, ovf, cur_lut());
    else
      hipLaunchKernelGGL(k_axpyn_dense<false>, dim3(gr), dim3(BLK), lds, st, grp, n, colr, tm, dst, ovf, cur_lut());
    return;
  }
  hipLaunchKernelGGL(k_axpyn, dim3(fgrid(grp, (int64_t)grp.T * dst.C)), dim3(BLK), lds, st, grp, n, colr, L, tm, dst,
                     ovf, cur_lut());
}
void launch_fill_u64v(uint64_t *p, int64_t n, uint64_t x, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_v, dim3((unsigned)std::min<int64_t>((n + BLK - 1) / BLK, 8192)), dim3(BLK), 0, st, p, n,
                     x);
}

bool launch_mroot_terms(const GroupDev &grp, int64_t n, const uint8_t *colr, LevelDev La, LevelDev Lb,
                        const RegDev *a, const TabDev *nt, const uint64_t *wq, int nterms, int Ca, int sa, RegDev b,
                        uint64_t w, AccDev acc, hipStream_t st) {
  if (nterms < 1 || nterms > 4 || Ca > 256 || getenv_flag_off("CC_NJMAP") || getenv_flag_off("CC_FUSE_ROOT"))
    return false;
  AxpyTerms tm{};
  tm.n = nterms;
  size_t lds = 0;
  for (int q = 0; q < nterms; q++) {
    tm.a[q] = a[q];
    tm.w[q] = wq[q];
    tm.nt[q] = nt ? nt[q] : TabDev{nullptr, 0, 0};
    tm.jm[q] = nullptr;
    tm.jmw[q] = tm.jns[q] = 0;
    if (tm.nt[q].val) {  // every NodeJoin term needs its split map
      if (!njmap_find(grp.k, sa - 2, tm.nt[q].s - 1, Ca, a[q].C, tm.nt[q].C, &tm.jm[q], &tm.jmw[q], &tm.jns[q]))
        return false;
      lds += (size_t)tm.jmw[q] * 4;
    } else if (a[q].C != Ca) {
      return false;
    }
  }
  if (lds > NJMAP_LDS_MAX) return false;
  // one colouring: chunks of rows staged in LDS per wavefront (CC_MROOT_ROWS=0: per-slot gathers)
  if (grp.T == 1 && Ca <= 64 && !getenv_flag_off("CC_MROOT_ROWS")) {
    // items per lane: 1 (CC_MROOT_IPL=2: two, more loads in flight but fewer wavefronts per SIMD; slower)
    static const int ipl = [] {
      const char *ev = getenv("CC_MROOT_IPL");
      return ev && *ev == '2' ? 2 : 1;
    }();
    const int R = ipl * 64 / Ca;
    int words = 0;
    for (int q = 0; q < nterms; q++)
      if (tm.nt[q].val) words += R * tm.a[q].C + (grp.dense ? 1 : R) * tm.nt[q].C;
    const int jm_words = (int)(lds / 4);
    words = std::max(1, words);
    const size_t lds2 = (size_t)(jm_words + 1) / 2 * 8 + (size_t)(BLK / 64) * words * 8;
    if (words <= 2048 && lds2 <= 64 * 1024) {
      const dim3 gr(grp.dense ? (unsigned)std::max<int64_t>(1, std::min<int64_t>((grp.n_lim + 3) / 4, 65536)) : 8192u);
      const uint16_t *lut = cur_lut();
      if (grp.dense && ipl == 2)
        launch_mroot_rows_nt<true, 2>(nterms, gr, lds2, st, grp, n, colr, La, Lb, tm, Ca, sa, b, w, acc, lut, jm_words,
                                      words);
      else if (grp.dense)
        launch_mroot_rows_nt<true, 1>(nterms, gr, lds2, st, grp, n, colr, La, Lb, tm, Ca, sa, b, w, acc, lut, jm_words,
                                      words);
      else if (ipl == 2)
        launch_mroot_rows_nt<false, 2>(nterms, gr, lds2, st, grp, n, colr, La, Lb, tm, Ca, sa, b, w, acc, lut,
                                       jm_words, words);
      else
        launch_mroot_rows_nt<false, 1>(nterms, gr, lds2, st, grp, n, colr, La, Lb, tm, Ca, sa, b, w, acc, lut,
                                       jm_words, words);
      return true;
    }
  }
  if (grp.dense) {
    const int gr = (int)std::max<int64_t>(1, std::min<int64_t>((grp.n_lim + 3) / 4, 65536));
    hipLaunchKernelGGL(k_mroot_terms<true>, dim3(gr), dim3(BLK), lds, st, grp, n, colr, La, Lb, tm, Ca, sa, b, w, acc,
                       cur_lut());
  } else {
    hipLaunchKernelGGL(k_mroot_terms<false>, dim3(fgrid(grp, (int64_t)grp.T * Ca)), dim3(BLK), lds, st, grp, n, colr,
                       La, Lb, tm, Ca, sa, b, w, acc, cur_lut());
  }
  return true;
}

void launch_mroot(const GroupDev &grp, int64_t n, const uint8_t *colr, LevelDev La, LevelDev Lb, RegDev a, RegDev b,
                  uint64_t w, AccDev acc, hipStream_t st) {
  hipLaunchKernelGGL(k_mroot, dim3(fgrid(grp, 1)), dim3(BLK), 0, st, grp, n, colr, La, Lb, a, b, w,
                     acc, cur_lut());
}

void launch_munary(const GroupDev &grp, int64_t n, const uint8_t *colr, LevelDev La, LevelDev Lb, RegDev a,
                   RegDev b, uint64_t w, int at_u, uint64_t *out, int s_out, int C_out, uint32_t *ovf,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_munary, dim3(fgrid(grp, (int64_t)grp.T * C_out)), dim3(BLK), 0, st, grp, n, colr, La, Lb, a,
                     b, w, at_u, out, s_out, C_out, ovf, cur_lut());
}

void launch_medge(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev La, LevelDev Lb, RegDev a,
                  RegDev b, TabDev etab, int e_src_first, int out_first_is_x, uint64_t w, uint64_t *out, int s_out,
                  int C_out, uint32_t *ovf, hipStream_t st) {
  // vertex-major (CC_MEDGE_V=0: one thread per (entry, trial, slot), each scanning the neighbour list)
  if ((int64_t)grp.T * C_out <= 64 && !getenv_flag_off("CC_MEDGE_V")) {
    const int gr = (int)std::max<int64_t>(1, std::min<int64_t>((grp.dense ? grp.n_lim : 65536) / 4 + 1, 65536));
    if (grp.dense)
      hipLaunchKernelGGL(k_medge_v<true>, dim3(gr), dim3(BLK), 0, st, g, grp, colr, La, Lb, a, b, etab, e_src_first,
                         out_first_is_x, w, out, s_out, C_out, ovf, cur_lut());
    else
      hipLaunchKernelGGL(k_medge_v<false>, dim3(gr), dim3(BLK), 0, st, g, grp, colr, La, Lb, a, b, etab, e_src_first,
                         out_first_is_x, w, out, s_out, C_out, ovf, cur_lut());
    return;
  }
  hipLaunchKernelGGL(k_medge, dim3(fgrid(grp, (int64_t)grp.T * C_out)), dim3(BLK), 0, st, g, grp, colr, La, Lb, a, b,
                     etab, e_src_first, out_first_is_x, w, out, s_out, C_out, ovf, cur_lut());
}

void launch_mpair(const GroupDev &grp, int64_t n, const uint8_t *colr, RegDev a, RegDev b, uint64_t w, RegDev stage,
                  int32_t *keys, uint64_t *vals, uint64_t cap, unsigned long long *cnt, uint32_t *ovf,
                  hipStream_t st) {
  launch_fill_u64(stage.mask, grp.n_lim, st);
  hipLaunchKernelGGL(k_mpair, dim3(fgrid(grp, (int64_t)grp.T * stage.C)), dim3(BLK), 0, st, grp, n, colr, a, b, w,
                     stage, ovf, cur_lut());
  hipLaunchKernelGGL(k_pair_emit, dim3(fgrid(grp, 1)), dim3(BLK), 0, st, grp, stage, keys, vals, cap, cnt);
}

void launch_pair_gather(const int64_t *idx, int64_t m2, const uint64_t *vals, int64_t per, uint64_t *tab,
                        hipStream_t st) {
  const int64_t N = m2 * per;
  if (N <= 0) return;
  hipLaunchKernelGGL(k_pair_gather, dim3((unsigned)std::min<int64_t>((N + BLK - 1) / BLK, 8192)), dim3(BLK), 0, st,
                     idx, m2, vals, per, tab);
}

void launch_medge_t(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, const int32_t *lowcnt,
                    int max_low, TabDev ntab, LevelDev Lb, RegDev b, TabDev etab, int e_src_first,
                    int out_first_is_u, uint64_t w, uint64_t *out, int s_out, int C_out, uint32_t *ovf,
                    hipStream_t st) {
  int64_t N = (int64_t)grp.B * max_low * grp.T * C_out;
  int gr = (int)std::max<int64_t>(1, std::min<int64_t>((N + BLK - 1) / BLK, 65536));
  hipLaunchKernelGGL(k_medge_t, dim3(gr), dim3(BLK), 0, st, g, grp, colr, lowcnt, max_low, ntab, Lb, b, etab,
                     e_src_first, out_first_is_u, w, out, s_out, C_out, ovf, cur_lut());
}

}  // namespace cc
