// Grouped path: B sources (<= 64) and T colourings per launch.
//
// The frontier of a cycle program is organised by path length: the entries of
// depth d are the (vertex, source) pairs that a high-starting walk of d edges
// reaches (every register of that depth has a row per entry, whatever its
// annotations, since reachability does not depend on colours or tables).
// Dense groups -- the sources with the widest reach -- keep a row for every
// (v, b) with v < n_lim, rows of unreachable pairs holding zeros.  Sparse groups
// list their entries: a level is built by marking (plain byte stores, no
// atomics) and a deterministic compaction pass that numbers the marks in
// vertex order.
//
// EdgeJoin is a pull: a team of lanes owns one output entry (w, b) and strides
// over w's neighbours below u_b; each lane reads the whole row of its
// neighbour's entry and adds every input slot to the output slot it becomes
// (data edge: the signature gains chi(v) -- Section 4.3, Procedure 1) or to the
// output slots of all its products with the edge table (annotated edge:
// EdgeJoin of Section 4.4), accumulating in LDS.  NodeJoin, AXPY and the
// merges are flat: one thread per output slot.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "slot_math.h"

namespace cc {

namespace {

using namespace dev;

constexpr int CH = 8192;  // flags per compaction chunk (32 per thread)

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
__device__ __forceinline__ int64_t entry_of(const GroupDev &g, const LevelDev &L, int64_t v, int b) {
  if (g.dense) return v < g.n_lim ? v * g.B + b : -1;
  return L.idx[v * g.B + b];
}
// row of register r for (v, b), or -1 when it has none (sparse) or is known
// to be zero (dense: its activity bit is clear)
__device__ __forceinline__ int64_t row_of(const GroupDev &g, const LevelDev &L, const RegDev &r, int64_t v, int b) {
  if (g.dense) return (v < g.n_lim && ((r.mask[v] >> b) & 1ull)) ? v * g.B + b : -1;
  return L.idx[v * g.B + b];
}
__device__ __forceinline__ bool live(const GroupDev &g, const RegDev &r, int64_t v, int b) {
  return !g.dense || ((r.mask[v] >> b) & 1ull);
}

// ------------------------------------------------------------------ levels (sparse groups)
// depth 1: the lower neighbours of each source
__global__ void k_mark_init(GraphDev g, GroupDev grp, const int32_t *lowcnt, int max_low, LevelDev L) {
  const int64_t N = (int64_t)grp.B * max_low;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / max_low), j = (int)(i - (int64_t)b * max_low);
    const int64_t u = grp.src[b];
    if (j >= lowcnt[u]) continue;
    const int64_t x = g.col[g.rp[u] + j];
    L.flag[x * grp.B + b] = 1;
    L.vflag[x] = 1;
  }
}

// depth d+1 from depth d: every lower neighbour w < u_b of an entry (v, b)
__global__ void k_mark_next(GraphDev g, GroupDev grp, LevelDev Lin, LevelDev Lout) {
  constexpr int TEAM = 16;
  const int teams = BLK / TEAM, team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int64_t N = *Lin.cnt;
  for (int64_t e = (int64_t)blockIdx.x * teams + team; e < N; e += (int64_t)gridDim.x * teams) {
    const int64_t x = Lin.list[e];
    const int64_t v = x >> 6;
    const int b = (int)(x & 63);
    const int64_t u = grp.src[b];
    for (int64_t ee = g.rp[v] + lane; ee < g.rp[v + 1]; ee += TEAM) {
      const int64_t w = g.col[ee];
      if (w >= u) break;
      Lout.flag[w * grp.B + b] = 1;
      Lout.vflag[w] = 1;
    }
  }
}

// Compaction walks vertices in chunks of CH (32 per thread): only vertices
// with their per-vertex mark set have their B source marks read.
__device__ __forceinline__ uint32_t count_marks(const uint8_t *flag, int64_t v, int B) {
  uint32_t c = 0;
  for (int b = 0; b < B; b++) c += flag[v * B + b] != 0;
  return c;
}

// count marks per chunk
__global__ void k_cmp_count(const uint8_t *flag, const uint8_t *vflag, int64_t nv, int B, uint32_t *bcnt) {
  __shared__ uint32_t s[BLK];
  const int64_t lo = (int64_t)blockIdx.x * CH + (int64_t)threadIdx.x * (CH / BLK);
  uint32_t c = 0;
  for (int i = 0; i < CH / BLK; i++)
    if (lo + i < nv && vflag[lo + i]) c += count_marks(flag, lo + i, B);
  s[threadIdx.x] = c;
  __syncthreads();
  for (int o = BLK / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bcnt[blockIdx.x] = s[0];
}

// exclusive scan of the chunk counts (one workgroup); total into *cnt
__global__ void k_cmp_scan(uint32_t *bcnt, int nb, uint32_t *cnt) {
  __shared__ uint32_t s[BLK + 1];
  const int per = (nb + BLK - 1) / BLK;
  const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, lo + per);
  uint32_t sum = 0;
  for (int i = lo; i < hi; i++) sum += bcnt[i];
  s[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int i = 0; i < BLK; i++) {
      uint32_t x = s[i];
      s[i] = run;
      run += x;
    }
    s[BLK] = run;
    *cnt = run;
  }
  __syncthreads();
  uint32_t run = s[threadIdx.x];
  for (int i = lo; i < hi; i++) {
    uint32_t x = bcnt[i];
    bcnt[i] = run;
    run += x;
  }
}

// number the marks in (vertex, source) order: idx and list, clearing the marks
__global__ void k_cmp_emit(uint8_t *flag, uint8_t *vflag, int64_t nv, const uint32_t *boff, int B, int32_t *idx,
                           int64_t *list) {
  __shared__ uint32_t s[BLK];
  const int per = CH / BLK;
  const int64_t lo = (int64_t)blockIdx.x * CH + (int64_t)threadIdx.x * per;
  uint32_t c = 0;
  for (int i = 0; i < per; i++)
    if (lo + i < nv && vflag[lo + i]) c += count_marks(flag, lo + i, B);
  s[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int i = 0; i < BLK; i++) {
      uint32_t x = s[i];
      s[i] = run;
      run += x;
    }
  }
  __syncthreads();
  uint32_t id = boff[blockIdx.x] + s[threadIdx.x];
  for (int i = 0; i < per; i++) {
    const int64_t v = lo + i;
    if (v >= nv || !vflag[v]) continue;
    vflag[v] = 0;
    for (int b = 0; b < B; b++) {
      const int64_t f = v * B + b;
      if (!flag[f]) continue;
      flag[f] = 0;
      idx[f] = (int32_t)id;
      list[id] = v * 64 + b;
      id++;
    }
  }
}

__global__ void k_level_reset(GroupDev grp, LevelDev L) {
  const int64_t N = *L.cnt;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = L.list[e];
    L.idx[(x >> 6) * grp.B + (x & 63)] = -1;
  }
}
__global__ void k_zero_cnt(uint32_t *c) { *c = 0; }

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
  uint64_t ofm = 0;
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
  }
  flag_trials(ovf, ofm);
}

// ------------------------------------------------------------------ EdgeJoin
// dst[(w,b)][R'] = sum over v in N(w), v < u_b, (v,b) an entry of the lower
// level, of sum over splits R' \ {chi v} = R + Re of a[(v,b)][R] * E(v,w)[Re].
template <int TEAM>
__global__ __launch_bounds__(BLK) void k_ej(GraphDev g, GroupDev grp, const uint8_t *colr, LevelDev Lin, LevelDev Lout,
                                            RegDev a, RegDev dst, TabDev et, int e_src_first, uint32_t *ovf,
                                            const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint32_t s_min[256];   // unranked input slots (data edges)
  __shared__ int s_nz[BLK / TEAM];
  extern __shared__ uint64_t s_acc[];
  load_rank(s_rank, lut);
  constexpr int teams = BLK / TEAM;
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int T = grp.T, C = dst.C, Ca = a.C;
  const int TC = T * C;
  const int ra = a.s - 2;
  for (int c = threadIdx.x; c < Ca && c < 256; c += BLK) s_min[c] = unrank(lut, ra, c);
  // accumulators: low and high 32-bit halves of every addend, summed apart
  // (non-returning LDS adds; the halves cannot overflow), joined at the end
  uint64_t *acc = s_acc + (int64_t)team * 2 * TC;
  const int64_t N = nentries(grp, Lout);
  uint64_t ofm = 0;
  for (int64_t e0 = (int64_t)blockIdx.x * teams; e0 < N; e0 += (int64_t)gridDim.x * teams) {
    const int64_t e = e0 + team;
    const bool valid = e < N;
    __syncthreads();
    for (int q = lane; q < 2 * TC; q += TEAM) acc[q] = 0;
    if (lane == 0) s_nz[team] = 0;
    __syncthreads();
    int64_t w = 0;
    int b = 0;
    if (valid) entry_vb(grp, Lout, e, w, b);
    const int64_t u = valid ? grp.src[b] : 0;
    if (valid && w < u) {
      for (int t = 0; t < T; t++) {
        const int cu = colr[(int64_t)t * g.n + u], cw = colr[(int64_t)t * g.n + w];
        if (cu == cw) continue;
        uint64_t *at_acc = acc + 2 * t * C;
        for (int64_t ee = g.rp[w] + lane; ee < g.rp[w + 1]; ee += TEAM) {
          const int64_t v = g.col[ee];
          if (v >= u) break;
          const int64_t id = row_of(grp, Lin, a, v, b);
          if (id < 0) continue;
          const int cv = colr[(int64_t)t * g.n + v];
          if (cv == cu || cv == cw) continue;
          const uint64_t *at = a.val + (id * T + t) * Ca;
          if (!et.val) {
            for (int c0 = 0; c0 < Ca; c0 += 4) {
              uint64_t x[4];
#pragma unroll
              for (int q = 0; q < 4; q++) x[q] = c0 + q < Ca ? at[c0 + q] : 0;
#pragma unroll
              for (int q = 0; q < 4; q++) {
                if (!x[q]) continue;
                const uint32_t R = spread2(s_min[c0 + q], cu, cv);
                if ((R >> cw) & 1u) continue;
                const int o = s_rank[squeeze2(R | (1u << cv), cu, cw)];
                atomicAdd((unsigned long long *)&at_acc[2 * o], (unsigned long long)(x[q] & 0xffffffffull));
                atomicAdd((unsigned long long *)&at_acc[2 * o + 1], (unsigned long long)(x[q] >> 32));
              }
            }
          } else {
            const int64_t tslot = e_src_first ? g.rev[ee] : ee;
            const uint64_t *er = et.val + (tslot * T + t) * et.C;
            for (int co = 0; co < C; co++) {
              const uint32_t Rp = spread2(unrank(lut, dst.s - 2, co), cu, cw);
              if (!((Rp >> cv) & 1u)) continue;
              const uint32_t R = Rp & ~(1u << cv);
              uint64_t sum = 0;
              bool of = false;
              uint32_t s1 = R;
              for (;;) {
                if (__popc(s1) == ra) {
                  uint64_t xa = at[s_rank[squeeze2(s1, cu, cv)]];
                  if (xa) {
                    uint64_t y = er[s_rank[squeeze2(R & ~s1, cv, cw)]];
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
        }
      }
    }
    __syncthreads();
    if (valid) {
      uint64_t *drow = dst.val + e * (int64_t)TC;
      bool nz = false;
      for (int q = lane; q < TC; q += TEAM) {
        const uint64_t lo = acc[2 * q], hi = acc[2 * q + 1];
        // value = hi * 2^32 + lo; both halves are sums of 32-bit parts
        const uint64_t hs = hi + (lo >> 32);
        if (hs >> 32) ofm |= 1ull << (q / C);
        const uint64_t v = (hs << 32) | (lo & 0xffffffffull);
        drow[q] = v;
        nz |= v != 0;
      }
      if (nz) s_nz[team] = 1;
    }
    if (grp.dense) {
      __syncthreads();
      if (valid && lane == 0) {
        if (s_nz[team]) atomicOr((unsigned long long *)&dst.mask[w], 1ull << b);
        else atomicAnd((unsigned long long *)&dst.mask[w], ~(1ull << b));
      }
    }
  }
  flag_trials(ovf, ofm);
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
  uint64_t ofm = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t e = i / per;
    const int r = (int)(i - e * per), t = r / C, c = r - t * C;
    int64_t v;
    int b;
    entry_vb(grp, L, e, v, b);
    if (!live(grp, a, v, b)) continue;
    const int64_t u = grp.src[b];
    uint64_t acc = 0;
    bool of = false;
    if (v < u) {
      const int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
      if (cu != cv) {
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
}

// ------------------------------------------------------------------ AXPY
// dst = (first ? 0 : dst) + w * a, slot by slot (same level, same rows)
__global__ __launch_bounds__(BLK) void k_axpy(GroupDev grp, LevelDev L, RegDev a, RegDev dst, uint64_t w, int first,
                                              uint32_t *ovf) {
  const int T = grp.T, C = dst.C;
  const int64_t N = nentries(grp, L) * T * C;
  uint64_t ofm = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    bool of = false;
    bool on = true;
    if (grp.dense) {
      const int64_t row = i / ((int64_t)T * C);
      on = (a.mask[row / grp.B] >> (row % grp.B)) & 1ull;
      if (!on && !first) continue;
    }
    uint64_t y = first ? 0 : dst.val[i];
    if (on) add_ck(y, mul_ck(w, a.val[i], of), of);
    dst.val[i] = y;
    if (of) ofm |= 1ull << ((i / C) % T);
  }
  flag_trials(ovf, ofm);
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

// ------------------------------------------------------------------ root merge
// count[t] += w * sum over entries (v, b) of both levels of
//             sum over R of a[(v,b)][R] * b[(v,b)][K \ {chi u, chi v} \ R]
__global__ __launch_bounds__(BLK) void k_mroot(GroupDev grp, int64_t n, const uint8_t *colr, LevelDev La,
                                               LevelDev Lb, RegDev a, RegDev bb, uint64_t w, AccDev acc,
                                               const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint64_t s_acc[2 * 64];
  for (int i = threadIdx.x; i < 2 * 64; i += blockDim.x) s_acc[i] = 0;
  load_rank(s_rank, lut);
  const int T = grp.T, Ca = a.C, Cb = bb.C, k = grp.k;
  const uint32_t Kmask = (1u << k) - 1u;
  const int64_t per = (int64_t)T * Ca;
  const int64_t N = nentries(grp, La) * per;
  uint64_t lo0 = 0, hi0 = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t e = i / per;
    if (grp.dense && !((a.mask[e / grp.B] >> (e % grp.B)) & 1ull)) continue;
    const uint64_t x = a.val[i];
    if (!x) continue;
    const int r = (int)(i - e * per), t = r / Ca, c = r - t * Ca;
    int64_t v;
    int b;
    entry_vb(grp, La, e, v, b);
    if (!live(grp, a, v, b)) continue;
    const int64_t eb = row_of(grp, Lb, bb, v, b);
    if (eb < 0) continue;
    const int64_t u = grp.src[b];
    const int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
    if (cu == cv) continue;
    const uint32_t R1 = spread2(unrank(lut, a.s - 2, c), cu, cv);
    const uint32_t R2 = Kmask & ~R1 & ~(1u << cu) & ~(1u << cv);
    const uint64_t y = bb.val[(eb * T + t) * Cb + s_rank[squeeze2(R2, cu, cv)]];
    if (!y) continue;
    uint64_t pl = x * y, ph = __umul64hi(x, y);
    if (w != 1) {
      uint64_t l2 = pl * w, c2 = __umul64hi(pl, w);
      uint64_t h2 = ph * w + c2;
      if (__umul64hi(ph, w) != 0 || h2 < c2) atomicOr(&acc.ovf[t], 1u);
      pl = l2;
      ph = h2;
    }
    if (acc.per_src) atomic_add128(&acc.per_src[2 * (u * T + t)], pl, ph);
    if (T == 1) {
      uint64_t s = lo0 + pl;
      hi0 += ph + (s < pl ? 1u : 0u);
      lo0 = s;
    } else {
      atomic_add128(&s_acc[2 * t], pl, ph);
    }
  }
  if (T == 1 && (lo0 | hi0)) atomic_add128(&s_acc[0], lo0, hi0);
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += blockDim.x)
    if (s_acc[2 * t] | s_acc[2 * t + 1]) atomic_add128(&acc.sum[2 * t], s_acc[2 * t], s_acc[2 * t + 1]);
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
  uint64_t ofm = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t e = i / per;
    const int r = (int)(i - e * per), t = r / C_out, c = r - t * C_out;
    int64_t v;
    int b;
    entry_vb(grp, La, e, v, b);
    const int64_t u = grp.src[b];
    if (v >= u || !live(grp, a, v, b)) continue;
    const int64_t eb = row_of(grp, Lb, bb, v, b);
    if (eb < 0) continue;
    const int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
    if (cu == cv) continue;
    const int ckey = at_u ? cu : cv, coth = at_u ? cv : cu;
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
    if (s) atomic_add_ck(&out[((at_u ? u : v) * T + t) * C_out + c], mul_ck(s, w, of), of);
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
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
  uint64_t ofm = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < N; i += (int64_t)gridDim.x * BLK) {
    const int64_t e = i / per;
    const int r = (int)(i - e * per), t = r / C_out, c = r - t * C_out;
    int64_t x;
    int b;
    entry_vb(grp, La, e, x, b);
    const int64_t u = grp.src[b];
    if (x >= u || !live(grp, a, x, b)) continue;
    const int cu = colr[(int64_t)t * g.n + u], cx = colr[(int64_t)t * g.n + x];
    if (cu == cx) continue;
    const uint64_t *ar = a.val + (e * T + t) * Ca;
    bool of = false;
    for (int64_t ee = g.rp[x]; ee < g.rp[x + 1]; ee++) {
      const int64_t y = g.col[ee];
      if (y >= u) break;
      const int64_t eb = row_of(grp, Lb, bb, y, b);
      if (eb < 0) continue;
      const int cy = colr[(int64_t)t * g.n + y];
      if (cy == cx || cy == cu) continue;
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
      }
    }
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
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
  uint64_t ofm = 0;
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
    }
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
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

void launch_level_init(const GraphDev &g, const GroupDev &grp, const int32_t *lowcnt, int max_low, LevelDev L,
                       hipStream_t st) {
  int64_t N = (int64_t)grp.B * max_low;
  hipLaunchKernelGGL(k_mark_init, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((N + BLK - 1) / BLK, 4096))),
                     dim3(BLK), 0, st, g, grp, lowcnt, max_low, L);
}

static void compact(const GroupDev &grp, LevelDev L, hipStream_t st) {
  const int64_t nf = grp.n_lim * (int64_t)grp.B;
  const int64_t nv = grp.n_lim;
  const int nb = (int)((nv + CH - 1) / CH);
  // the chunk counts live past the end of the list (which holds at most nf entries)
  uint32_t *bcnt = (uint32_t *)(L.list + nf);
  hipLaunchKernelGGL(k_cmp_count, dim3(nb), dim3(BLK), 0, st, L.flag, L.vflag, nv, grp.B, bcnt);
  hipLaunchKernelGGL(k_cmp_scan, dim3(1), dim3(BLK), 0, st, bcnt, nb, L.cnt);
  hipLaunchKernelGGL(k_cmp_emit, dim3(nb), dim3(BLK), 0, st, L.flag, L.vflag, nv, bcnt, grp.B, L.idx, L.list);
}

void launch_level_next(const GraphDev &g, const GroupDev &grp, LevelDev Lin, LevelDev Lout, hipStream_t st) {
  hipLaunchKernelGGL(k_mark_next, dim3(8192), dim3(BLK), 0, st, g, grp, Lin, Lout);
  compact(grp, Lout, st);
}

void launch_level_compact(const GroupDev &grp, LevelDev L, hipStream_t st) { compact(grp, L, st); }

void launch_level_reset(const GroupDev &grp, LevelDev L, hipStream_t st) {
  hipLaunchKernelGGL(k_level_reset, dim3(4096), dim3(BLK), 0, st, grp, L);
  hipLaunchKernelGGL(k_zero_cnt, dim3(1), dim3(1), 0, st, L.cnt);
}

void launch_init(const GraphDev &g, const GroupDev &grp, const int32_t *lowcnt, int max_low, const uint8_t *colr,
                 LevelDev L, RegDev dst, TabDev etab, int e_src_first, TabDev ntab, uint32_t *ovf, hipStream_t st) {
  int64_t N = (int64_t)grp.B * max_low * grp.T * dst.C;
  int gr = (int)std::max<int64_t>(1, std::min<int64_t>((N + BLK - 1) / BLK, 65536));
  hipLaunchKernelGGL(k_init, dim3(gr), dim3(BLK), 0, st, g, grp, lowcnt, max_low, colr, L, dst, etab, e_src_first,
                     ntab, ovf, cur_lut());
}

void launch_ej(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev Lin, LevelDev Lout, RegDev a,
               RegDev dst, TabDev etab, int e_src_first, uint32_t *ovf, hipStream_t st) {
  const int TC = grp.T * dst.C;
  const int gr = grp.dense ? (int)std::max<int64_t>(1, std::min<int64_t>(grp.n_lim * grp.B / 4, 65536)) : 8192;
  const size_t row = (size_t)2 * TC * 8;  // two accumulator words per slot
  if (16 * row <= 48 * 1024)
    hipLaunchKernelGGL(k_ej<16>, dim3(gr), dim3(BLK), 16 * row, st, g, grp, colr, Lin, Lout, a, dst, etab,
                       e_src_first, ovf, cur_lut());
  else if (4 * row <= 48 * 1024)
    hipLaunchKernelGGL(k_ej<64>, dim3(gr), dim3(BLK), 4 * row, st, g, grp, colr, Lin, Lout, a, dst, etab,
                       e_src_first, ovf, cur_lut());
  else
    hipLaunchKernelGGL(k_ej<256>, dim3(gr), dim3(BLK), row, st, g, grp, colr, Lin, Lout, a, dst, etab,
                       e_src_first, ovf, cur_lut());
}

void launch_nj(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, LevelDev L, RegDev a, RegDev dst,
               TabDev ntab, uint32_t *ovf, hipStream_t st) {
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
void launch_fill_u64v(uint64_t *p, int64_t n, uint64_t x, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_v, dim3((unsigned)std::min<int64_t>((n + BLK - 1) / BLK, 8192)), dim3(BLK), 0, st, p, n,
                     x);
}

void launch_mroot(const GroupDev &grp, int64_t n, const uint8_t *colr, LevelDev La, LevelDev Lb, RegDev a, RegDev b,
                  uint64_t w, AccDev acc, hipStream_t st) {
  hipLaunchKernelGGL(k_mroot, dim3(fgrid(grp, (int64_t)grp.T * a.C)), dim3(BLK), 0, st, grp, n, colr, La, Lb, a, b, w,
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
  hipLaunchKernelGGL(k_medge, dim3(fgrid(grp, (int64_t)grp.T * C_out)), dim3(BLK), 0, st, g, grp, colr, La, Lb, a, b,
                     etab, e_src_first, out_first_is_x, w, out, s_out, C_out, ovf, cur_lut());
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
