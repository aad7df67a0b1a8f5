// Device kernels for the degree-based colour-coding dynamic program on gfx950.
//
// Signatures (Section 4.2: the set of colours used by a partial match) are
// k-bit masks.  A table keyed by vertices whose colours are fixed stores only
// the remaining colours: for a path key (u, v) of signature size s the slots
// are the (s-2)-subsets of K \ {chi(u), chi(v)}; for a unary key x of size s,
// the (s-1)-subsets of K \ {chi(x)}; for an edge key (x, y), the (s-2)-subsets
// of K \ {chi(x), chi(y)}.  A subset is stored at its colex rank after the
// excluded colour bits are squeezed out.
//
// Every kernel is output-stationary: a thread owns one output slot (trial,
// colour subset) of one output key and sums, over the joined entries, the
// products over all ways to split its subset between the operands (the
// disjoint-signature condition of NodeJoin / EdgeJoin / the cycle merge,
// Section 4.4).  Sums and products are checked: a table entry that leaves 64
// bits raises the trial's overflow flag instead of wrapping.
//
// Frontier domains.  A group processes B sources (<= 64) and T colourings.
// In dense mode the domain of a register is every (v, b) with v < n_lim and
// its activity byte says whether (v, b) holds an entry; in sparse mode the
// register also keeps a list of its active (v, b) pairs and kernels walk the
// list.  Either way each entry's C slots for T trials are contiguous.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "kernels.h"
#include "slot_math.h"

namespace cc {

namespace {

using namespace dev;

// a zero word: gathers of inactive lanes read it instead of branching
__device__ uint64_t g_zero[8];

// ------------------------------------------------------------------ colours
__global__ void k_colour(const int32_t *orig, int64_t n, int k, uint64_t seed, int t0, int T, uint8_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * T) return;
  int t = (int)(i / n);
  int64_t r = i - (int64_t)t * n;
  uint64_t key = mix64(seed + (uint64_t)(t0 + t));
  uint64_t h = mix64(key ^ (uint64_t)(uint32_t)orig[r]);
  out[i] = (uint8_t)(((h >> 32) * (uint64_t)k) >> 32);
}

__global__ void k_permute(const uint8_t *by_orig, const int32_t *orig, int64_t n, int T, uint8_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * T) return;
  int t = (int)(i / n);
  int64_t r = i - (int64_t)t * n;
  out[i] = by_orig[(int64_t)t * n + orig[r]];
}

__global__ void k_fill_u8(uint8_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}
__global__ void k_fill_u64(uint64_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}


// ------------------------------------------------------------------ domains
// Vertex domain of a register: every v < n_lim (dense) or its vertex list.
__device__ __forceinline__ int64_t vdomain(const GroupDev &g, const RegDev &r) {
  return g.dense ? g.n_lim : (int64_t)(*r.vcnt);
}
__device__ __forceinline__ int64_t vertex_at(const GroupDev &g, const RegDev &r, int64_t i) {
  return g.dense ? i : (int64_t)r.vlist[i];
}
// list vertex v in a sparse register (once)
__device__ __forceinline__ void list_vertex(RegDev &r, int64_t v) {
  if (set_act(r.vmark, v)) {
    uint32_t pos = atomicAdd(r.vcnt, 1u);
    r.vlist[pos] = (int32_t)v;
  }
}

// Per-thread work items over (source b, trial t, slot c) of one vertex.
template <int NI>
struct Items {
  int b[NI], t[NI], c[NI];
  bool on[NI];
  __device__ __forceinline__ void init(int B, int T, int C) {
#pragma unroll
    for (int i = 0; i < NI; i++) {
      int it = threadIdx.x + i * BLK;
      on[i] = it < B * T * C;
      int p = on[i] ? it / C : 0;
      c[i] = on[i] ? it - p * C : 0;
      b[i] = p / T;
      t[i] = p - b[i] * T;
    }
  }
};

__global__ void k_clear_list(uint8_t *act, uint8_t *vmark, const int32_t *vlist, uint32_t *vcnt, int B) {
  int64_t N = *vcnt;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N * B; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t v = vlist[i / B];
    int b = (int)(i % B);
    act[v * B + b] = 0;
    if (b == 0) vmark[v] = 0;
  }
}
__global__ void k_reset_cnt(uint32_t *cnt) { *cnt = 0; }

// ------------------------------------------------------------------ INIT
// dst[x][b] for x in the lower prefix of u_b's row:
//   value over rest R (subset of K \ {chi u, chi x}, size s-2) =
//   sum over splits R = Ra + Re of  A_h[u][Ra] * E(u,x)[Re]
// (A_h absent: identity {chi u}; E absent: the data edge, {chi u, chi x} -> 1).
__global__ void k_init(GraphDev g, GroupDev grp, const int32_t *lowcnt, int max_low, const uint8_t *colr,
                       RegDev dst, TabDev et, int e_src_first, TabDev nt, uint32_t *ovf, const uint16_t *lut,
                       int P) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int epb = blockDim.x / P, lane = threadIdx.x % P, sub = threadIdx.x / P;
  const int C = dst.C, T = grp.T, B = grp.B;
  const int items = T * C;
  const int64_t N = (int64_t)B * max_low;
  const int sa = nt.val ? nt.s : 1;
  for (int64_t e0 = (int64_t)blockIdx.x * epb; e0 < N; e0 += (int64_t)gridDim.x * epb) {
    int64_t en = e0 + sub;
    if (en >= N) continue;
    int b = (int)(en / max_low);
    int j = (int)(en - (int64_t)b * max_low);
    int64_t u = grp.src[b];
    if (j >= lowcnt[u]) continue;
    int64_t es = g.rp[u] + j;
    int64_t x = g.col[es];
    int64_t ent = x * B + b;
    if (lane == 0) {
      dst.act[ent] = 1;
      if (!grp.dense) list_vertex(dst, x);
    }
    int64_t tslot = e_src_first ? es : g.rev[es];
    for (int it = lane; it < items; it += P) {
      int t = it / C, c = it - t * C;
      int cu = colr[(int64_t)t * g.n + u], cx = colr[(int64_t)t * g.n + x];
      uint64_t acc = 0;
      bool of = false;
      if (cu != cx) {
        uint32_t R = spread2(unrank(lut, dst.s - 2, c), cu, cx);
        uint32_t sub_ = R;
        for (;;) {
          if (__popc(sub_) == sa - 1) {
            uint32_t Re = R & ~sub_;
            uint64_t va = nt.val ? nt.val[((int64_t)u * T + t) * nt.C + s_rank[squeeze1(sub_, cu)]] : 1;
            uint64_t ve = et.val ? et.val[(tslot * T + t) * et.C + s_rank[squeeze2(Re, cu, cx)]] : (Re ? 0 : 1);
            if (va && ve) add_ck(acc, mul_ck(va, ve, of), of);
          }
          if (sub_ == 0) break;
          sub_ = (sub_ - 1) & R;
        }
      }
      dst.val[(ent * T + t) * C + c] = acc;
      if (of) atomicOr(&ovf[t], 1u);
    }
  }
}

// ------------------------------------------------------------------ MARK (sparse EdgeJoin, structure)
// For every listed vertex v of a and every neighbour w < n_lim: sources b
// active at v with w < u_b become active at w; w is listed in dst.
__global__ void k_mark(GraphDev g, GroupDev grp, RegDev a, RegDev dst) {
  __shared__ uint8_t s_m[64];
  const int B = grp.B;
  const int64_t N = *a.vcnt;
  for (int64_t vi = blockIdx.x; vi < N; vi += gridDim.x) {
    int64_t v = a.vlist[vi];
    __syncthreads();
    if (threadIdx.x < B) s_m[threadIdx.x] = a.act[v * B + threadIdx.x];
    __syncthreads();
    uint64_t mask = 0;
    for (int b = 0; b < B; b++)
      if (s_m[b]) mask |= 1ull << b;
    for (int64_t e = g.rp[v] + threadIdx.x; e < g.rp[v + 1]; e += blockDim.x) {
      int64_t w = g.col[e];
      if (w >= grp.n_lim) break;
      // sources are in decreasing rank: w < u_b holds for b below a cut
      int cut = 0;
      while (cut < B && grp.src[cut] > w) cut++;
      uint64_t mw = mask & (cut >= 64 ? ~0ull : ((1ull << cut) - 1ull));
      if (!mw) continue;
      while (mw) {
        int b = __ffsll((unsigned long long)mw) - 1;
        mw &= mw - 1;
        dst.act[w * B + b] = 1;
      }
      list_vertex(dst, w);
    }
  }
}

// ------------------------------------------------------------------ EdgeJoin (pull, vertex-major)
// dst[w][b][R'] = sum over v in N(w), v < u_b, (v,b) active in a, of
//                 sum over splits R' \ {chi v} = R + Re of a[v][b][R] * E(v,w)[Re].
// One workgroup per output vertex w; lanes span every (b, t, slot) of the
// group; each chunk of 64 neighbours is staged in LDS with its colours and
// activity so that a neighbour's whole [b][t][slot] block is read together.
template <int NI>
__global__ __launch_bounds__(BLK) void k_ej(GraphDev g, GroupDev grp, const uint8_t *colr, RegDev a, RegDev dst,
                                            TabDev et, int e_src_first, uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ int32_t s_v[64];
  __shared__ int64_t s_e[64];
  __shared__ uint8_t s_c[64 * 64];
  __shared__ uint8_t s_a[64 * 64];
  __shared__ uint8_t s_any[64];
  load_rank(s_rank, lut);
  const int B = grp.B, T = grp.T, C = dst.C, Ca = a.C;
  const int ra = a.s - 2;
  Items<NI> I;
  I.init(B, T, C);
  int cu[NI];
  int64_t ub[NI];
#pragma unroll
  for (int i = 0; i < NI; i++) {
    ub[i] = grp.src[I.b[i]];
    cu[i] = colr[(int64_t)I.t[i] * g.n + ub[i]];
  }
  const int64_t N = vdomain(grp, dst);
  for (int64_t wi = blockIdx.x; wi < N; wi += gridDim.x) {
    const int64_t w = vertex_at(grp, dst, wi);
    __syncthreads();
    if (threadIdx.x < 64) s_any[threadIdx.x] = 0;
    uint64_t acc[NI];
    uint32_t Rp[NI];
    bool ok[NI];
    int cw[NI];
#pragma unroll
    for (int i = 0; i < NI; i++) {
      acc[i] = 0;
      cw[i] = colr[(int64_t)I.t[i] * g.n + w];
      ok[i] = I.on[i] && w < ub[i] && cw[i] != cu[i];
      Rp[i] = ok[i] ? spread2(unrank(lut, dst.s - 2, I.c[i]), cu[i], cw[i]) : 0u;
    }
    uint64_t ofm = 0;
    const int64_t rs = g.rp[w], re = g.rp[w + 1];
    for (int64_t e0 = rs; e0 < re; e0 += 64) {
      __syncthreads();
      const int cnt = (int)min((int64_t)64, re - e0);
      if (threadIdx.x < cnt) {
        int64_t v = g.col[e0 + threadIdx.x];
        s_v[threadIdx.x] = v < grp.n_lim ? (int32_t)v : -1;
        s_e[threadIdx.x] = e0 + threadIdx.x;
      }
      __syncthreads();
      for (int q = threadIdx.x; q < cnt * T; q += BLK) {
        int j = q / T, t = q - j * T;
        int v = s_v[j];
        s_c[q] = v >= 0 ? colr[(int64_t)t * g.n + v] : 0;
      }
      for (int q = threadIdx.x; q < cnt * B; q += BLK) {
        int j = q / B, b = q - j * B;
        int v = s_v[j];
        uint8_t x = (v >= 0 && v < grp.src[b] && w < grp.src[b]) ? a.act[(int64_t)v * B + b] : 0;
        s_a[q] = x;
        if (x) s_any[b] = 1;
      }
      __syncthreads();
      const bool last = s_v[cnt - 1] < 0;
      if (!et.val) {
        // data edges: gather four neighbours at a time, every load issued
        // (inactive lanes read a zero word) so that they are all in flight
        for (int j0 = 0; j0 < cnt; j0 += 4) {
          uint64_t x[4][NI];
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const int j = j0 + q;
            const int v = j < cnt ? s_v[j] : -1;
#pragma unroll
            for (int i = 0; i < NI; i++) {
              const uint64_t *ptr = g_zero;
              if (v >= 0 && ok[i] && s_a[j * B + I.b[i]]) {
                const int cv = s_c[j * T + I.t[i]];
                if ((Rp[i] >> cv) & 1u)
                  ptr = a.val + (((int64_t)v * B + I.b[i]) * T + I.t[i]) * Ca +
                        s_rank[squeeze2(Rp[i] & ~(1u << cv), cu[i], cv)];
              }
              x[q][i] = *ptr;
            }
          }
#pragma unroll
          for (int i = 0; i < NI; i++) {
            bool of = false;
#pragma unroll
            for (int q = 0; q < 4; q++) add_ck(acc[i], x[q][i], of);
            if (of) ofm |= 1ull << I.t[i];
          }
        }
        if (last) break;
        continue;
      }
      for (int j = 0; j < cnt; j++) {
        const int v = s_v[j];
        if (v < 0) break;
#pragma unroll
        for (int i = 0; i < NI; i++) {
          if (!ok[i] || !s_a[j * B + I.b[i]]) continue;
          const int cv = s_c[j * T + I.t[i]];
          if (!((Rp[i] >> cv) & 1u)) continue;
          const uint32_t R = Rp[i] & ~(1u << cv);
          const uint64_t *av = a.val + (((int64_t)v * B + I.b[i]) * T + I.t[i]) * Ca;
          bool of = false;
          if (!et.val) {
            add_ck(acc[i], av[s_rank[squeeze2(R, cu[i], cv)]], of);
          } else {
            const int64_t e = s_e[j];
            const int64_t tslot = e_src_first ? g.rev[e] : e;
            const uint64_t *ev = et.val + (tslot * T + I.t[i]) * et.C;
            uint32_t s1 = R;
            for (;;) {
              if (__popc(s1) == ra) {
                uint64_t x = av[s_rank[squeeze2(s1, cu[i], cv)]];
                if (x) {
                  uint64_t y = ev[s_rank[squeeze2(R & ~s1, cv, cw[i])]];
                  if (y) add_ck(acc[i], mul_ck(x, y, of), of);
                }
              }
              if (s1 == 0) break;
              s1 = (s1 - 1) & R;
            }
          }
          if (of) ofm |= 1ull << I.t[i];
        }
      }
      if (last) break;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NI; i++)
      if (I.on[i]) dst.val[((w * B + I.b[i]) * T + I.t[i]) * C + I.c[i]] = acc[i];
    if (grp.dense && threadIdx.x < B) dst.act[w * B + threadIdx.x] = s_any[threadIdx.x];
    flag_trials(ovf, ofm);
    if (grp.prof && threadIdx.x == 0) {
      uint64_t sc = 0;
      for (int64_t e = rs; e < re; e++) {
        if (g.col[e] >= grp.n_lim) break;
        sc++;
      }
      atomicAdd((unsigned long long *)&grp.prof[0], (unsigned long long)sc);
    }
    if (grp.prof && threadIdx.x < B && s_any[threadIdx.x]) {
      // active in-neighbours of (w, b)
      uint64_t ac = 0;
      for (int64_t e = rs; e < re; e++) {
        int64_t v = g.col[e];
        if (v >= grp.n_lim) break;
        if (v < grp.src[threadIdx.x] && a.act[v * B + threadIdx.x]) ac++;
      }
      atomicAdd((unsigned long long *)&grp.prof[1], (unsigned long long)ac);
      atomicAdd((unsigned long long *)&grp.prof[2], 1ull);
    }
  }
}

// ------------------------------------------------------------------ EdgeJoin over data edges (scatter)
// The same join for a data edge (alpha_2 = {chi v, chi w}), input-stationary:
// per output vertex w, lanes span the [b][t][input slot] block of a
// neighbour, so each active neighbour's block is read once, coalesced, and
// every input slot S is added, in LDS, to the output slot S + chi(v) (when
// chi(w) is not already in S).  Accumulators: B * T * C_out words of
// dynamic LDS.
template <int NI>
__global__ __launch_bounds__(BLK) void k_ejs(GraphDev g, GroupDev grp, const uint8_t *colr, RegDev a, RegDev dst,
                                             uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ int32_t s_v[64];
  __shared__ uint8_t s_c[64 * 64];
  __shared__ uint8_t s_a[64 * 64];
  __shared__ uint8_t s_any[64];
  extern __shared__ uint64_t s_out[];
  load_rank(s_rank, lut);
  const int B = grp.B, T = grp.T, C = dst.C, Ca = a.C;
  const int outs = B * T * C;
  Items<NI> I;
  I.init(B, T, Ca);
  int cu[NI];
  int64_t ub[NI];
  uint32_t min_[NI];
#pragma unroll
  for (int i = 0; i < NI; i++) {
    ub[i] = grp.src[I.b[i]];
    cu[i] = colr[(int64_t)I.t[i] * g.n + ub[i]];
    min_[i] = I.on[i] ? unrank(lut, a.s - 2, I.c[i]) : 0u;
  }
  const int64_t N = vdomain(grp, dst);
  uint64_t ofm = 0;
  for (int64_t wi = blockIdx.x; wi < N; wi += gridDim.x) {
    const int64_t w = vertex_at(grp, dst, wi);
    __syncthreads();
    for (int q = threadIdx.x; q < outs; q += BLK) s_out[q] = 0;
    if (threadIdx.x < 64) s_any[threadIdx.x] = 0;
    int cw[NI];
    bool ok[NI];
#pragma unroll
    for (int i = 0; i < NI; i++) {
      cw[i] = colr[(int64_t)I.t[i] * g.n + w];
      ok[i] = I.on[i] && w < ub[i] && cw[i] != cu[i];
    }
    const int64_t rs = g.rp[w], re = g.rp[w + 1];
    for (int64_t e0 = rs; e0 < re; e0 += 64) {
      __syncthreads();
      const int cnt = (int)min((int64_t)64, re - e0);
      if (threadIdx.x < cnt) {
        int64_t v = g.col[e0 + threadIdx.x];
        s_v[threadIdx.x] = v < grp.n_lim ? (int32_t)v : -1;
      }
      __syncthreads();
      for (int q = threadIdx.x; q < cnt * T; q += BLK) {
        int j = q / T, t = q - j * T;
        int v = s_v[j];
        s_c[q] = v >= 0 ? colr[(int64_t)t * g.n + v] : 0;
      }
      for (int q = threadIdx.x; q < cnt * B; q += BLK) {
        int j = q / B, b = q - j * B;
        int v = s_v[j];
        uint8_t x = (v >= 0 && v < grp.src[b] && w < grp.src[b]) ? a.act[(int64_t)v * B + b] : 0;
        s_a[q] = x;
        if (x) s_any[b] = 1;
      }
      __syncthreads();
      const bool last = s_v[cnt - 1] < 0;
      for (int j0 = 0; j0 < cnt; j0 += 4) {
        uint64_t val[4][NI];
        int slot[4][NI];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int j = j0 + q;
          const int v = j < cnt ? s_v[j] : -1;
#pragma unroll
          for (int i = 0; i < NI; i++) {
            slot[q][i] = -1;
            val[q][i] = 0;
            if (v >= 0 && ok[i] && s_a[j * B + I.b[i]]) {
              const int cv = s_c[j * T + I.t[i]];
              if (cv != cu[i] && cv != cw[i]) {
                const uint32_t R = spread2(min_[i], cu[i], cv);
                if (!((R >> cw[i]) & 1u)) {
                  slot[q][i] = s_rank[squeeze2(R | (1u << cv), cu[i], cw[i])];
                  val[q][i] = a.val[(((int64_t)v * B + I.b[i]) * T + I.t[i]) * Ca + I.c[i]];
                }
              }
            }
          }
        }
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
          for (int i = 0; i < NI; i++)
            if (slot[q][i] >= 0 && val[q][i]) {
              uint64_t *p = &s_out[(I.b[i] * T + I.t[i]) * C + slot[q][i]];
              unsigned long long old = atomicAdd((unsigned long long *)p, (unsigned long long)val[q][i]);
              if ((uint64_t)old + val[q][i] < (uint64_t)old) ofm |= 1ull << I.t[i];
            }
      }
      if (last) break;
    }
    __syncthreads();
    uint64_t *drow = dst.val + w * (int64_t)outs;
    for (int q = threadIdx.x; q < outs; q += BLK) drow[q] = s_out[q];
    if (grp.dense && threadIdx.x < B) dst.act[w * B + threadIdx.x] = s_any[threadIdx.x];
  }
  flag_trials(ovf, ofm);
}

// ------------------------------------------------------------------ NodeJoin
// dst[v][b][R'] = sum over splits R' = R + Ra of a[v][b][R] * A[v][Ra]
// One thread per output slot (vertex, source, trial, slot).
__global__ __launch_bounds__(BLK) void k_nj(GroupDev grp, int64_t n, const uint8_t *colr, RegDev a, RegDev dst,
                                            TabDev nt, uint32_t *ovf, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int B = grp.B, T = grp.T, C = dst.C, Ca = a.C;
  const int rA = nt.s - 1;
  const int64_t per = (int64_t)B * T * C;
  const int64_t N = vdomain(grp, a) * per;
  uint64_t ofm = 0;
  for (int64_t idx = (int64_t)blockIdx.x * BLK + threadIdx.x; idx < N; idx += (int64_t)gridDim.x * BLK) {
    const int64_t vi = idx / per;
    const int r = (int)(idx - vi * per);
    const int b = r / (T * C), r2 = r - b * T * C, t = r2 / C, c = r2 - t * C;
    const int64_t v = vertex_at(grp, a, vi);
    const int64_t ent = v * B + b;
    if (!a.act[ent]) continue;
    const int cu = colr[(int64_t)t * n + grp.src[b]], cv = colr[(int64_t)t * n + v];
    uint64_t acc = 0;
    bool of = false;
    if (cu != cv) {
      const uint32_t Rp = spread2(unrank(lut, dst.s - 2, c), cu, cv);
      const uint64_t *av = a.val + (ent * T + t) * Ca;
      const uint64_t *nv = nt.val + (v * T + t) * nt.C;
      uint32_t sA = Rp;
      for (;;) {
        if (__popc(sA) == rA) {
          uint64_t y = nv[s_rank[squeeze1(sA, cv)]];
          if (y) {
            uint64_t x = av[s_rank[squeeze2(Rp & ~sA, cu, cv)]];
            if (x) add_ck(acc, mul_ck(x, y, of), of);
          }
        }
        if (sA == 0) break;
        sA = (sA - 1) & Rp;
      }
    }
    dst.val[(ent * T + t) * C + c] = acc;
    if (of) ofm |= 1ull << t;
  }
  flag_trials(ovf, ofm);
}

// ------------------------------------------------------------------ AXPY
// Sparse mode, first pass: list in dst every vertex of a not yet there and
// start its row from zero; copy a's activity into dst.
__global__ void k_axpy_mark(GroupDev grp, RegDev a, RegDev dst) {
  __shared__ int s_new;
  const int B = grp.B;
  const int64_t per = (int64_t)B * grp.T * dst.C;
  const int64_t N = *a.vcnt;
  for (int64_t vi = blockIdx.x; vi < N; vi += gridDim.x) {
    const int64_t v = a.vlist[vi];
    __syncthreads();
    if (threadIdx.x == 0) {
      s_new = 0;
      if (set_act(dst.vmark, v)) {
        uint32_t pos = atomicAdd(dst.vcnt, 1u);
        dst.vlist[pos] = (int32_t)v;
        s_new = 1;
      }
    }
    __syncthreads();
    if (s_new)
      for (int64_t j = threadIdx.x; j < per; j += BLK) dst.val[v * per + j] = 0;
    for (int b = threadIdx.x; b < B; b += BLK)
      if (a.act[v * B + b]) dst.act[v * B + b] = 1;
  }
}

// dst += w * a over a's domain, one thread per slot.  A dense dst on its
// first AXPY is written over the whole domain (w * a where a is active, 0
// elsewhere), activity included.
__global__ __launch_bounds__(BLK) void k_axpy(GroupDev grp, RegDev a, RegDev dst, uint64_t w, int first,
                                              uint32_t *ovf) {
  const int B = grp.B, T = grp.T, C = dst.C;
  const int64_t per = (int64_t)B * T * C;
  const int64_t N = vdomain(grp, a) * per;
  uint64_t ofm = 0;
  for (int64_t idx = (int64_t)blockIdx.x * BLK + threadIdx.x; idx < N; idx += (int64_t)gridDim.x * BLK) {
    const int64_t vi = idx / per;
    const int r = (int)(idx - vi * per);
    const int b = r / (T * C);
    const int64_t v = vertex_at(grp, a, vi);
    const int64_t ent = v * B + b;
    const int64_t o = v * per + r;
    const bool act = a.act[ent] != 0;
    bool of = false;
    if (grp.dense && first) {
      dst.val[o] = act ? mul_ck(w, a.val[o], of) : 0;
      if (r - b * T * C == 0) dst.act[ent] = act ? 1 : 0;
    } else if (act) {
      uint64_t y = dst.val[o];
      add_ck(y, mul_ck(w, a.val[o], of), of);
      dst.val[o] = y;
      if (grp.dense && r - b * T * C == 0) dst.act[ent] = 1;
    }
    if (of) ofm |= 1ull << ((r / C) % T);
  }
  flag_trials(ovf, ofm);
}

// ------------------------------------------------------------------ root merge
// count[t] += w * sum over (v, b) active in both, of
//             sum over R of a[v][b][R] * b[v][b][K \ {chi u, chi v} \ R]
// One thread per slot of a; 128-bit partial sums per thread (one trial) or
// in LDS (several trials).
__global__ __launch_bounds__(BLK) void k_mroot(GroupDev grp, int64_t n, const uint8_t *colr, RegDev a, RegDev bb,
                                               uint64_t w, AccDev acc, const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint64_t s_acc[2 * 64];
  for (int i = threadIdx.x; i < 2 * 64; i += blockDim.x) s_acc[i] = 0;
  load_rank(s_rank, lut);
  const int B = grp.B, T = grp.T, Ca = a.C, Cb = bb.C, k = grp.k;
  const uint32_t Kmask = (1u << k) - 1u;
  const int64_t per = (int64_t)B * T * Ca;
  const int64_t N = vdomain(grp, a) * per;
  uint64_t lo0 = 0, hi0 = 0;
  for (int64_t idx = (int64_t)blockIdx.x * BLK + threadIdx.x; idx < N; idx += (int64_t)gridDim.x * BLK) {
    const int64_t vi = idx / per;
    const int r = (int)(idx - vi * per);
    const int b = r / (T * Ca), r2 = r - b * T * Ca, t = r2 / Ca, c = r2 - t * Ca;
    const int64_t v = vertex_at(grp, a, vi);
    const int64_t ent = v * B + b;
    if (!a.act[ent] || !bb.act[ent]) continue;
    const uint64_t x = a.val[v * per + r];
    if (!x) continue;
    const int64_t u = grp.src[b];
    const int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
    if (cu == cv) continue;
    const uint32_t R1 = spread2(unrank(lut, a.s - 2, c), cu, cv);
    const uint32_t R2 = Kmask & ~R1 & ~(1u << cu) & ~(1u << cv);
    const uint64_t y = bb.val[(ent * T + t) * Cb + s_rank[squeeze2(R2, cu, cv)]];
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
// MU: out[u_b][R'] += w * sum_v sum over splits of R' \ {chi v} of a[v][b][.] * b[v][b][.]
//     (items over (b, t, slot); partial sums stay in registers across vertices)
template <int NI>
__global__ __launch_bounds__(BLK) void k_mu(GroupDev grp, int64_t n, const uint8_t *colr, RegDev a, RegDev bb,
                                            uint64_t w, uint64_t *out, int s_out, int C_out, uint32_t *ovf,
                                            const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int B = grp.B, T = grp.T, Ca = a.C, Cb = bb.C;
  const int ra = a.s - 2;
  Items<NI> I;
  I.init(B, T, C_out);
  int cu[NI];
  uint32_t Rq[NI];
  uint64_t acc[NI];
#pragma unroll
  for (int i = 0; i < NI; i++) {
    cu[i] = colr[(int64_t)I.t[i] * n + grp.src[I.b[i]]];
    Rq[i] = I.on[i] ? spread1(unrank(lut, s_out - 1, I.c[i]), cu[i]) : 0u;
    acc[i] = 0;
  }
  uint64_t ofm = 0;
  const int64_t N = vdomain(grp, a);
  for (int64_t vi = blockIdx.x; vi < N; vi += gridDim.x) {
    const int64_t v = vertex_at(grp, a, vi);
#pragma unroll
    for (int i = 0; i < NI; i++) {
      if (!I.on[i]) continue;
      const int64_t ent = v * B + I.b[i];
      if (!a.act[ent] || !bb.act[ent]) continue;
      const int t = I.t[i];
      const int cv = colr[(int64_t)t * n + v];
      if (cv == cu[i] || !((Rq[i] >> cv) & 1u)) continue;
      const uint32_t R = Rq[i] & ~(1u << cv);
      const uint64_t *av = a.val + (ent * T + t) * Ca;
      const uint64_t *bv = bb.val + (ent * T + t) * Cb;
      bool of = false;
      uint32_t s1 = R;
      for (;;) {
        if (__popc(s1) == ra) {
          uint64_t x = av[s_rank[squeeze2(s1, cu[i], cv)]];
          if (x) {
            uint64_t y = bv[s_rank[squeeze2(R & ~s1, cu[i], cv)]];
            if (y) add_ck(acc[i], mul_ck(x, y, of), of);
          }
        }
        if (s1 == 0) break;
        s1 = (s1 - 1) & R;
      }
      if (of) ofm |= 1ull << t;
    }
  }
#pragma unroll
  for (int i = 0; i < NI; i++)
    if (I.on[i] && acc[i]) {
      bool of = false;
      uint64_t s = mul_ck(acc[i], w, of);
      atomic_add_ck(&out[((int64_t)grp.src[I.b[i]] * T + I.t[i]) * C_out + I.c[i]], s, of);
      if (of) ofm |= 1ull << I.t[i];
    }
  flag_trials(ovf, ofm);
}

// MV: out[v][R'] += w * sum_b sum over splits of R' \ {chi u_b} of a[v][b][.] * b[v][b][.]
//     (items over (t, slot) of the output row of v, sources summed in the thread)
template <int NI>
__global__ __launch_bounds__(BLK) void k_mv(GroupDev grp, int64_t n, const uint8_t *colr, RegDev a, RegDev bb,
                                            uint64_t w, uint64_t *out, int s_out, int C_out, uint32_t *ovf,
                                            const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int B = grp.B, T = grp.T, Ca = a.C, Cb = bb.C;
  const int ra = a.s - 2;
  Items<NI> I;
  I.init(1, T, C_out);
  uint64_t ofm = 0;
  const int64_t N = vdomain(grp, a);
  for (int64_t vi = blockIdx.x; vi < N; vi += gridDim.x) {
    const int64_t v = vertex_at(grp, a, vi);
#pragma unroll
    for (int i = 0; i < NI; i++) {
      if (!I.on[i]) continue;
      const int t = I.t[i];
      const int cv = colr[(int64_t)t * n + v];
      const uint32_t Rq = spread1(unrank(lut, s_out - 1, I.c[i]), cv);
      uint64_t acc = 0;
      bool of = false;
      for (int b = 0; b < B; b++) {
        const int64_t ent = v * B + b;
        if (!a.act[ent] || !bb.act[ent]) continue;
        const int cu = colr[(int64_t)t * n + grp.src[b]];
        if (cu == cv || !((Rq >> cu) & 1u)) continue;
        const uint32_t R = Rq & ~(1u << cu);
        const uint64_t *av = a.val + (ent * T + t) * Ca;
        const uint64_t *bv = bb.val + (ent * T + t) * Cb;
        uint32_t s1 = R;
        for (;;) {
          if (__popc(s1) == ra) {
            uint64_t x = av[s_rank[squeeze2(s1, cu, cv)]];
            if (x) {
              uint64_t y = bv[s_rank[squeeze2(R & ~s1, cu, cv)]];
              if (y) add_ck(acc, mul_ck(x, y, of), of);
            }
          }
          if (s1 == 0) break;
          s1 = (s1 - 1) & R;
        }
      }
      if (acc) {
        const int64_t o = (v * T + t) * C_out + I.c[i];
        uint64_t y = out[o];
        add_ck(y, mul_ck(acc, w, of), of);
        out[o] = y;
      }
      if (of) ofm |= 1ull << t;
    }
  }
  flag_trials(ovf, ofm);
}

// ------------------------------------------------------------------ edge merge
// T[x,y][R'] += w * sum_b a[x][b][R1] * E(x,y)[Re] * b[y][b][R2],
//               R' \ {chi u_b} = R1 + Re + R2
// One workgroup per vertex x of a; items over (neighbour j of a 64-chunk, t, slot).
__global__ __launch_bounds__(BLK) void k_medge(GraphDev g, GroupDev grp, const uint8_t *colr, RegDev a, RegDev bb,
                                               TabDev et, int e_src_first, int out_first_is_x, uint64_t w,
                                               uint64_t *out, int s_out, int C_out, uint32_t *ovf,
                                               const uint16_t *lut) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint8_t s_ax[64];
  load_rank(s_rank, lut);
  const int B = grp.B, T = grp.T, Ca = a.C, Cb = bb.C;
  const int ra = a.s - 2, rb = bb.s - 2;
  uint64_t ofm = 0;
  const int64_t N = vdomain(grp, a);
  for (int64_t xi = blockIdx.x; xi < N; xi += gridDim.x) {
    const int64_t x = vertex_at(grp, a, xi);
    __syncthreads();
    if (threadIdx.x < B) s_ax[threadIdx.x] = (x < grp.src[threadIdx.x]) ? a.act[x * B + threadIdx.x] : 0;
    __syncthreads();
    const int64_t rs = g.rp[x], re = g.rp[x + 1];
    const int64_t per = (int64_t)T * C_out;
    for (int64_t q = threadIdx.x; q < (re - rs) * per; q += BLK) {
      const int64_t e = rs + q / per;
      const int r = (int)(q % per);
      const int t = r / C_out, c = r - t * C_out;
      const int64_t y = g.col[e];
      if (y >= grp.n_lim) continue;
      const int cx = colr[(int64_t)t * g.n + x], cy = colr[(int64_t)t * g.n + y];
      if (cx == cy) continue;
      const uint32_t Rp = spread2(unrank(lut, s_out - 2, c), cx, cy);
      const int64_t tslot = e_src_first ? e : g.rev[e];
      const uint64_t *ev = et.val ? et.val + (tslot * T + t) * et.C : nullptr;
      uint64_t s = 0;
      bool of = false;
      for (int b = 0; b < B; b++) {
        if (!s_ax[b] || y >= grp.src[b]) continue;
        const int64_t enty = y * B + b;
        if (!bb.act[enty]) continue;
        const int cu = colr[(int64_t)t * g.n + grp.src[b]];
        if (cu == cx || cu == cy || !((Rp >> cu) & 1u)) continue;
        const uint32_t R = Rp & ~(1u << cu);
        const uint64_t *av = a.val + ((x * B + b) * T + t) * Ca;
        const uint64_t *bv = bb.val + (enty * T + t) * Cb;
        uint32_t s1 = R;
        for (;;) {
          if (__popc(s1) == ra) {
            uint64_t xa = av[s_rank[squeeze2(s1, cu, cx)]];
            if (xa) {
              uint32_t Q = R & ~s1;
              uint32_t s2 = Q;
              for (;;) {
                if (__popc(s2) == rb) {
                  uint64_t xb = bv[s_rank[squeeze2(s2, cu, cy)]];
                  uint32_t Qe = Q & ~s2;
                  uint64_t xe = ev ? ev[s_rank[squeeze2(Qe, cx, cy)]] : (Qe == 0 ? 1u : 0u);
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
      }
      if (s) {
        const int64_t oslot = out_first_is_x ? e : g.rev[e];
        const int64_t o = (oslot * T + t) * C_out + c;
        uint64_t y0 = out[o];
        add_ck(y0, mul_ck(s, w, of), of);
        out[o] = y0;
      }
      if (of) ofm |= 1ull << t;
    }
  }
  flag_trials(ovf, ofm);
}

// T[u,y] += w * A[u][Ra] * E(u,y)[Re] * b[y][b][R2] over the lower neighbours y of u_b.
__global__ void k_medge_t(GraphDev g, GroupDev grp, const uint8_t *colr, const int32_t *lowcnt, int max_low,
                          TabDev nt, RegDev bb, TabDev et, int e_src_first, int out_first_is_u, uint64_t w,
                          uint64_t *out, int s_out, int C_out, uint32_t *ovf, const uint16_t *lut, int P) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int epb = blockDim.x / P, lane = threadIdx.x % P, sub = threadIdx.x / P;
  const int Cb = bb.C, T = grp.T, B = grp.B;
  const int items = T * C_out;
  const int64_t N = (int64_t)B * max_low;
  const int rA = nt.val ? nt.s - 1 : 0, rb = bb.s - 2;
  uint64_t ofm = 0;
  for (int64_t e0 = (int64_t)blockIdx.x * epb; e0 < N; e0 += (int64_t)gridDim.x * epb) {
    int64_t en = e0 + sub;
    if (en >= N) continue;
    int b = (int)(en / max_low);
    int j = (int)(en - (int64_t)b * max_low);
    int64_t u = grp.src[b];
    if (j >= lowcnt[u]) continue;
    int64_t es = g.rp[u] + j;
    int64_t y = g.col[es];
    int64_t enty = y * B + b;
    if (!bb.act[enty]) continue;
    int64_t tslot = e_src_first ? es : g.rev[es];
    int64_t oslot = out_first_is_u ? es : g.rev[es];
    for (int it = lane; it < items; it += P) {
      int t = it / C_out, c = it - t * C_out;
      int cu = colr[(int64_t)t * g.n + u], cy = colr[(int64_t)t * g.n + y];
      if (cu == cy) continue;
      uint32_t R = spread2(unrank(lut, s_out - 2, c), cu, cy);
      const uint64_t *bv = bb.val + (enty * T + t) * Cb;
      const uint64_t *ev = et.val ? et.val + (tslot * T + t) * et.C : nullptr;
      const uint64_t *av = nt.val ? nt.val + ((int64_t)u * T + t) * nt.C : nullptr;
      uint64_t s = 0;
      bool of = false;
      uint32_t sA = R;
      for (;;) {
        if (__popc(sA) == rA) {
          uint64_t xa = av ? av[s_rank[squeeze1(sA, cu)]] : 1u;
          if (xa) {
            uint32_t Q = R & ~sA;
            uint32_t s2 = Q;
            for (;;) {
              if (__popc(s2) == rb) {
                uint64_t xb = bv[s_rank[squeeze2(s2, cu, cy)]];
                uint32_t Qe = Q & ~s2;
                uint64_t xe = ev ? ev[s_rank[squeeze2(Qe, cu, cy)]] : (Qe == 0 ? 1u : 0u);
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
        const int64_t o = (oslot * T + t) * C_out + c;
        uint64_t y0 = out[o];
        add_ck(y0, mul_ck(s, w, of), of);
        out[o] = y0;
      }
      if (of) ofm |= 1ull << t;
    }
  }
  flag_trials(ovf, ofm);
}

// ------------------------------------------------------------------ leaf block
// U[x][R'] = sum over y in N(x) of sum over splits R' \ {chi y} = Ra + Re + Rb of
//            A_a[x][Ra] * E(x,y)[Re] * A_b[y][Rb]
__global__ void k_leaf(GraphDev g, int T, const uint8_t *colr, TabDev na, TabDev ea, int e_src_first, TabDev nb,
                       uint64_t *out, int s_out, int C_out, uint32_t *ovf, const uint16_t *lut, int P) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int epb = blockDim.x / P, lane = threadIdx.x % P, sub = threadIdx.x / P;
  const int items = T * C_out;
  const int64_t N = g.n;
  const int rA = na.val ? na.s - 1 : 0, rB = nb.val ? nb.s - 1 : 0;
  uint64_t ofm = 0;
  for (int64_t e0 = (int64_t)blockIdx.x * epb; e0 < N; e0 += (int64_t)gridDim.x * epb) {
    int64_t x = e0 + sub;
    if (x >= N) continue;
    for (int it = lane; it < items; it += P) {
      int t = it / C_out, c = it - t * C_out;
      int cx = colr[(int64_t)t * g.n + x];
      uint32_t Rp = spread1(unrank(lut, s_out - 1, c), cx);
      const uint64_t *av = na.val ? na.val + (x * T + t) * na.C : nullptr;
      uint64_t s = 0;
      bool of = false;
      for (int64_t e = g.rp[x]; e < g.rp[x + 1]; e++) {
        int64_t y = g.col[e];
        int cy = colr[(int64_t)t * g.n + y];
        if (!((Rp >> cy) & 1u)) continue;
        uint32_t R = Rp & ~(1u << cy);
        const uint64_t *bv = nb.val ? nb.val + (y * T + t) * nb.C : nullptr;
        int64_t tslot = e_src_first ? e : g.rev[e];
        const uint64_t *ev = ea.val ? ea.val + (tslot * T + t) * ea.C : nullptr;
        uint32_t sA = R;
        for (;;) {
          if (__popc(sA) == rA) {
            uint64_t xa = av ? av[s_rank[squeeze1(sA, cx)]] : 1u;
            if (xa) {
              uint32_t Q = R & ~sA;
              uint32_t sB = Q;
              for (;;) {
                if (__popc(sB) == rB) {
                  uint64_t xb = bv ? bv[s_rank[squeeze1(sB, cy)]] : 1u;
                  uint32_t Qe = Q & ~sB;
                  uint64_t xe = ev ? ev[s_rank[squeeze2(Qe, cx, cy)]] : (Qe == 0 ? 1u : 0u);
                  if (xb && xe) add_ck(s, mul_ck(mul_ck(xa, xb, of), xe, of), of);
                }
                if (sB == 0) break;
                sB = (sB - 1) & Q;
              }
            }
          }
          if (sA == 0) break;
          sA = (sA - 1) & R;
        }
      }
      out[(x * T + t) * C_out + c] = s;
      if (of) ofm |= 1ull << t;
    }
  }
  flag_trials(ovf, ofm);
}

// ------------------------------------------------------------------ singleton root
__global__ void k_root_single(int64_t n, int T, TabDev U, AccDev acc) {
  __shared__ uint64_t s_acc[2 * 64];
  for (int i = threadIdx.x; i < 2 * 64; i += blockDim.x) s_acc[i] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * T; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t x = i / T;
    int t = (int)(i - x * T);
    uint64_t v = U.val[(x * T + t) * U.C];
    if (v) {
      atomic_add128(&s_acc[2 * t], v, 0);
      if (acc.per_src) atomic_add128(&acc.per_src[2 * (x * T + t)], v, 0);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += blockDim.x) atomic_add128(&acc.sum[2 * t], s_acc[2 * t], s_acc[2 * t + 1]);
}

// ------------------------------------------------------------------ launch helpers
inline int pick_p(int items) {
  int p = 1;
  while (p < items && p < BLK) p <<= 1;
  return p;
}
inline int grid_for(int64_t entries, int P) {
  int epb = BLK / P;
  int64_t g = (entries + epb - 1) / epb;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}
// workgroups for a vertex-domain kernel
inline int vgrid(const GroupDev &grp) {
  if (!grp.dense) return 4096;
  return (int)std::max<int64_t>(1, std::min<int64_t>(grp.n_lim, 65536));
}

#define DISPATCH_NI(items, KERNEL, ...)                                                        \
  do {                                                                                         \
    int _ni = ((items) + BLK - 1) / BLK;                                                       \
    if (_ni <= 1) hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__);                                  \
    else if (_ni <= 2) hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__);                             \
    else if (_ni <= 4) hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__);                             \
    else if (_ni <= 8) hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__);                             \
    else if (_ni <= 16) hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);                           \
    else hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__);                                          \
  } while (0)

}  // namespace

int max_items_per_vertex() { return 32 * BLK; }

// colex rank / unrank tables (per device, built once)
const uint16_t *lut_device(int device) {
  static std::mutex mu;
  static std::vector<uint16_t *> tabs;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)tabs.size() <= device) tabs.resize(device + 1, nullptr);
  if (tabs[device]) return tabs[device];
  std::vector<uint16_t> h(LUT_SIZE, 0);
  // colex rank of m among masks with the same popcount: sum_i C(p_i, i+1)
  auto C = [](int n, int r) -> int {
    if (r < 0 || r > n) return 0;
    long c = 1;
    for (int i = 1; i <= r; i++) c = c * (n - r + i) / i;
    return (int)c;
  };
  std::vector<std::vector<uint32_t>> byr(12);
  for (uint32_t m = 0; m < 2048; m++) {
    int idx = 0, i = 0;
    for (int p = 0; p < 11; p++)
      if (m >> p & 1u) idx += C(p, ++i);
    h[LUT_RANK + m] = (uint16_t)idx;
    byr[__builtin_popcount(m)].push_back(m);
  }
  int off = 0;
  for (int r = 0; r <= 11; r++) {
    h[LUT_OFF + r] = (uint16_t)off;
    std::vector<uint32_t> v = byr[r];
    std::sort(v.begin(), v.end(), [&](uint32_t a, uint32_t b) { return h[a] < h[b]; });
    for (uint32_t m : v) h[LUT_UNRANK + off++] = (uint16_t)m;
  }
  uint16_t *d = nullptr;
  if (hipMalloc(&d, sizeof(uint16_t) * LUT_SIZE) != hipSuccess) return nullptr;
  if (hipMemcpy(d, h.data(), sizeof(uint16_t) * LUT_SIZE, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  tabs[device] = d;
  return d;
}

static const uint16_t *cur_lut() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return lut_device(dev);
}

void launch_colour(const int32_t *orig, int64_t n, int k, uint64_t seed, int t0, int T, uint8_t *out,
                   hipStream_t st) {
  int64_t tot = n * T;
  hipLaunchKernelGGL(k_colour, dim3((unsigned)((tot + BLK - 1) / BLK)), dim3(BLK), 0, st, orig, n, k, seed, t0, T,
                     out);
}
void launch_permute_colours(const uint8_t *by_orig, const int32_t *orig, int64_t n, int T, uint8_t *out,
                            hipStream_t st) {
  int64_t tot = n * T;
  hipLaunchKernelGGL(k_permute, dim3((unsigned)((tot + BLK - 1) / BLK)), dim3(BLK), 0, st, by_orig, orig, n, T, out);
}
void launch_fill_u8(uint8_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t g = std::min<int64_t>((n + BLK - 1) / BLK, 8192);
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)g), dim3(BLK), 0, st, p, n);
}
void launch_fill_u64(uint64_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t g = std::min<int64_t>((n + BLK - 1) / BLK, 8192);
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)g), dim3(BLK), 0, st, p, n);
}
void launch_clear_list(RegDev r, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_list, dim3(1024), dim3(BLK), 0, st, r.act, r.vmark, r.vlist, r.vcnt, B);
  hipLaunchKernelGGL(k_reset_cnt, dim3(1), dim3(1), 0, st, r.vcnt);
}

void launch_init(const GraphDev &g, const GroupDev &grp, const int32_t *lowcnt, int max_low, const uint8_t *colr,
                 RegDev dst, TabDev etab, int e_src_first, TabDev ntab, uint32_t *ovf, hipStream_t st) {
  int P = pick_p(grp.T * dst.C);
  int64_t N = (int64_t)grp.B * max_low;
  hipLaunchKernelGGL(k_init, dim3(grid_for(N, P)), dim3(BLK), 0, st, g, grp, lowcnt, max_low, colr, dst, etab,
                     e_src_first, ntab, ovf, cur_lut(), P);
}
void launch_mark(const GraphDev &g, const GroupDev &grp, RegDev a, RegDev dst, hipStream_t st) {
  hipLaunchKernelGGL(k_mark, dim3(4096), dim3(BLK), 0, st, g, grp, a, dst);
}
void launch_ej(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, RegDev a, RegDev dst, TabDev etab,
               int e_src_first, uint32_t *ovf, hipStream_t st) {
  const int outs = grp.B * grp.T * dst.C;
  if (!etab.val && !grp.prof && outs <= 4096) {
    int items_in = grp.B * grp.T * a.C;
    size_t lds = sizeof(uint64_t) * (size_t)outs;
    DISPATCH_NI(items_in, k_ejs, dim3(vgrid(grp)), dim3(BLK), lds, st, g, grp, colr, a, dst, ovf, cur_lut());
    return;
  }
  int items = grp.B * grp.T * dst.C;
  DISPATCH_NI(items, k_ej, dim3(vgrid(grp)), dim3(BLK), 0, st, g, grp, colr, a, dst, etab, e_src_first, ovf,
              cur_lut());
}
// workgroups for a kernel with one thread per (vertex, source, trial, slot)
static int fgrid(const GroupDev &grp, int C) {
  if (!grp.dense) return 8192;
  int64_t tot = grp.n_lim * (int64_t)grp.B * grp.T * C;
  return (int)std::max<int64_t>(1, std::min<int64_t>((tot + BLK - 1) / BLK, 65536));
}
void launch_nj(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, RegDev a, RegDev dst, TabDev ntab,
               uint32_t *ovf, hipStream_t st) {
  hipLaunchKernelGGL(k_nj, dim3(fgrid(grp, dst.C)), dim3(BLK), 0, st, grp, g.n, colr, a, dst, ntab, ovf, cur_lut());
}
void launch_axpy(const GroupDev &grp, RegDev a, RegDev dst, uint64_t w, int first, uint32_t *ovf, hipStream_t st) {
  if (!grp.dense) hipLaunchKernelGGL(k_axpy_mark, dim3(4096), dim3(BLK), 0, st, grp, a, dst);
  hipLaunchKernelGGL(k_axpy, dim3(fgrid(grp, dst.C)), dim3(BLK), 0, st, grp, a, dst, w, first, ovf);
}
void launch_mroot(const GroupDev &grp, int64_t n, const uint8_t *colr, RegDev a, RegDev b, uint64_t w,
                  AccDev acc, hipStream_t st) {
  hipLaunchKernelGGL(k_mroot, dim3(fgrid(grp, a.C)), dim3(BLK), 0, st, grp, n, colr, a, b, w, acc, cur_lut());
}
void launch_mu(const GroupDev &grp, int64_t n, const uint8_t *colr, RegDev a, RegDev b, uint64_t w, uint64_t *out,
               int s_out, int C_out, uint32_t *ovf, hipStream_t st) {
  int items = grp.B * grp.T * C_out;
  DISPATCH_NI(items, k_mu, dim3(vgrid(grp)), dim3(BLK), 0, st, grp, n, colr, a, b, w, out, s_out, C_out, ovf,
              cur_lut());
}
void launch_mv(const GroupDev &grp, int64_t n, const uint8_t *colr, RegDev a, RegDev b, uint64_t w, uint64_t *out,
               int s_out, int C_out, uint32_t *ovf, hipStream_t st) {
  int items = grp.T * C_out;
  DISPATCH_NI(items, k_mv, dim3(vgrid(grp)), dim3(BLK), 0, st, grp, n, colr, a, b, w, out, s_out, C_out, ovf,
              cur_lut());
}
void launch_medge(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, RegDev a, RegDev b, TabDev etab,
                  int e_src_first, int out_first_is_x, uint64_t w, uint64_t *out, int s_out, int C_out,
                  uint32_t *ovf, hipStream_t st) {
  hipLaunchKernelGGL(k_medge, dim3(vgrid(grp)), dim3(BLK), 0, st, g, grp, colr, a, b, etab, e_src_first,
                     out_first_is_x, w, out, s_out, C_out, ovf, cur_lut());
}
void launch_medge_t(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, const int32_t *lowcnt,
                    int max_low, TabDev ntab, RegDev b, TabDev etab, int e_src_first, int out_first_is_u,
                    uint64_t w, uint64_t *out, int s_out, int C_out, uint32_t *ovf, hipStream_t st) {
  int P = pick_p(grp.T * C_out);
  int64_t N = (int64_t)grp.B * max_low;
  hipLaunchKernelGGL(k_medge_t, dim3(grid_for(N, P)), dim3(BLK), 0, st, g, grp, colr, lowcnt, max_low, ntab, b,
                     etab, e_src_first, out_first_is_u, w, out, s_out, C_out, ovf, cur_lut(), P);
}
void launch_leaf(const GraphDev &g, int T, int k, const uint8_t *colr, TabDev na, TabDev ea, int e_src_first,
                 TabDev nb, uint64_t *out, int s_out, int C_out, uint32_t *ovf, hipStream_t st) {
  (void)k;
  int P = pick_p(T * C_out);
  hipLaunchKernelGGL(k_leaf, dim3(grid_for(g.n, P)), dim3(BLK), 0, st, g, T, colr, na, ea, e_src_first, nb, out,
                     s_out, C_out, ovf, cur_lut(), P);
}
void launch_root_single(int64_t n, int T, TabDev u, AccDev acc, hipStream_t st) {
  int64_t g = std::min<int64_t>((n * T + BLK - 1) / BLK, 8192);
  hipLaunchKernelGGL(k_root_single, dim3((unsigned)std::max<int64_t>(1, g)), dim3(BLK), 0, st, n, T, u, acc);
}

}  // namespace cc
