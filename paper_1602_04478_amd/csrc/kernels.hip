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

namespace cc {

namespace {

constexpr int BLK = 256;
constexpr int LUT_RANK = 0, LUT_UNRANK = 2048, LUT_OFF = 4096, LUT_SIZE = 4112;

__device__ __forceinline__ uint32_t squeeze2(uint32_t m, int c1, int c2) {
  int lo = min(c1, c2), hi = max(c1, c2);
  uint32_t a = m & ((1u << lo) - 1u);
  uint32_t b = (m >> (lo + 1)) & ((1u << (hi - lo - 1)) - 1u);
  uint32_t c = m >> (hi + 1);
  return a | (b << lo) | (c << (hi - 1));
}
__device__ __forceinline__ uint32_t spread2(uint32_t m, int c1, int c2) {
  int lo = min(c1, c2), hi = max(c1, c2);
  uint32_t a = m & ((1u << lo) - 1u);
  uint32_t b = (m >> lo) & ((1u << (hi - lo - 1)) - 1u);
  uint32_t c = m >> (hi - 1);
  return a | (b << (lo + 1)) | (c << (hi + 1));
}
__device__ __forceinline__ uint32_t squeeze1(uint32_t m, int c) {
  return (m & ((1u << c) - 1u)) | ((m >> (c + 1)) << c);
}
__device__ __forceinline__ uint32_t spread1(uint32_t m, int c) {
  return (m & ((1u << c) - 1u)) | ((m >> c) << (c + 1));
}
__device__ __forceinline__ uint32_t unrank(const uint16_t *lut, int r, int idx) {
  return lut[LUT_UNRANK + lut[LUT_OFF + r] + idx];
}

// acc += a (checked)
__device__ __forceinline__ void add_ck(uint64_t &acc, uint64_t a, bool &of) {
  uint64_t s = acc + a;
  of |= s < acc;
  acc = s;
}
// a * b (checked)
__device__ __forceinline__ uint64_t mul_ck(uint64_t a, uint64_t b, bool &of) {
  of |= __umul64hi(a, b) != 0;
  return a * b;
}
// global acc += a (checked through the returned old value)
__device__ __forceinline__ void atomic_add_ck(uint64_t *p, uint64_t a, bool &of) {
  if (a == 0) return;
  unsigned long long old = atomicAdd((unsigned long long *)p, (unsigned long long)a);
  of |= (uint64_t)old + a < (uint64_t)old;
}
// 128-bit add into (lo, hi) pair in LDS or global memory
__device__ __forceinline__ void atomic_add128(uint64_t *p, uint64_t lo, uint64_t hi) {
  if (lo) {
    unsigned long long old = atomicAdd((unsigned long long *)p, (unsigned long long)lo);
    if ((uint64_t)old + lo < (uint64_t)old) hi += 1;
  }
  if (hi) atomicAdd((unsigned long long *)(p + 1), (unsigned long long)hi);
}

__device__ __forceinline__ void load_rank(uint16_t *s_rank, const uint16_t *lut) {
  for (int i = threadIdx.x; i < 2048; i += blockDim.x) s_rank[i] = lut[LUT_RANK + i];
  __syncthreads();
}

// decode entry e of a domain into (v, b)
__device__ __forceinline__ void decode(const GroupDev &g, const int64_t *list, int64_t e, int64_t &v, int &b) {
  if (g.dense) {
    v = e / g.B;
    b = (int)(e - v * g.B);
  } else {
    int64_t x = list[e];
    v = x >> 6;
    b = (int)(x & 63);
  }
}

__device__ __forceinline__ int64_t domain_size(const GroupDev &g, const uint32_t *cnt) {
  return g.dense ? g.n_lim * (int64_t)g.B : (int64_t)(*cnt);
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// set the activity byte of entry i; returns true if it was clear
__device__ __forceinline__ bool set_act(uint8_t *act, int64_t i) {
  uint32_t *word = (uint32_t *)(act + (i & ~(int64_t)3));
  int sh = 8 * (int)(i & 3);
  uint32_t old = atomicOr(word, 1u << sh);
  return ((old >> sh) & 0xffu) == 0;
}

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

__global__ void k_clear_list(uint8_t *act, const int64_t *list, uint32_t *cnt, int B) {
  int64_t N = *cnt;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t x = list[i];
    act[(x >> 6) * B + (x & 63)] = 0;
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
  const int sa = nt.val ? nt.s : 1, se = et.val ? et.s : 2;
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
      if (grp.dense) dst.act[ent] = 1;
      else {
        set_act(dst.act, ent);
        uint32_t pos = atomicAdd(dst.cnt, 1u);
        dst.list[pos] = x * 64 + b;
      }
    }
    int64_t tslot = e_src_first ? es : g.rev[es];
    for (int it = lane; it < items; it += P) {
      int t = it / C, c = it - t * C;
      int cu = colr[(int64_t)t * g.n + u], cx = colr[(int64_t)t * g.n + x];
      uint64_t acc = 0;
      bool of = false;
      if (cu != cx) {
        uint32_t R = spread2(unrank(lut, dst.s - 2, c), cu, cx);
        // enumerate Ra (node table part, size sa-1)
        uint32_t sub_ = R;
        for (;;) {
          if (__popc(sub_) == sa - 1) {
            uint32_t Re = R & ~sub_;
            uint64_t va = nt.val ? nt.val[((int64_t)u * T + t) * nt.C + s_rank[squeeze1(sub_, cu)]] : 1;
            uint64_t ve = et.val ? et.val[(tslot * T + t) * et.C + s_rank[squeeze2(Re, cu, cx)]] : 1;
            if (va && ve) add_ck(acc, mul_ck(va, ve, of), of);
          }
          if (sub_ == 0) break;
          sub_ = (sub_ - 1) & R;
        }
        (void)se;
      }
      dst.val[(ent * T + t) * C + c] = acc;
      if (of) atomicOr(&ovf[t], 1u);
    }
  }
}

// ------------------------------------------------------------------ MARK (sparse EdgeJoin, structure)
__global__ void k_mark(GraphDev g, GroupDev grp, RegDev a, RegDev dst) {
  const int64_t N = *a.cnt;
  const int P = 16;
  const int epb = blockDim.x / P, lane = threadIdx.x % P, sub = threadIdx.x / P;
  const int B = grp.B;
  for (int64_t e0 = (int64_t)blockIdx.x * epb; e0 < N; e0 += (int64_t)gridDim.x * epb) {
    int64_t en = e0 + sub;
    if (en >= N) continue;
    int64_t xv = a.list[en];
    int64_t v = xv >> 6;
    int b = (int)(xv & 63);
    int64_t u = grp.src[b];
    for (int64_t e = g.rp[v] + lane; e < g.rp[v + 1]; e += P) {
      int64_t w = g.col[e];
      if (w >= u) break;
      if (set_act(dst.act, w * B + b)) {
        uint32_t pos = atomicAdd(dst.cnt, 1u);
        dst.list[pos] = w * 64 + b;
      }
    }
  }
}

// ------------------------------------------------------------------ EdgeJoin (pull)
// dst[w][b][R'] = sum over v in N(w), v < u_b, (v,b) active in a, of
//                 sum over splits R' \ {chi v} = R + Re of a[v][b][R] * E(v,w)[Re].
__global__ void k_ej(GraphDev g, GroupDev grp, const uint8_t *colr, RegDev a, RegDev dst, TabDev et,
                     int e_src_first, uint32_t *ovf, const uint16_t *lut, int P) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int epb = blockDim.x / P, lane = threadIdx.x % P, sub = threadIdx.x / P;
  const int C = dst.C, Ca = a.C, T = grp.T, B = grp.B;
  const int items = T * C;
  const int64_t N = domain_size(grp, dst.cnt);
  const int ra = a.s - 2;  // size of a's rest
  for (int64_t e0 = (int64_t)blockIdx.x * epb; e0 < N; e0 += (int64_t)gridDim.x * epb) {
    int64_t en = e0 + sub;
    if (en >= N) continue;
    int64_t w;
    int b;
    decode(grp, dst.list, en, w, b);
    int64_t u = grp.src[b];
    int64_t ent = w * B + b;
    if (w >= u) {
      if (grp.dense && lane == 0) dst.act[ent] = 0;
      continue;
    }
    bool any = false;
    const int64_t rs = g.rp[w], re = g.rp[w + 1];
    for (int it = lane; it < items; it += P) {
      int t = it / C, c = it - t * C;
      int cu = colr[(int64_t)t * g.n + u], cw = colr[(int64_t)t * g.n + w];
      uint64_t acc = 0;
      bool of = false;
      uint32_t Rp = cu != cw ? spread2(unrank(lut, dst.s - 2, c), cu, cw) : 0u;
      for (int64_t e = rs; e < re; e++) {
        int64_t v = g.col[e];
        if (v >= u) break;
        if (!a.act[v * B + b]) continue;
        any = true;
        if (cu == cw) continue;
        int cv = colr[(int64_t)t * g.n + v];
        if (!((Rp >> cv) & 1u)) continue;
        uint32_t R = Rp & ~(1u << cv);
        const uint64_t *av = a.val + ((v * B + b) * T + t) * Ca;
        if (!et.val) {
          add_ck(acc, av[s_rank[squeeze2(R, cu, cv)]], of);
        } else {
          int64_t tslot = e_src_first ? g.rev[e] : e;
          const uint64_t *ev = et.val + (tslot * T + t) * et.C;
          uint32_t s1 = R;
          for (;;) {
            if (__popc(s1) == ra) {
              uint64_t x = av[s_rank[squeeze2(s1, cu, cv)]];
              if (x) {
                uint64_t y = ev[s_rank[squeeze2(R & ~s1, cv, cw)]];
                if (y) add_ck(acc, mul_ck(x, y, of), of);
              }
            }
            if (s1 == 0) break;
            s1 = (s1 - 1) & R;
          }
        }
      }
      dst.val[(ent * T + t) * C + c] = acc;
      if (of) atomicOr(&ovf[t], 1u);
    }
    if (grp.dense && lane == 0) dst.act[ent] = any ? 1 : 0;
  }
}

// ------------------------------------------------------------------ NodeJoin
// dst[v][b][R'] = sum over splits R' = R + Ra of a[v][b][R] * A[v][Ra]
__global__ void k_nj(GroupDev grp, int64_t n, const uint8_t *colr, RegDev a, RegDev dst, TabDev nt,
                     uint32_t *ovf, const uint16_t *lut, int P) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int epb = blockDim.x / P, lane = threadIdx.x % P, sub = threadIdx.x / P;
  const int C = dst.C, Ca = a.C, T = grp.T, B = grp.B;
  const int items = T * C;
  const int64_t N = domain_size(grp, a.cnt);
  const int rA = nt.s - 1;
  for (int64_t e0 = (int64_t)blockIdx.x * epb; e0 < N; e0 += (int64_t)gridDim.x * epb) {
    int64_t en = e0 + sub;
    if (en >= N) continue;
    int64_t v;
    int b;
    decode(grp, a.list, en, v, b);
    int64_t ent = v * B + b;
    if (grp.dense && !a.act[ent]) continue;
    int64_t u = grp.src[b];
    for (int it = lane; it < items; it += P) {
      int t = it / C, c = it - t * C;
      int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
      uint64_t acc = 0;
      bool of = false;
      if (cu != cv) {
        uint32_t Rp = spread2(unrank(lut, dst.s - 2, c), cu, cv);
        const uint64_t *av = a.val + (ent * T + t) * Ca;
        const uint64_t *nv = nt.val + ((int64_t)v * T + t) * nt.C;
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
      if (of) atomicOr(&ovf[t], 1u);
    }
  }
}

// ------------------------------------------------------------------ AXPY
// Sparse mode, phase 1: give dst an entry (zeroed) for every entry of a.
__global__ void k_axpy_mark(GroupDev grp, RegDev a, RegDev dst) {
  const int64_t N = *a.cnt;
  const int T = grp.T, C = dst.C, B = grp.B;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t x = a.list[i];
    int64_t ent = (x >> 6) * B + (x & 63);
    if (set_act(dst.act, ent)) {
      uint32_t pos = atomicAdd(dst.cnt, 1u);
      dst.list[pos] = x;
      uint64_t *d = dst.val + ent * T * C;
      for (int j = 0; j < T * C; j++) d[j] = 0;
    }
  }
}

// dst += w * a over a's entries.  Dense mode with `first`: the whole domain
// is written (w * a where a is active, 0 elsewhere).
__global__ void k_axpy(GroupDev grp, RegDev a, RegDev dst, uint64_t w, int first, uint32_t *ovf) {
  const int T = grp.T, C = dst.C, B = grp.B;
  const int64_t per = (int64_t)T * C;
  const int64_t N = domain_size(grp, a.cnt) * per;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t en = i / per;
    int64_t r = i - en * per;
    int64_t v;
    int b;
    decode(grp, a.list, en, v, b);
    int64_t ent = v * B + b;
    bool act = a.act[ent] != 0;
    if (grp.dense) {
      if (!act && !first) continue;
      bool of = false;
      uint64_t x = act ? mul_ck(w, a.val[ent * per + r], of) : 0;
      if (first) {
        dst.val[ent * per + r] = x;
      } else {
        uint64_t y = dst.val[ent * per + r];
        add_ck(y, x, of);
        dst.val[ent * per + r] = y;
      }
      if (r == 0) {
        if (first) dst.act[ent] = act ? 1 : 0;
        else if (act) dst.act[ent] = 1;
      }
      if (of) atomicOr(&ovf[(int)(r / C)], 1u);
    } else {
      bool of = false;
      uint64_t y = dst.val[ent * per + r];
      add_ck(y, mul_ck(w, a.val[ent * per + r], of), of);
      dst.val[ent * per + r] = y;
      if (of) atomicOr(&ovf[(int)(r / C)], 1u);
    }
  }
}

// ------------------------------------------------------------------ root merge
// count[t] += w * sum over (v, b) active in both, of
//             sum over R of a[v][b][R] * b[v][b][K \ {chi u, chi v} \ R]
__global__ void k_mroot(GroupDev grp, int64_t n, const uint8_t *colr, RegDev a, RegDev bb, uint64_t w,
                        AccDev acc, const uint16_t *lut, int P) {
  __shared__ uint16_t s_rank[2048];
  __shared__ uint64_t s_acc[2 * 64];
  for (int i = threadIdx.x; i < 2 * 64; i += blockDim.x) s_acc[i] = 0;
  load_rank(s_rank, lut);
  const int epb = blockDim.x / P, lane = threadIdx.x % P, sub = threadIdx.x / P;
  const int Ca = a.C, Cb = bb.C, T = grp.T, B = grp.B, k = grp.k;
  const int items = T * Ca;
  const int64_t N = domain_size(grp, a.cnt);
  const uint32_t Kmask = (1u << k) - 1u;
  for (int64_t e0 = (int64_t)blockIdx.x * epb; e0 < N; e0 += (int64_t)gridDim.x * epb) {
    int64_t en = e0 + sub;
    if (en >= N) continue;
    int64_t v;
    int b;
    decode(grp, a.list, en, v, b);
    int64_t ent = v * B + b;
    if (!a.act[ent] || !bb.act[ent]) continue;
    int64_t u = grp.src[b];
    for (int it = lane; it < items; it += P) {
      int t = it / Ca, c = it - t * Ca;
      int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
      if (cu == cv) continue;
      uint64_t x = a.val[(ent * T + t) * Ca + c];
      if (!x) continue;
      uint32_t R1 = spread2(unrank(lut, a.s - 2, c), cu, cv);
      uint32_t R2 = Kmask & ~R1 & ~(1u << cu) & ~(1u << cv);
      uint64_t y = bb.val[(ent * T + t) * Cb + s_rank[squeeze2(R2, cu, cv)]];
      if (!y) continue;
      uint64_t lo = x * y, hi = __umul64hi(x, y);
      if (w != 1) {
        uint64_t lo2 = lo * w, c2 = __umul64hi(lo, w);
        uint64_t hi2 = hi * w + c2;
        if (__umul64hi(hi, w) != 0 || hi2 < c2) atomicOr(&acc.ovf[t], 1u);
        lo = lo2;
        hi = hi2;
      }
      atomic_add128(&s_acc[2 * t], lo, hi);
      if (acc.per_src) atomic_add128(&acc.per_src[2 * (u * T + t)], lo, hi);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += blockDim.x) atomic_add128(&acc.sum[2 * t], s_acc[2 * t], s_acc[2 * t + 1]);
}

// ------------------------------------------------------------------ merges into unary tables
// MU: out[u_b][R'] += w * sum_v sum over splits of R' \ {chi v} of a[v][b][.] * b[v][b][.]
// MV: out[v][R']   += w * sum_b sum over splits of R' \ {chi u}  (same products)
template <bool AT_U>
__global__ void k_munary(GroupDev grp, int64_t n, const uint8_t *colr, RegDev a, RegDev bb, uint64_t w,
                         uint64_t *out, int s_out, int C_out, uint32_t *ovf, const uint16_t *lut, int P) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int epb = blockDim.x / P, lane = threadIdx.x % P, sub = threadIdx.x / P;
  const int Ca = a.C, Cb = bb.C, T = grp.T, B = grp.B;
  const int items = T * C_out;
  const int64_t N = domain_size(grp, a.cnt);
  const int ra = a.s - 2;
  for (int64_t e0 = (int64_t)blockIdx.x * epb; e0 < N; e0 += (int64_t)gridDim.x * epb) {
    int64_t en = e0 + sub;
    if (en >= N) continue;
    int64_t v;
    int b;
    decode(grp, a.list, en, v, b);
    int64_t ent = v * B + b;
    if (!a.act[ent] || !bb.act[ent]) continue;
    int64_t u = grp.src[b];
    for (int it = lane; it < items; it += P) {
      int t = it / C_out, c = it - t * C_out;
      int cu = colr[(int64_t)t * n + u], cv = colr[(int64_t)t * n + v];
      if (cu == cv) continue;
      int ckey = AT_U ? cu : cv, cother = AT_U ? cv : cu;
      uint32_t Rp = spread1(unrank(lut, s_out - 1, c), ckey);
      if (!((Rp >> cother) & 1u)) continue;
      uint32_t R = Rp & ~(1u << cother);
      const uint64_t *av = a.val + (ent * T + t) * Ca;
      const uint64_t *bv = bb.val + (ent * T + t) * Cb;
      uint64_t s = 0;
      bool of = false;
      uint32_t s1 = R;
      for (;;) {
        if (__popc(s1) == ra) {
          uint64_t x = av[s_rank[squeeze2(s1, cu, cv)]];
          if (x) {
            uint64_t y = bv[s_rank[squeeze2(R & ~s1, cu, cv)]];
            if (y) add_ck(s, mul_ck(x, y, of), of);
          }
        }
        if (s1 == 0) break;
        s1 = (s1 - 1) & R;
      }
      if (s) {
        s = mul_ck(s, w, of);
        int64_t key = AT_U ? u : v;
        atomic_add_ck(&out[((int64_t)key * T + t) * C_out + c], s, of);
      }
      if (of) atomicOr(&ovf[t], 1u);
    }
  }
}

// ------------------------------------------------------------------ edge merge
// T[x,y][R'] += w * a[x][b][R1] * E(x,y)[Re] * b[y][b][R2],  R' \ {chi u} = R1 + Re + R2
__global__ void k_medge(GraphDev g, GroupDev grp, const uint8_t *colr, RegDev a, RegDev bb, TabDev et,
                        int e_src_first, int out_first_is_x, uint64_t w, uint64_t *out, int s_out, int C_out,
                        uint32_t *ovf, const uint16_t *lut, int P) {
  __shared__ uint16_t s_rank[2048];
  load_rank(s_rank, lut);
  const int epb = blockDim.x / P, lane = threadIdx.x % P, sub = threadIdx.x / P;
  const int Ca = a.C, Cb = bb.C, T = grp.T, B = grp.B;
  const int items = T * C_out;
  const int64_t N = domain_size(grp, a.cnt);
  const int ra = a.s - 2, rb = bb.s - 2;
  for (int64_t e0 = (int64_t)blockIdx.x * epb; e0 < N; e0 += (int64_t)gridDim.x * epb) {
    int64_t en = e0 + sub;
    if (en >= N) continue;
    int64_t x;
    int b;
    decode(grp, a.list, en, x, b);
    int64_t entx = x * B + b;
    if (!a.act[entx]) continue;
    int64_t u = grp.src[b];
    for (int64_t e = g.rp[x]; e < g.rp[x + 1]; e++) {
      int64_t y = g.col[e];
      if (y >= u) break;
      int64_t enty = y * B + b;
      if (!bb.act[enty]) continue;
      int64_t tslot = e_src_first ? e : g.rev[e];
      int64_t oslot = out_first_is_x ? e : g.rev[e];
      for (int it = lane; it < items; it += P) {
        int t = it / C_out, c = it - t * C_out;
        int cu = colr[(int64_t)t * g.n + u], cx = colr[(int64_t)t * g.n + x], cy = colr[(int64_t)t * g.n + y];
        if (cx == cy || cu == cx || cu == cy) continue;
        uint32_t Rp = spread2(unrank(lut, s_out - 2, c), cx, cy);
        if (!((Rp >> cu) & 1u)) continue;
        uint32_t R = Rp & ~(1u << cu);
        const uint64_t *av = a.val + (entx * T + t) * Ca;
        const uint64_t *bv = bb.val + (enty * T + t) * Cb;
        const uint64_t *ev = et.val ? et.val + (tslot * T + t) * et.C : nullptr;
        uint64_t s = 0;
        bool of = false;
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
        if (s) {
          s = mul_ck(s, w, of);
          atomic_add_ck(&out[(oslot * T + t) * C_out + c], s, of);
        }
        if (of) atomicOr(&ovf[t], 1u);
      }
    }
  }
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
        s = mul_ck(s, w, of);
        atomic_add_ck(&out[(oslot * T + t) * C_out + c], s, of);
      }
      if (of) atomicOr(&ovf[t], 1u);
    }
  }
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
      if (of) atomicOr(&ovf[t], 1u);
    }
  }
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
inline int grid_for(int64_t entries, int P, bool known) {
  if (!known) return 2048;
  int epb = BLK / P;
  int64_t g = (entries + epb - 1) / epb;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

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
  hipLaunchKernelGGL(k_clear_list, dim3(1024), dim3(BLK), 0, st, r.act, r.list, r.cnt, B);
  hipLaunchKernelGGL(k_reset_cnt, dim3(1), dim3(1), 0, st, r.cnt);
}

void launch_init(const GraphDev &g, const GroupDev &grp, const int32_t *lowcnt, int max_low, const uint8_t *colr,
                 RegDev dst, TabDev etab, int e_src_first, TabDev ntab, uint32_t *ovf, hipStream_t st) {
  int P = pick_p(grp.T * dst.C);
  int64_t N = (int64_t)grp.B * max_low;
  hipLaunchKernelGGL(k_init, dim3(grid_for(N, P, true)), dim3(BLK), 0, st, g, grp, lowcnt, max_low, colr, dst, etab,
                     e_src_first, ntab, ovf, cur_lut(), P);
}
void launch_mark(const GraphDev &g, const GroupDev &grp, RegDev a, RegDev dst, hipStream_t st) {
  hipLaunchKernelGGL(k_mark, dim3(2048), dim3(BLK), 0, st, g, grp, a, dst);
}
void launch_ej(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, RegDev a, RegDev dst, TabDev etab,
               int e_src_first, uint32_t *ovf, hipStream_t st) {
  int P = pick_p(grp.T * dst.C);
  hipLaunchKernelGGL(k_ej, dim3(grid_for(grp.n_lim * grp.B, P, grp.dense)), dim3(BLK), 0, st, g, grp, colr, a, dst,
                     etab, e_src_first, ovf, cur_lut(), P);
}
void launch_nj(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, RegDev a, RegDev dst, TabDev ntab,
               uint32_t *ovf, hipStream_t st) {
  int P = pick_p(grp.T * dst.C);
  hipLaunchKernelGGL(k_nj, dim3(grid_for(grp.n_lim * grp.B, P, grp.dense)), dim3(BLK), 0, st, grp, g.n, colr, a,
                     dst, ntab, ovf, cur_lut(), P);
}
void launch_axpy(const GroupDev &grp, RegDev a, RegDev dst, uint64_t w, int first, uint32_t *ovf, hipStream_t st) {
  if (!grp.dense) hipLaunchKernelGGL(k_axpy_mark, dim3(1024), dim3(BLK), 0, st, grp, a, dst);
  int64_t tot = grp.n_lim * grp.B * (int64_t)grp.T * dst.C;
  int g = grp.dense ? (int)std::min<int64_t>((tot + BLK - 1) / BLK, 65536) : 2048;
  hipLaunchKernelGGL(k_axpy, dim3(std::max(1, g)), dim3(BLK), 0, st, grp, a, dst, w, first, ovf);
}
void launch_mroot(const GroupDev &grp, int64_t n, const uint8_t *colr, RegDev a, RegDev b, uint64_t w,
                  AccDev acc, hipStream_t st) {
  int P = pick_p(grp.T * a.C);
  hipLaunchKernelGGL(k_mroot, dim3(grid_for(grp.n_lim * grp.B, P, grp.dense)), dim3(BLK), 0, st, grp, n, colr, a, b,
                     w, acc, cur_lut(), P);
}
void launch_mu(const GroupDev &grp, int64_t n, const uint8_t *colr, RegDev a, RegDev b, uint64_t w, uint64_t *out,
               int s_out, int C_out, uint32_t *ovf, hipStream_t st) {
  int P = pick_p(grp.T * C_out);
  hipLaunchKernelGGL(k_munary<true>, dim3(grid_for(grp.n_lim * grp.B, P, grp.dense)), dim3(BLK), 0, st, grp, n,
                     colr, a, b, w, out, s_out, C_out, ovf, cur_lut(), P);
}
void launch_mv(const GroupDev &grp, int64_t n, const uint8_t *colr, RegDev a, RegDev b, uint64_t w, uint64_t *out,
               int s_out, int C_out, uint32_t *ovf, hipStream_t st) {
  int P = pick_p(grp.T * C_out);
  hipLaunchKernelGGL(k_munary<false>, dim3(grid_for(grp.n_lim * grp.B, P, grp.dense)), dim3(BLK), 0, st, grp, n,
                     colr, a, b, w, out, s_out, C_out, ovf, cur_lut(), P);
}
void launch_medge(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, RegDev a, RegDev b, TabDev etab,
                  int e_src_first, int out_first_is_x, uint64_t w, uint64_t *out, int s_out, int C_out,
                  uint32_t *ovf, hipStream_t st) {
  int P = pick_p(grp.T * C_out);
  hipLaunchKernelGGL(k_medge, dim3(grid_for(grp.n_lim * grp.B, P, grp.dense)), dim3(BLK), 0, st, g, grp, colr, a, b,
                     etab, e_src_first, out_first_is_x, w, out, s_out, C_out, ovf, cur_lut(), P);
}
void launch_medge_t(const GraphDev &g, const GroupDev &grp, const uint8_t *colr, const int32_t *lowcnt,
                    int max_low, TabDev ntab, RegDev b, TabDev etab, int e_src_first, int out_first_is_u,
                    uint64_t w, uint64_t *out, int s_out, int C_out, uint32_t *ovf, hipStream_t st) {
  int P = pick_p(grp.T * C_out);
  int64_t N = (int64_t)grp.B * max_low;
  hipLaunchKernelGGL(k_medge_t, dim3(grid_for(N, P, true)), dim3(BLK), 0, st, g, grp, colr, lowcnt, max_low, ntab,
                     b, etab, e_src_first, out_first_is_u, w, out, s_out, C_out, ovf, cur_lut(), P);
}
void launch_leaf(const GraphDev &g, int T, int k, const uint8_t *colr, TabDev na, TabDev ea, int e_src_first,
                 TabDev nb, uint64_t *out, int s_out, int C_out, uint32_t *ovf, hipStream_t st) {
  (void)k;
  int P = pick_p(T * C_out);
  hipLaunchKernelGGL(k_leaf, dim3(grid_for(g.n, P, true)), dim3(BLK), 0, st, g, T, colr, na, ea, e_src_first, nb,
                     out, s_out, C_out, ovf, cur_lut(), P);
}
void launch_root_single(int64_t n, int T, TabDev u, AccDev acc, hipStream_t st) {
  int64_t g = std::min<int64_t>((n * T + BLK - 1) / BLK, 8192);
  hipLaunchKernelGGL(k_root_single, dim3((unsigned)std::max<int64_t>(1, g)), dim3(BLK), 0, st, n, T, u, acc);
}

}  // namespace cc
