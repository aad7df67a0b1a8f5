// One-workgroup-per-source path for sources with small high-starting reach.
//
// Most sources of a power-law graph have few lower neighbours, so the
// vertices their high-starting paths reach are few.  For those, a single
// workgroup runs the whole frontier program of a cycle block for one source
// at a time.  The key vertices at each path length (depth) are built once,
// sorted, in LDS: they are the same for every register of that depth, since
// the vertices a high-starting walk of a given length reaches do not depend
// on colours or annotations.  For every step the list of (key, lower-depth
// key) matches is kept with it.  The values of every register live in a
// per-workgroup slice of global scratch.  Sources are taken from a shared
// counter; a source whose keys or matches do not fit is handed back, before
// any output is written, to the grouped path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "kernels.h"
#include "slot_math.h"

namespace cc {

namespace {

using namespace dev;

// Two sizes: the small one (keys 6144, expansion buffer 4096) keeps several
// workgroups per compute unit for the many small sources; the large one
// (16384 / 16384, most of a compute unit's 160 KiB of LDS) takes what the
// small one hands back.
constexpr int KPOOL_S = 6144, EMAX_S = 4096;
constexpr int KPOOL_L = 16384, EMAX_L = 16384;
constexpr int DMAX = 12;
constexpr int RMAX = 64;     // registers per program

__device__ __forceinline__ int find_key(const int32_t *k, int n, int32_t v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (k[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && k[lo] == v) ? lo : -1;
}

// exclusive scan of a[0..n) in place; returns the total.  s_part holds BLK+1.
__device__ int64_t block_scan(int32_t *a, int n, int64_t *s_part) {
  const int per = (n + BLK - 1) / BLK;
  const int lo = min(n, (int)threadIdx.x * per), hi = min(n, lo + per);
  int64_t sum = 0;
  for (int i = lo; i < hi; i++) sum += a[i];
  s_part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < BLK; i++) {
      int64_t x = s_part[i];
      s_part[i] = run;
      run += x;
    }
    s_part[BLK] = run;
  }
  __syncthreads();
  int64_t run = s_part[threadIdx.x];
  for (int i = lo; i < hi; i++) {
    int32_t x = a[i];
    a[i] = (int32_t)run;
    run += x;
  }
  const int64_t tot = s_part[BLK];
  __syncthreads();
  return tot;
}

__device__ void bitonic(int32_t *s, int n2) {
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += BLK) {
        int ixj = i ^ j;
        if (ixj > i) {
          bool up = (i & k) == 0;
          int32_t a = s[i], b = s[ixj];
          if ((a > b) == up) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
}

__device__ __forceinline__ int64_t align8(int64_t x) { return (x + 7) & ~(int64_t)7; }

template <int KPOOL, int EMAX>
__global__ __launch_bounds__(BLK) void k_light(LightArgs A) {
  __shared__ uint16_t s_rank[2048];
  __shared__ int32_t s_k[KPOOL];   // keys over all depths
  __shared__ int32_t s_c[EMAX];    // expansion buffer (with duplicates)
  __shared__ int s_koff[DMAX + 2];
  __shared__ int64_t s_mo[DMAX][3];  // per step: offsets of the match offsets, key positions, slots
  __shared__ int64_t s_roff[RMAX];
  __shared__ int64_t s_part[BLK + 1];
  __shared__ uint64_t s_acc[2 * 64];
  __shared__ int s_si, s_n, s_fail;
  load_rank(s_rank, A.lut);
  const GraphDev &g = A.g;
  const int T = A.T, k = A.k;
  const uint32_t Kmask = (1u << k) - 1u;
  uint8_t *base = A.scratch + (int64_t)blockIdx.x * A.scratch_per_wg;
  // profiling (A.prof set): algorithmic bytes read and written by this
  // thread, counted as in the grouped kernels (rows of the registers and
  // tables, 4 B per scanned neighbour)
  uint64_t prd = 0, pwr = 0;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      s_si = (int)atomicAdd(A.next, 1u);
      s_fail = 0;
    }
    for (int i = threadIdx.x; i < 2 * 64; i += BLK) s_acc[i] = 0;
    __syncthreads();
    const int si = s_si;
    if (si >= A.nsrc) break;
    const int64_t u = A.src[si];
    // later path vertices lie below u (degree order), or anywhere with the filter off
    const int64_t ub = A.nofilter ? (int64_t)INT_MAX : u;
    // ------------------------------------------------ structure
    const int n1 = A.lowcnt[u];
    if (n1 > KPOOL) {
      if (threadIdx.x == 0) s_fail = 1;
    } else {
      for (int i = threadIdx.x; i < n1; i += BLK) s_k[i] = g.col[g.rp[u] + i];
      if (threadIdx.x == 0) {
        s_koff[0] = 0;
        s_koff[1] = n1;
      }
    }
    __syncthreads();
    int64_t cur = 0;
    for (int j = 1; j < A.D && !s_fail; j++) {
      const int k0 = s_koff[j - 1], k1 = s_koff[j];
      if (threadIdx.x == 0) s_n = 0;
      __syncthreads();
      for (int i = k0 + threadIdx.x; i < k1; i += BLK) {
        int64_t v = s_k[i];
        if (A.prof) prd += 16;
        for (int64_t e = g.rp[v]; e < g.rp[v + 1]; e++) {
          int32_t w = g.col[e];
          if (w >= ub) break;
          if (A.prof) prd += 4;
          int pos = atomicAdd(&s_n, 1);
          if (pos < EMAX) s_c[pos] = w;
        }
      }
      __syncthreads();
      const int nc = s_n;
      if (nc > EMAX) {
        if (threadIdx.x == 0) s_fail = 1;
        __syncthreads();
        break;
      }
      int n2 = 1;
      while (n2 < nc) n2 <<= 1;
      for (int i = nc + threadIdx.x; i < n2; i += BLK) s_c[i] = INT_MAX;
      __syncthreads();
      bitonic(s_c, n2);
      // unique keys, in order, appended at s_k[k1..)
      {
        const int per = (nc + BLK - 1) / BLK;
        const int lo = min(nc, (int)threadIdx.x * per), hi = min(nc, lo + per);
        int cnt = 0;
        for (int i = lo; i < hi; i++) cnt += (i == 0 || s_c[i] != s_c[i - 1]);
        s_part[threadIdx.x] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
          int64_t run = 0;
          for (int i = 0; i < BLK; i++) {
            int64_t x = s_part[i];
            s_part[i] = run;
            run += x;
          }
          s_part[BLK] = run;
          if (k1 + run > KPOOL) s_fail = 1;
          else s_koff[j + 1] = k1 + (int)run;
        }
        __syncthreads();
        if (!s_fail) {
          int o = k1 + (int)s_part[threadIdx.x];
          for (int i = lo; i < hi; i++)
            if (i == 0 || s_c[i] != s_c[i - 1]) s_k[o++] = s_c[i];
        }
        __syncthreads();
      }
      if (s_fail) break;
      // matches of step j -> j+1: for each key w, its lower-depth neighbours
      const int nn = s_koff[j + 1] - k1;
      const int64_t o_off = align8(cur);
      const int64_t o_p = align8(o_off + 4 * (int64_t)(nn + 1));
      if (o_p > A.scratch_per_wg) {
        if (threadIdx.x == 0) s_fail = 1;
        __syncthreads();
        break;
      }
      int32_t *offs = (int32_t *)(base + o_off);
      for (int wi = threadIdx.x; wi < nn; wi += BLK) {
        int64_t w = s_k[k1 + wi];
        int c = 0;
        for (int64_t e = g.rp[w]; e < g.rp[w + 1]; e++) {
          int32_t v = g.col[e];
          if (v >= ub) break;
          c += find_key(s_k + k0, k1 - k0, v) >= 0;
        }
        offs[wi] = c;
      }
      __syncthreads();
      const int64_t M = block_scan(offs, nn, s_part);
      const int64_t o_e = align8(o_p + 4 * M);
      const int64_t end = o_e + 8 * M;
      if (end > A.scratch_per_wg) {
        if (threadIdx.x == 0) s_fail = 1;
        __syncthreads();
        break;
      }
      if (threadIdx.x == 0) {
        offs[nn] = (int32_t)M;
        s_mo[j][0] = o_off;
        s_mo[j][1] = o_p;
        s_mo[j][2] = o_e;
      }
      int32_t *mp = (int32_t *)(base + o_p);
      int64_t *me = (int64_t *)(base + o_e);
      for (int wi = threadIdx.x; wi < nn; wi += BLK) {
        int64_t w = s_k[k1 + wi];
        int pos = offs[wi];
        for (int64_t e = g.rp[w]; e < g.rp[w + 1]; e++) {
          int32_t v = g.col[e];
          if (v >= ub) break;
          int q = find_key(s_k + k0, k1 - k0, v);
          if (q >= 0) {
            mp[pos] = q;
            me[pos] = e;
            pos++;
          }
        }
      }
      cur = end;
      __syncthreads();
    }
    if (!s_fail && threadIdx.x == 0) {
      int64_t c2 = align8(cur);
      for (int r = 0; r < A.nregs; r++) {
        int d = A.reg_depth[r];
        int64_t nk = s_koff[d] - s_koff[d - 1];
        s_roff[r] = c2;
        c2 = align8(c2 + 8 * nk * T * A.reg_C[r]);
      }
      if (c2 > A.scratch_per_wg) s_fail = 1;
    }
    __syncthreads();
    if (s_fail) {
      if (threadIdx.x == 0) {
        uint32_t pos = atomicAdd(A.nfail, 1u);
        A.fail[pos] = (int32_t)u;
      }
      continue;
    }
    // ------------------------------------------------ values
    for (int oi = 0; oi < A.nops; oi++) {
      const LOp op = A.ops[oi];
      uint64_t ofm = 0;
      if (op.kind == OP_INIT) {
        const int C = A.reg_C[op.dst], s = A.reg_s[op.dst];
        uint64_t *dv = (uint64_t *)(base + s_roff[op.dst]);
        const TabDev et = op.tab >= 0 ? A.tabs[op.tab] : TabDev{nullptr, 0, 0};
        const TabDev nt = op.ntab >= 0 ? A.tabs[op.ntab] : TabDev{nullptr, 0, 0};
        const int sa = nt.val ? nt.s : 1;
        for (int it = threadIdx.x; it < n1 * T * C; it += BLK) {
          const int xi = it / (T * C), r = it - xi * T * C, t = r / C, c = r - t * C;
          const int64_t es = g.rp[u] + xi;
          const int64_t x = s_k[xi];
          const int cu = A.colr[(int64_t)t * g.n + u], cx = A.colr[(int64_t)t * g.n + x];
          const int64_t tslot = op.tab_src_first ? es : g.rev[es];
          uint64_t acc = 0;
          bool of = false;
          if (cu != cx) {
            const uint32_t R = spread2(unrank(A.lut, s - 2, c), cu, cx);
            uint32_t sub = R;
            for (;;) {
              if (__popc(sub) == sa - 1) {
                uint32_t Re = R & ~sub;
                uint64_t va = nt.val ? nt.val[((int64_t)u * T + t) * nt.C + s_rank[squeeze1(sub, cu)]] : 1;
                uint64_t ve = et.val ? et.val[(tslot * T + t) * et.C + s_rank[squeeze2(Re, cu, cx)]] : (Re ? 0 : 1);
                if (va && ve) add_ck(acc, mul_ck(va, ve, of), of);
              }
              if (sub == 0) break;
              sub = (sub - 1) & R;
            }
          }
          dv[(int64_t)xi * T * C + t * C + c] = acc;
          if (of) ofm |= 1ull << t;
          if (A.prof) {
            pwr += 8;
            if (c == 0) prd += 4 + 2 + 8 * ((nt.val ? nt.C : 0) + (et.val ? et.C : 0));
          }
        }
      } else if (op.kind == OP_NJ) {
        const int d = A.reg_depth[op.a];
        const int kk0 = s_koff[d - 1], nk = s_koff[d] - kk0;
        const int C = A.reg_C[op.dst], Ca = A.reg_C[op.a], s = A.reg_s[op.dst];
        const uint64_t *av = (const uint64_t *)(base + s_roff[op.a]);
        uint64_t *dv = (uint64_t *)(base + s_roff[op.dst]);
        const TabDev nt = A.tabs[op.tab];
        const int rA = nt.s - 1;
        for (int it = threadIdx.x; it < nk * T * C; it += BLK) {
          const int i = it / (T * C), r = it - i * T * C, t = r / C, c = r - t * C;
          const int64_t v = s_k[kk0 + i];
          const int cu = A.colr[(int64_t)t * g.n + u], cv = A.colr[(int64_t)t * g.n + v];
          uint64_t acc = 0;
          bool of = false;
          if (cu != cv) {
            const uint32_t Rp = spread2(unrank(A.lut, s - 2, c), cu, cv);
            const uint64_t *ar = av + ((int64_t)i * T + t) * Ca;
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
          dv[((int64_t)i * T + t) * C + c] = acc;
          if (of) ofm |= 1ull << t;
          if (A.prof) {
            pwr += 8;
            if (c == 0 && cu != cv) prd += 8 * (uint64_t)(Ca + nt.C);
          }
        }
      } else if (op.kind == OP_EJ) {
        const int j = A.reg_depth[op.a];
        const int kk0 = s_koff[j - 1], kk1 = s_koff[j], nn = s_koff[j + 1] - kk1;
        const int C = A.reg_C[op.dst], Ca = A.reg_C[op.a], s = A.reg_s[op.dst], ra = A.reg_s[op.a] - 2;
        const uint64_t *av = (const uint64_t *)(base + s_roff[op.a]);
        uint64_t *dv = (uint64_t *)(base + s_roff[op.dst]);
        const int32_t *offs = (const int32_t *)(base + s_mo[j][0]);
        const int32_t *mp = (const int32_t *)(base + s_mo[j][1]);
        const int64_t *me = (const int64_t *)(base + s_mo[j][2]);
        const TabDev et = op.tab >= 0 ? A.tabs[op.tab] : TabDev{nullptr, 0, 0};
        for (int it = threadIdx.x; it < nn * T * C; it += BLK) {
          const int wi = it / (T * C), r = it - wi * T * C, t = r / C, c = r - t * C;
          const int64_t w = s_k[kk1 + wi];
          const int cu = A.colr[(int64_t)t * g.n + u], cw = A.colr[(int64_t)t * g.n + w];
          uint64_t acc = 0;
          bool of = false;
          if (cu != cw) {
            const uint32_t Rp = spread2(unrank(A.lut, s - 2, c), cu, cw);
            for (int m = offs[wi]; m < offs[wi + 1]; m++) {
              const int p = mp[m];
              const int64_t v = s_k[kk0 + p];
              const int cv = A.colr[(int64_t)t * g.n + v];
              if (!((Rp >> cv) & 1u)) continue;
              const uint32_t R = Rp & ~(1u << cv);
              const uint64_t *ar = av + ((int64_t)p * T + t) * Ca;
              if (!et.val) {
                add_ck(acc, ar[s_rank[squeeze2(R, cu, cv)]], of);
              } else {
                const int64_t e = me[m];
                const int64_t tslot = op.tab_src_first ? g.rev[e] : e;
                const uint64_t *er = et.val + (tslot * T + t) * et.C;
                uint32_t s1 = R;
                for (;;) {
                  if (__popc(s1) == ra) {
                    uint64_t x = ar[s_rank[squeeze2(s1, cu, cv)]];
                    if (x) {
                      uint64_t y = er[s_rank[squeeze2(R & ~s1, cv, cw)]];
                      if (y) add_ck(acc, mul_ck(x, y, of), of);
                    }
                  }
                  if (s1 == 0) break;
                  s1 = (s1 - 1) & R;
                }
              }
            }
          }
          dv[((int64_t)wi * T + t) * C + c] = acc;
          if (of) ofm |= 1ull << t;
          if (A.prof) {
            pwr += 8;
            if (c == 0)  // per (output key, trial): the scanned matches and the input rows they relax
              for (int m = offs[wi]; m < offs[wi + 1]; m++) {
                prd += 4;
                const int cv = A.colr[(int64_t)t * g.n + s_k[kk0 + mp[m]]];
                if (cu != cw && cv != cu && cv != cw) prd += 8 * (uint64_t)(Ca + (et.val ? et.C : 0));
              }
          }
        }
      } else if (op.kind == OP_AXPY) {
        const int d = A.reg_depth[op.a];
        const int nk = s_koff[d] - s_koff[d - 1];
        const int C = A.reg_C[op.dst];
        const uint64_t *av = (const uint64_t *)(base + s_roff[op.a]);
        uint64_t *dv = (uint64_t *)(base + s_roff[op.dst]);
        for (int it = threadIdx.x; it < nk * T * C; it += BLK) {
          bool of = false;
          uint64_t x = mul_ck(op.w, av[it], of);
          uint64_t y = op.first ? 0 : dv[it];
          add_ck(y, x, of);
          dv[it] = y;
          if (of) ofm |= 1ull << ((it / C) % T);
          if (A.prof) {
            prd += op.first ? 8 : 16;
            pwr += 8;
          }
        }
      } else if (op.kind == OP_MROOT) {
        const int da = A.reg_depth[op.a], db = A.reg_depth[op.b];
        const int ka = s_koff[da - 1], na = s_koff[da] - ka;
        const int kb = s_koff[db - 1], nb = s_koff[db] - kb;
        const int Ca = A.reg_C[op.a], Cb = A.reg_C[op.b], sa = A.reg_s[op.a];
        const uint64_t *av = (const uint64_t *)(base + s_roff[op.a]);
        const uint64_t *bv = (const uint64_t *)(base + s_roff[op.b]);
        for (int it = threadIdx.x; it < na * T * Ca; it += BLK) {
          const int i = it / (T * Ca), r = it - i * T * Ca, t = r / Ca, c = r - t * Ca;
          const uint64_t x = av[it];
          if (!x) continue;
          const int32_t v = s_k[ka + i];
          const int pb = (da == db) ? i : find_key(s_k + kb, nb, v);
          if (pb < 0) continue;
          const int cu = A.colr[(int64_t)t * g.n + u], cv = A.colr[(int64_t)t * g.n + v];
          if (cu == cv) continue;
          if (A.prof) prd += 16;
          const uint32_t R1 = spread2(unrank(A.lut, sa - 2, c), cu, cv);
          const uint32_t R2 = Kmask & ~R1 & ~(1u << cu) & ~(1u << cv);
          const uint64_t y = bv[((int64_t)pb * T + t) * Cb + s_rank[squeeze2(R2, cu, cv)]];
          if (!y) continue;
          uint64_t lo = x * y, hi = __umul64hi(x, y);
          if (op.w != 1) {
            uint64_t l2 = lo * op.w, c2 = __umul64hi(lo, op.w);
            uint64_t h2 = hi * op.w + c2;
            if (__umul64hi(hi, op.w) != 0 || h2 < c2) ofm |= 1ull << t;
            lo = l2;
            hi = h2;
          }
          atomic_add128(&s_acc[2 * t], lo, hi);
        }
      } else if (op.kind == OP_MU || op.kind == OP_MV) {
        const bool at_u = op.kind == OP_MU;
        const int da = A.reg_depth[op.a], db = A.reg_depth[op.b];
        const int ka = s_koff[da - 1], na = s_koff[da] - ka;
        const int kb = s_koff[db - 1], nb = s_koff[db] - kb;
        const int Ca = A.reg_C[op.a], Cb = A.reg_C[op.b], ra = A.reg_s[op.a] - 2;
        const uint64_t *av = (const uint64_t *)(base + s_roff[op.a]);
        const uint64_t *bv = (const uint64_t *)(base + s_roff[op.b]);
        const int Co = A.C_out;
        for (int it = threadIdx.x; it < na * T * Co; it += BLK) {
          const int i = it / (T * Co), r = it - i * T * Co, t = r / Co, c = r - t * Co;
          const int32_t v = s_k[ka + i];
          const int pb = (da == db) ? i : find_key(s_k + kb, nb, v);
          if (pb < 0) continue;
          const int cu = A.colr[(int64_t)t * g.n + u], cv = A.colr[(int64_t)t * g.n + v];
          if (cu == cv) continue;
          const int ckey = at_u ? cu : cv, coth = at_u ? cv : cu;
          const uint32_t Rq = spread1(unrank(A.lut, A.s_out - 1, c), ckey);
          if (!((Rq >> coth) & 1u)) continue;
          const uint32_t R = Rq & ~(1u << coth);
          const uint64_t *ar = av + ((int64_t)i * T + t) * Ca;
          const uint64_t *br = bv + ((int64_t)pb * T + t) * Cb;
          uint64_t acc = 0;
          bool of = false;
          uint32_t s1 = R;
          for (;;) {
            if (__popc(s1) == ra) {
              uint64_t x = ar[s_rank[squeeze2(s1, cu, cv)]];
              if (x) {
                uint64_t y = br[s_rank[squeeze2(R & ~s1, cu, cv)]];
                if (y) add_ck(acc, mul_ck(x, y, of), of);
              }
            }
            if (s1 == 0) break;
            s1 = (s1 - 1) & R;
          }
          if (acc) {
            const int64_t key = at_u ? u : v;
            atomic_add_ck(&A.out[(key * T + t) * Co + c], mul_ck(acc, op.w, of), of);
          }
          if (of) ofm |= 1ull << t;
        }
      } else if (op.kind == OP_MEDGE) {
        const int da = A.reg_depth[op.a], db = A.reg_depth[op.b];
        const int ka = s_koff[da - 1], na = s_koff[da] - ka;
        const int kb = s_koff[db - 1], nb = s_koff[db] - kb;
        const int Ca = A.reg_C[op.a], Cb = A.reg_C[op.b], ra = A.reg_s[op.a] - 2, rb = A.reg_s[op.b] - 2;
        const uint64_t *av = (const uint64_t *)(base + s_roff[op.a]);
        const uint64_t *bv = (const uint64_t *)(base + s_roff[op.b]);
        const TabDev et = op.tab >= 0 ? A.tabs[op.tab] : TabDev{nullptr, 0, 0};
        const int Co = A.C_out;
        for (int it = threadIdx.x; it < na * T * Co; it += BLK) {
          const int i = it / (T * Co), r = it - i * T * Co, t = r / Co, c = r - t * Co;
          const int64_t x = s_k[ka + i];
          const int cu = A.colr[(int64_t)t * g.n + u], cx = A.colr[(int64_t)t * g.n + x];
          if (cu == cx) continue;
          const uint64_t *ar = av + ((int64_t)i * T + t) * Ca;
          bool of = false;
          for (int64_t e = g.rp[x]; e < g.rp[x + 1]; e++) {
            const int32_t y = g.col[e];
            if (y >= ub) break;
            const int pb = find_key(s_k + kb, nb, y);
            if (pb < 0) continue;
            const int cy = A.colr[(int64_t)t * g.n + y];
            if (cy == cx || cy == cu) continue;
            const uint32_t Rp = spread2(unrank(A.lut, A.s_out - 2, c), cx, cy);
            if (!((Rp >> cu) & 1u)) continue;
            const uint32_t R = Rp & ~(1u << cu);
            const uint64_t *br = bv + ((int64_t)pb * T + t) * Cb;
            const int64_t tslot = op.tab_src_first ? e : g.rev[e];
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
              const int64_t oslot = op.first ? e : g.rev[e];
              atomic_add_ck(&A.out[(oslot * T + t) * Co + c], mul_ck(s, op.w, of), of);
            }
          }
          if (of) ofm |= 1ull << t;
        }
      } else if (op.kind == OP_MEDGE_T) {
        const int db = A.reg_depth[op.b];
        const int kb = s_koff[db - 1], nb = s_koff[db] - kb;
        const int Cb = A.reg_C[op.b], rb = A.reg_s[op.b] - 2;
        const uint64_t *bv = (const uint64_t *)(base + s_roff[op.b]);
        const TabDev et = op.tab >= 0 ? A.tabs[op.tab] : TabDev{nullptr, 0, 0};
        const TabDev nt = op.ntab >= 0 ? A.tabs[op.ntab] : TabDev{nullptr, 0, 0};
        const int rA = nt.val ? nt.s - 1 : 0;
        const int Co = A.C_out;
        for (int it = threadIdx.x; it < n1 * T * Co; it += BLK) {
          const int jj = it / (T * Co), r = it - jj * T * Co, t = r / Co, c = r - t * Co;
          const int64_t es = g.rp[u] + jj;
          const int32_t y = g.col[es];
          const int pb = find_key(s_k + kb, nb, y);
          if (pb < 0) continue;
          const int cu = A.colr[(int64_t)t * g.n + u], cy = A.colr[(int64_t)t * g.n + y];
          if (cu == cy) continue;
          const uint32_t R = spread2(unrank(A.lut, A.s_out - 2, c), cu, cy);
          const uint64_t *br = bv + ((int64_t)pb * T + t) * Cb;
          const int64_t tslot = op.tab_src_first ? es : g.rev[es];
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
            const int64_t oslot = op.first ? es : g.rev[es];
            atomic_add_ck(&A.out[(oslot * T + t) * Co + c], mul_ck(s, op.w, of), of);
          }
          if (of) ofm |= 1ull << t;
        }
      }
      flag_trials(A.acc.ovf, ofm);
      __syncthreads();
    }
    // root contributions of this source
    for (int t = threadIdx.x; t < T; t += BLK) {
      uint64_t lo = s_acc[2 * t], hi = s_acc[2 * t + 1];
      if (lo | hi) {
        atomic_add128(&A.acc.sum[2 * t], lo, hi);
        if (A.acc.per_src) atomic_add128(&A.acc.per_src[2 * (u * T + t)], lo, hi);
      }
    }
  }
  if (A.prof) {
    for (int o = 32; o > 0; o >>= 1) {
      prd += __shfl_xor(prd, o);
      pwr += __shfl_xor(pwr, o);
    }
    if ((threadIdx.x & 63) == 0) {
      uint64_t *pc = A.prof + 3 * ((blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) % PROF_LANES);
      if (prd) atomicAdd((unsigned long long *)&pc[0], (unsigned long long)prd);
      if (pwr) atomicAdd((unsigned long long *)&pc[1], (unsigned long long)pwr);
    }
  }
}

}  // namespace

int light_max_depth() { return DMAX; }
int light_max_regs() { return RMAX; }

void launch_light(const LightArgs &a, int grid, bool large, hipStream_t st) {
  if (large)
    hipLaunchKernelGGL((k_light<KPOOL_L, EMAX_L>), dim3(grid), dim3(BLK), 0, st, a);
  else
    hipLaunchKernelGGL((k_light<KPOOL_S, EMAX_S>), dim3(grid), dim3(BLK), 0, st, a);
}

}  // namespace cc
