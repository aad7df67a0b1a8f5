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
// Sections 5.1-5.2).  Sums and products are checked: a table entry that leaves 64
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

// the same, with (seed, first trial) read from device memory (replayable launches)
__global__ void k_colour_dev(const int32_t *orig, int64_t n, int k, const uint64_t *param, int T, uint8_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * T) return;
  int t = (int)(i / n);
  int64_t r = i - (int64_t)t * n;
  uint64_t key = mix64(param[0] + param[1] + (uint64_t)t);
  uint64_t h = mix64(key ^ (uint64_t)(uint32_t)orig[r]);
  out[i] = (uint8_t)(((h >> 32) * (uint64_t)k) >> 32);
}

// plain streaming copy, 16 bytes per lane per step
__global__ void k_copy16(const uint4 *__restrict__ a, uint4 *__restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void k_permute(const uint8_t *by_orig, const int32_t *orig, int64_t n, int T, uint8_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * T) return;
  int t = (int)(i / n);
  int64_t r = i - (int64_t)t * n;
  out[i] = by_orig[(int64_t)t * n + orig[r]];
}

__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = x;
}
__global__ void k_fill_u64(uint64_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
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
}  // namespace


// A one-time host-to-device copy on a stream of its own (non-blocking: it
// must not touch the legacy stream, which other threads' stream captures
// forbid), waited for before returning.
bool upload_sync(void *d, const void *h, size_t bytes) {
  hipStream_t s;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return false;
  bool ok = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s) == hipSuccess && hipStreamSynchronize(s) == hipSuccess;
  (void)hipStreamDestroy(s);
  return ok;
}

// colex rank / unrank tables (per device, built once, in the constant-table pool)
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
  uint16_t *d = (uint16_t *)table_pool_alloc(sizeof(uint16_t) * LUT_SIZE);
  if (!d) return nullptr;
  if (!upload_sync(d, h.data(), sizeof(uint16_t) * LUT_SIZE)) return nullptr;
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
void launch_colour_dev(const int32_t *orig, int64_t n, int k, const uint64_t *param, int T, uint8_t *out,
                       hipStream_t st) {
  int64_t tot = n * T;
  hipLaunchKernelGGL(k_colour_dev, dim3((unsigned)((tot + BLK - 1) / BLK)), dim3(BLK), 0, st, orig, n, k, param, T,
                     out);
}
void launch_copy16(const void *a, void *b, int64_t n16, hipStream_t st) {
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)std::min<int64_t>((n16 + BLK - 1) / BLK, 1 << 16)), dim3(BLK), 0, st,
                     (const uint4 *)a, (uint4 *)b, n16);
}
void launch_permute_colours(const uint8_t *by_orig, const int32_t *orig, int64_t n, int T, uint8_t *out,
                            hipStream_t st) {
  int64_t tot = n * T;
  hipLaunchKernelGGL(k_permute, dim3((unsigned)((tot + BLK - 1) / BLK)), dim3(BLK), 0, st, by_orig, orig, n, T, out);
}
void launch_fill_u8(uint8_t *p, int64_t n, hipStream_t st, uint8_t x) {
  if (n <= 0) return;
  int64_t g = std::min<int64_t>((n + BLK - 1) / BLK, 8192);
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)g), dim3(BLK), 0, st, p, n, x);
}
void launch_fill_u64(uint64_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t g = std::min<int64_t>((n + BLK - 1) / BLK, 8192);
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)g), dim3(BLK), 0, st, p, n);
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
