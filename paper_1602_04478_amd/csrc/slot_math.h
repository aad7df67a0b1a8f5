// Device helpers shared by the kernels: colour-subset slot arithmetic and
// checked 64-bit integer accumulation.
//
// A table keyed by vertices whose colours are fixed stores only the remaining
// colours: those colour bits are squeezed out of the k-bit signature mask and
// the rest is stored at its colex rank among masks of the same popcount.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cc {
namespace dev {

constexpr int BLK = 256;
constexpr int LUT_RANK = 0, LUT_UNRANK = 2048, LUT_OFF = 4096, LUT_SIZE = 4112;

__host__ __device__ __forceinline__ uint32_t squeeze2(uint32_t m, int c1, int c2) {
  int lo = min(c1, c2), hi = max(c1, c2);
  uint32_t a = m & ((1u << lo) - 1u);
  uint32_t b = (m >> (lo + 1)) & ((1u << (hi - lo - 1)) - 1u);
  uint32_t c = m >> (hi + 1);
  return a | (b << lo) | (c << (hi - 1));
}
__host__ __device__ __forceinline__ uint32_t spread2(uint32_t m, int c1, int c2) {
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

// The bits of x placed at the set bits of m, lowest first (parallel deposit).
__device__ __forceinline__ uint32_t deposit(uint32_t x, uint32_t m) {
  uint32_t r = 0;
  for (; m && x; x >>= 1) {
    const uint32_t low = m & (0u - m);
    if (x & 1u) r |= low;
    m ^= low;
  }
  return r;
}
// The next larger integer with the same number of set bits (x > 0): with
// deposit() it walks the subsets of a given size of a mask in order.
__device__ __forceinline__ uint32_t next_comb(uint32_t x) {
  const uint32_t c = x & (0u - x), r = x + c;
  return (((r ^ x) >> 2) >> __builtin_ctz(c)) | r;
}

// acc += a (checked)
__device__ __forceinline__ void add_ck(uint64_t &acc, uint64_t a, bool &of) {
  uint64_t s = acc + a;
  of |= s < acc;
  acc = s;
}
// a * b (checked).  Both factors below 2^32 (the common case): one 32 x 32
// multiply and no overflow is possible; otherwise the high word decides.
__device__ __forceinline__ uint64_t mul_ck(uint64_t a, uint64_t b, bool &of) {
  if (((a | b) >> 32) == 0) return (uint64_t)(uint32_t)a * (uint32_t)b;
  of |= __umul64hi(a, b) != 0;
  return a * b;
}
// the 128-bit product (lo, hi) of a and b
__device__ __forceinline__ void mul_wide(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
  if (((a | b) >> 32) == 0) {
    lo = (uint64_t)(uint32_t)a * (uint32_t)b;
    hi = 0;
  } else {
    lo = a * b;
    hi = __umul64hi(a, b);
  }
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

// raise the overflow flag of every trial in mask m
__device__ __forceinline__ void flag_trials(uint32_t *ovf, uint64_t m) {
  while (m) {
    int t = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    atomicOr(&ovf[t], 1u);
  }
}

__device__ __forceinline__ void load_rank(uint16_t *s_rank, const uint16_t *lut) {
  for (int i = threadIdx.x; i < 2048; i += blockDim.x) s_rank[i] = lut[LUT_RANK + i];
  __syncthreads();
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


}  // namespace dev
}  // namespace cc
