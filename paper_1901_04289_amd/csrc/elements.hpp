// Element access shared by the scaled-integer kernels: inner-index
// layouts of the real and complex products, limb counts, lowest set bits
// and 32-bit windows of the scaled mantissa integers.
#pragma once

#include "internal.hpp"

namespace arbgpu_impl {

// Part and sign of inner index k under an inner layout mode (see SliceParams).
__device__ __forceinline__ void inner_map(int mode, int64_t len, int64_t k, int &part, int64_t &kk, uint32_t &neg) {
  part = 0;
  kk = k;
  neg = 0;
  if (mode == 0) return;
  const bool second = k >= len;
  kk = second ? k - len : k;
  if (mode == 1) { part = second ? 1 : 0; neg = second ? 1u : 0u; }
  else if (mode == 2) { part = second ? 0 : 1; }
  else { part = second ? 1 : 0; }
}

__device__ __forceinline__ const arbgpu_arr &part_of(const arbgpu_arr *p, int i) { return i ? p[1] : p[0]; }

// position of the lowest set bit of |m| (INT32_MAX for zero)
__device__ __forceinline__ int low_bit(const arbgpu_arr &A, int64_t idx, int n, int e) {
  for (int q = n - 1; q >= 0; --q) {
    uint32_t v = A.limbs[(int64_t)q * A.ld + idx];
    if (v) return e - 32 * (q + 1) + __builtin_ctz(v);
  }
  return 0x7FFFFFFF;
}

__device__ __forceinline__ int elem_n(const arbgpu_arr &A, int64_t idx) {
  int n = A.nls[idx] & 0x7FFFFFFF;
  return n > A.cap ? A.cap : n;
}

// Bits [32w - s, 32w - s + 32) of the limb integer M (least significant limb
// is limb n-1 in memory), zero outside.
__device__ __forceinline__ uint32_t mant_chunk(const arbgpu_arr &A, int64_t idx, int n, int64_t o) {
  // o: bit offset into M (may be negative)
  const int64_t li = o >= 0 ? (o >> 5) : -((31 - o) >> 5);
  const uint32_t r = (uint32_t)(o - 32 * li);
  auto get = [&](int64_t i) -> uint32_t {
    return (i >= 0 && i < n) ? A.limbs[(int64_t)(n - 1 - i) * A.ld + idx] : 0u;
  };
  const uint32_t lo = get(li), hi = get(li + 1);
  return r ? ((lo >> r) | (hi << (32u - r))) : lo;
}

}  // namespace arbgpu_impl
