// Certification of a truncation from a window value and an error bound,
// for windows held as 64-bit columns in LDS (the LDS-window dot and the
// digit-product dot).  The window value V is a two's-complement integer
// whose 32-bit limbs sit in the low halves of the columns col[0 .. nW).
#pragma once

#include <stdint.h>

namespace arbgpu_impl {

// Bit length of the magnitude held in limbs x(0 .. n) (least significant first).
template <class X>
__device__ __forceinline__ int64_t bitlen_limbs(const X &x, int n) {
  for (int q = n - 1; q >= 0; --q)
    if (x(q)) return 32 * (int64_t)q + (32 - __builtin_clz(x(q)));
  return 0;
}

// One thread: whether the truncation to p bits is certified for every sum
// within err units of the window value.  With m = |V| - err and h = |V| +
// err the sum's magnitude lies strictly between them (the callers' error
// bounds are strict), so when both have the same bit length l > p and the
// same top p bits, the sum truncates to those bits and drops nonzero bits
// below them.  On success the columns hold a value whose truncation is the
// result (m, with its lowest bit set when no dropped bit of m is set, which
// keeps it below h and inside the cell) with the sign of V.  *hb receives
// the bit length of h: the sum's magnitude is below 2^hb units.  `hi` is
// scratch of nW limbs.
__device__ inline bool window_certify(int nW, uint64_t err, int p, int64_t *col, uint32_t *hi, int64_t *hb) {
  *hb = 0;
  if (err == 0) return true;   // exact: the window value is the sum
  auto m = [&](int c) { return (uint32_t)col[c]; };
  auto set = [&](int c, uint32_t v) { col[c] = (int64_t)v; };
  const bool neg = (m(nW - 1) >> 31) != 0;
  if (neg) {   // magnitude
    uint32_t cy = 1;
    for (int c = 0; c < nW; ++c) {
      const uint32_t v = ~m(c) + cy;
      cy = (cy && v == 0) ? 1u : 0u;
      set(c, v);
    }
  }
  uint64_t cy = err;
  for (int c = 0; c < nW; ++c) {
    const uint64_t v = (uint64_t)m(c) + (cy & 0xFFFFFFFFull);
    hi[c] = (uint32_t)v;
    cy = (cy >> 32) + (v >> 32);
  }
  const int64_t lb = cy ? 32 * (int64_t)nW + 1 : bitlen_limbs([&](int c) { return hi[c]; }, nW);
  *hb = lb;
  if (cy) return false;
  int64_t bw = (int64_t)err;
  for (int c = 0; c < nW; ++c) {
    const int64_t v = (int64_t)m(c) - (bw & 0xFFFFFFFFll);
    set(c, (uint32_t)v);
    bw = (int64_t)((uint64_t)bw >> 32) + (v < 0 ? 1 : 0);
  }
  if (bw) return false;   // |V| < err: not even the sign is known
  const int64_t la = bitlen_limbs(m, nW);
  if (la == 0 || la != lb || la <= p) return false;
  const int64_t cut = la - p;   // bits below `cut` are dropped
  bool low = false;
  for (int64_t bit = 0; bit < la; bit += 32) {
    const int q = (int)(bit >> 5);
    uint32_t keep = 0xFFFFFFFFu;
    if (bit + 32 <= cut) keep = 0u;
    else if (bit < cut) keep = 0xFFFFFFFFu << (uint32_t)(cut - bit);
    if ((m(q) & keep) != (hi[q] & keep)) return false;
    low |= (m(q) & ~keep) != 0;
  }
  if (!low) set(0, m(0) | 1u);   // cut >= 1, so bit 0 is a dropped bit
  if (neg) {   // back to two's complement of the signed value
    uint32_t c1 = 1;
    for (int c = 0; c < nW; ++c) {
      const uint32_t v = ~m(c) + c1;
      c1 = (c1 && v == 0) ? 1u : 0u;
      set(c, v);
    }
  }
  return true;
}

}  // namespace arbgpu_impl
