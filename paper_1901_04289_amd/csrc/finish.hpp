// Rounding of an exact integer product entry to the output format: the
// value is T * 2^scale with T an integer given as two's-complement limbs
// (least significant first).  The midpoint is |T| truncated toward zero to
// p bits with T's sign; the radius is rho_in plus one ulp 2^(e_m - p) when
// bits were dropped (Section 2 enclosure; one rounding per entry).
#pragma once

#include "internal.hpp"
#include "mpcore.hpp"

namespace arbgpu_impl {

// get(q) returns limb q of T for 0 <= q < nT.
template <class Get>
__device__ __forceinline__ void finish_entry(const Get &get, int nT, int64_t scale, const arbgpu_out &C,
                                             int64_t oidx, int p, int approx, double rin_m, int rin_e) {
  using namespace arb;
  // magnitude of the two's-complement integer, limb by limb
  const bool neg = (get(nT - 1) >> 31) != 0;
  int z = nT;   // lowest nonzero limb
  for (int q = 0; q < nT; ++q)
    if (get(q)) { z = q; break; }
  auto mag = [&](int q) -> uint32_t {
    if (q < 0 || q >= nT) return 0u;
    const uint32_t v = get(q);
    if (!neg) return v;
    return q > z ? ~v : (q == z ? (uint32_t)(0u - v) : 0u);
  };
  int qt = -1;
  for (int q = nT - 1; q >= 0; --q)
    if (mag(q)) { qt = q; break; }
  const int PL = (p + 31) >> 5;
  if (qt < 0) {
    for (int k = 0; k < PL; ++k) C.limbs[(int64_t)k * C.ld + oidx] = 0u;
    C.exp[oidx] = 0;
    C.nls[oidx] = 0;
    if (!approx) {
      C.rad_m[oidx] = rin_m;
      C.rad_e[oidx] = rin_m != 0.0 ? rin_e : 0;
    }
    if (C.status) C.status[oidx] = ARBGPU_ST_OK;
    return;
  }
  const int64_t bl = 32 * (int64_t)qt + (32 - __builtin_clz(mag(qt)));
  auto bits32 = [&](int64_t lo) -> uint32_t {   // bits [lo, lo + 32) of |T|
    const int64_t q0 = lo >= 0 ? (lo >> 5) : -((31 - lo) >> 5);
    const uint32_t r = (uint32_t)(lo - 32 * q0);
    const uint32_t a = mag((int)q0), b = mag((int)q0 + 1);
    return r ? ((a >> r) | (b << (32u - r))) : a;
  };
  int nout = 0;
  for (int k = 0; k < PL; ++k) {
    uint32_t v = bits32(bl - 32 * (int64_t)(k + 1));
    if (k == PL - 1) v &= 0xFFFFFFFFu << (32 * PL - p);
    C.limbs[(int64_t)k * C.ld + oidx] = v;
    if (v) nout = k + 1;
  }
  // bits of |T| below position bl - p
  const int64_t cut = bl - p;
  bool inexact = false;
  if (cut > 0) {
    const int64_t qc = cut >> 5;
    for (int64_t q = 0; q < qc && !inexact; ++q) inexact = mag((int)q) != 0;
    const uint32_t rc = (uint32_t)(cut & 31);
    if (!inexact && rc) inexact = (mag((int)qc) & ((1u << rc) - 1u)) != 0;
  }
  const int em = (int)(bl + scale);
  C.exp[oidx] = em;
  C.nls[oidx] = (int32_t)((uint32_t)nout | (neg ? 0x80000000u : 0u));
  if (!approx) {
    double rm = 0.0;
    int re = 0;
    ru_add_ext(rin_m, rin_e, inexact ? 0.5 : 0.0, em - p + 1, rm, re);
    C.rad_m[oidx] = rm;
    C.rad_e[oidx] = re;
  }
  if (C.status) C.status[oidx] = ARBGPU_ST_OK;
}

// Whether truncating T' (limbs via get) to p bits is also the truncation of
// every T with |T - T'| < 2^ebits: with bl the bit length of |T'| and
// u = bl - p, the dropped bits D = |T'| mod 2^u must keep the interval
// (|T'| - 2^ebits, |T'| + 2^ebits) strictly inside one cell (H 2^u,
// (H + 1) 2^u) of the truncation grid; bits [ebits + 1, u) of |T'| being
// neither all zero nor all one gives 2^(ebits+1) <= D <= 2^u - 2^(ebits+1) - 1.
// Then |T| has the same bit length and leading p bits, and is inexact.
template <class Get>
__device__ __forceinline__ bool certify_truncation(const Get &get, int nT, int p, int ebits) {
  const bool neg = (get(nT - 1) >> 31) != 0;
  int z = nT;
  for (int q = 0; q < nT; ++q)
    if (get(q)) { z = q; break; }
  auto mag = [&](int q) -> uint32_t {
    if (q < 0 || q >= nT) return 0u;
    const uint32_t v = get(q);
    if (!neg) return v;
    return q > z ? ~v : (q == z ? (uint32_t)(0u - v) : 0u);
  };
  int qt = -1;
  for (int q = nT - 1; q >= 0; --q)
    if (mag(q)) { qt = q; break; }
  if (qt < 0) return false;
  const int64_t bl = 32 * (int64_t)qt + (32 - __builtin_clz(mag(qt)));
  const int64_t u = bl - p, lo = (int64_t)ebits + 1;
  if (u < lo + 2) return false;
  bool any1 = false, any0 = false;
  for (int64_t b = lo; b < u && !(any1 && any0);) {
    const int q = (int)(b >> 5), r = (int)(b & 31);
    const int n = (int)((u - b) < (32 - r) ? (u - b) : (32 - r));
    const uint32_t mask = (n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u)) << r;
    const uint32_t v = mag(q) & mask;
    any1 |= v != 0;
    any0 |= v != mask;
    b += n;
  }
  return any1 && any0;
}

}  // namespace arbgpu_impl
