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

}  // namespace arbgpu_impl
