// Multi-limb fixed-point window arithmetic for the dot-product kernels.
//
// A window is NS 32-bit limbs, least significant first, holding a two's
// complement integer modulo 2^(32 NS).  Limb 0 has weight 2^lo; the top of
// the window is top = lo + 32 NS.  All arrays have compile-time sizes and
// are indexed with compile-time indices only, so they live in registers.
//
// Method (Johansson 2019, Section 3): every term m_i m'_i is aligned into
// one fixed-point accumulator and only the final sum is rounded; bits of a
// term below the window are discarded and counted as one ulp of error each
// (Section 3.4, steps 2, 3 and the discarded-limb case).  This file adds the
// exact decision on top: from the window value V and the error count err the
// truncation of the exact sum to p bits is either certified, or a narrower
// window (a "refinement level") is placed where the uncertainty sits; the
// window sums terms modulo 2^top there, which is exact because the remaining
// unknown quantity is known to be far smaller than 2^top.
#pragma once

#include <stdint.h>

#ifndef ARB_HD
#include <hip/hip_runtime.h>
#define ARB_HD __host__ __device__ __forceinline__
// Pointers into device global memory: declaring the address space lets
// the device compiler use global (not flat) memory instructions.
#if defined(__HIP_DEVICE_COMPILE__)
#define ARB_GLOBAL __attribute__((address_space(1)))
#endif
#endif

namespace arb {

#ifndef ARB_GLOBAL
#define ARB_GLOBAL
#endif

ARB_HD int bitlen32(uint32_t x) { return x ? 32 - __builtin_clz(x) : 0; }

// (hi:lo) >> r for r in [0, 31]
ARB_HD uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t r) {
  return r ? ((lo >> r) | (hi << (32u - r))) : lo;
}

template <int L>
ARB_HD int mbitlen(const uint32_t (&x)[L]) {
  int bl = 0;
#pragma unroll
  for (int i = 0; i < L; ++i)
    if (x[i]) bl = 32 * i + bitlen32(x[i]);
  return bl;
}

template <int L>
ARB_HD bool miszero(const uint32_t (&x)[L]) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) o |= x[i];
  return o == 0;
}

// x += y (mod 2^(32L)), y given as limbs xored with `inv` plus carry-in `cin`
// (inv = ~0, cin = 1 subtracts).
template <int L>
ARB_HD void madd_masked(uint32_t (&x)[L], const uint32_t (&y)[L], uint32_t inv, uint32_t cin) {
  uint64_t c = cin;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    uint64_t s = (uint64_t)x[i] + (uint64_t)(y[i] ^ inv) + c;
    x[i] = (uint32_t)s;
    c = s >> 32;
  }
}

template <int L>
ARB_HD void madd(uint32_t (&x)[L], const uint32_t (&y)[L]) { madd_masked<L>(x, y, 0u, 0u); }

// x = -x (mod 2^(32L))
template <int L>
ARB_HD void mneg(uint32_t (&x)[L]) {
  uint64_t c = 1;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    uint64_t s = (uint64_t)(~x[i]) + c;
    x[i] = (uint32_t)s;
    c = s >> 32;
  }
}

// x += v (small), x -= v (small); no overflow checks (callers keep headroom)
template <int L>
ARB_HD void madd_small(uint32_t (&x)[L], uint32_t v) {
  uint64_t c = v;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    uint64_t s = (uint64_t)x[i] + c;
    x[i] = (uint32_t)s;
    c = s >> 32;
  }
}
template <int L>
ARB_HD void msub_small(uint32_t (&x)[L], uint32_t v) {
  uint64_t b = v;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    uint64_t s = (uint64_t)x[i] - b;
    x[i] = (uint32_t)s;
    b = (s >> 63) & 1;
  }
}

// compare a > v for a small v
template <int L>
ARB_HD bool mgt_small(const uint32_t (&x)[L], uint32_t v) {
  uint32_t hi = 0;
#pragma unroll
  for (int i = 1; i < L; ++i) hi |= x[i];
  return hi != 0 || x[0] > v;
}

// y = low NO limbs of (z >> R); sticky |= (bits shifted below bit 0 != 0).
// z is clobbered.  The sticky bits are an OR over the limbs below the cut;
// the data moves through a barrel shifter whose stages run from the largest
// limb distance down, so only the limbs that can still reach the output are
// kept live at each stage.
template <int L, int NO>
ARB_HD void shr_sticky(uint32_t (&z)[L], uint32_t R, uint32_t (&y)[NO], uint32_t &sticky) {
  const uint32_t q = R >> 5, r = R & 31u;
  uint32_t st = 0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    st |= ((uint32_t)i < q) ? z[i] : 0u;
    st |= ((uint32_t)i == q && r) ? (z[i] << (32u - r)) : 0u;
  }
  sticky |= st;
  constexpr int NB = (L <= 1) ? 1 : (32 - __builtin_clz((unsigned)(L - 1)));
#pragma unroll
  for (int b = NB - 1; b >= 0; --b) {
    const int s = 1 << b;
    const bool on = (q >> b) & 1u;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      uint32_t nv = (i + s < L) ? z[i + s] : 0u;
      z[i] = on ? nv : z[i];
    }
  }
  const bool gone = q >= (uint32_t)L;
#pragma unroll
  for (int i = 0; i < NO; ++i) {
    uint32_t lo = (i < L) ? z[i] : 0u;
    uint32_t hi = (i + 1 < L) ? z[i + 1] : 0u;
    y[i] = gone ? 0u : funnel(hi, lo, r);
  }
}

// x <<= S (mod 2^(32L)), S < 32L
template <int L>
ARB_HD void shl_var(uint32_t (&x)[L], uint32_t S) {
  uint32_t q = S >> 5, r = S & 31u;
#pragma unroll
  for (int b = 0; (1 << b) < L; ++b) {
    const int s = 1 << b;
    const bool on = (q >> b) & 1u;
#pragma unroll
    for (int i = L - 1; i >= 0; --i) {
      uint32_t nv = (i - s >= 0) ? x[i - s] : 0u;
      x[i] = on ? nv : x[i];
    }
  }
  if (q >= (uint32_t)L) {
#pragma unroll
    for (int i = 0; i < L; ++i) x[i] = 0;
  }
#pragma unroll
  for (int i = L - 1; i >= 0; --i) {
    uint32_t lo = (i > 0) ? x[i - 1] : 0u;
    x[i] = r ? ((x[i] << r) | (lo >> (32u - r))) : x[i];
  }
}

// acc + hi 2^64 += a * b: one v_mad_u64_u32 whose carry out of the 64
// bits goes into hi.
ARB_HD void mac64(uint64_t &acc, uint32_t &hi, uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint64_t cy;
  asm("v_mad_u64_u32 %0, %2, %3, %4, %0\n\t"
      "v_addc_co_u32_e64 %1, %2, 0, %1, %2"
      : "+v"(acc), "+v"(hi), "=&s"(cy)
      : "v"(a), "v"(b));
#else
  const uint64_t pr = (uint64_t)a * b;
  acc += pr;
  hi += acc < pr ? 1u : 0u;
#endif
}

// Whether c holds in any active lane of the wave (c itself outside device
// code); the same in every lane, so a branch on it is uniform.
ARB_HD bool any_lane(bool c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_ballot_w64(c) != 0;
#else
  return c;
#endif
}

// The largest value of v in [0, 128) over the active lanes of the wave, the
// same in every lane (one ballot per bit); v itself outside device code.
ARB_HD int active_max7(int v) {
#if defined(__HIP_DEVICE_COMPILE__)
  int r = 0;
#pragma unroll
  for (int b = 6; b >= 0; --b) {
    const int c = r | (1 << b);
    if (any_lane(v >= c)) r = c;
  }
  return r;
#else
  return v;
#endif
}

// Product of LS-first limb arrays, p = a * b, column by column (each
// column's products in one 64-bit accumulator with a carry word), with
// the low products left out (the "mulhigh" of Section 3.4): a column
// k < kc is not formed unless another active lane of the wave needs it
// (the left-out pairs sum below sum_{s<kc} (s+1) 2^(64 + 32 s) <
// kc 2^(32 kc + 32) (1 + 2^-31) units of p's lowest limb), nor a product
// of limbs at or above na of a or nb of b in every active lane (those limbs
// are zero).  `skipped` tells whether a pair was left out.
template <int NA>
ARB_HD void mul_limbs(const uint32_t (&a)[NA], int na, const uint32_t (&b)[NA], int nb, uint32_t (&p)[2 * NA],
                      int kc, bool &skipped) {
  static_assert(NA < 128, "limb counts below 128");
  skipped = na > 0 && !any_lane(kc <= 0);
  const int nau = active_max7(na < NA ? na : NA), nbu = active_max7(nb < NA ? nb : NA);
  const bool full = nau >= NA && nbu >= NA;
  uint64_t acc = 0;
  uint32_t hi = 0;
#pragma unroll
  for (int k = 0; k < 2 * NA - 1; ++k) {
    if (any_lane(k >= kc)) {
      if (full) {
#pragma unroll
        for (int i = (k - NA + 1 > 0 ? k - NA + 1 : 0); i <= (k < NA - 1 ? k : NA - 1); ++i)
          mac64(acc, hi, a[i], b[k - i]);
      } else {
#pragma unroll
        for (int i = (k - NA + 1 > 0 ? k - NA + 1 : 0); i <= (k < NA - 1 ? k : NA - 1); ++i)
          if (i < nau && k - i < nbu) mac64(acc, hi, a[i], b[k - i]);   // uniform
      }
    }
    p[k] = (uint32_t)acc;
    acc = (acc >> 32) | ((uint64_t)hi << 32);
    hi = 0;
  }
  p[2 * NA - 1] = (uint32_t)acc;
}

// ---------------------------------------------------------------------------
// Directed-upward FP64 arithmetic for radii (error-free transformations, then
// one step up when the rounded result fell below the exact one).
// ---------------------------------------------------------------------------

ARB_HD double next_up(double x) {  // x >= 0, finite
  union { double d; uint64_t u; } v;
  v.d = x;
  v.u += 1;
  return v.d;
}

#pragma clang fp contract(off)
ARB_HD double ru_mul(double a, double b) {  // a, b >= 0
  double p = a * b;
  double e = __builtin_fma(a, b, -p);
  return e > 0.0 ? next_up(p) : p;
}

ARB_HD double ru_add(double a, double b) {  // a, b >= 0
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return e > 0.0 ? next_up(s) : s;
}

// a * 2^d for d <= 0: exact when the result stays at or above 2^-1001
// (normal); otherwise the upper bound 2^-1000.
ARB_HD double ru_scale_down(double a, int d) {
  if (a == 0.0) return 0.0;
  int ea;
  (void)__builtin_frexp(a, &ea);      // a < 2^ea
  if (ea + d < -1000) return __builtin_ldexp(1.0, -1000);
  return __builtin_ldexp(a, d);
}
#pragma clang fp contract(on)

// Extended-exponent upward sum of m1*2^e1 + m2*2^e2 (m >= 0, m <= 8) into
// a normalized (m in [0.5, 1), e), rounded up.
ARB_HD void ru_add_ext(double m1, int e1, double m2, int e2, double &mo, int &eo) {
  if (m1 == 0.0 && m2 == 0.0) { mo = 0.0; eo = 0; return; }
  if (m2 == 0.0 || (m1 != 0.0 && e1 >= e2)) {
    double s = ru_add(m1, ru_scale_down(m2, e2 - e1));
    int ex;
    mo = __builtin_frexp(s, &ex);
    eo = e1 + ex;
  } else {
    double s = ru_add(m2, ru_scale_down(m1, e1 - e2));
    int ex;
    mo = __builtin_frexp(s, &ex);
    eo = e2 + ex;
  }
}

}  // namespace arb
