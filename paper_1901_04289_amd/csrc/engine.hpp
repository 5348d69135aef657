// Per-output dot-product engine: setup pass, window accumulation, exact
// decision / refinement, radius accumulation and output encoding.
//
// Algorithm 1 of Johansson (2019): a setup pass over exponents only finds
// e_max, the number of nonzero terms and the radius frame; the window top is
// e_s = e_max + extend with extend = bc(N_nonzero) + 1 (Section 3.3, steps
// 9-11), so carries never overflow the top limb and the sign survives.  The
// evaluation pass adds the overlapping bits of every product (Section 3.4)
// and counts discarded nonzero bits as ulps in `err`.  Finalization
// (Algorithm 1, step 4) is replaced by `decide`, which returns the exact
// truncation of the exact sum to p bits or moves the window (see mpcore.hpp).
//
// The engine is written for one lane; the GPU kernels add the cross-lane
// reductions between the passes when several lanes share one output.
#pragma once

#include "mpcore.hpp"

namespace arb {

constexpr int kExpLimit = 1 << 28;   // |exponent| bound of the input format
constexpr int kMaxLevels = 256;      // refinement passes before handing over

// One operand as the engine sees it.
template <int NA>
struct Opnd {
  uint32_t l[NA];   // top min(n, NA) limbs, least significant first
  int n;            // limbs loaded (0 = zero)
  bool trunc;       // nonzero limbs were left out (n > NA)
  int e;            // exponent
  uint32_t sign;    // 0/1
  double rm;        // radius mantissa in [0.5, 1) or 0 (normalized)
  int re;           // radius exponent
};

// Upper bound of |m| as (mantissa in [0.5, 1], exponent e): the top 64
// bits rounded up to 53 bits.
template <int NA>
ARB_HD double mag_upper(const Opnd<NA> &o) {
  if (o.n == 0) return 0.0;
  uint32_t top = 0, second = 0, rest = o.trunc ? 1u : 0u;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    if (i == o.n - 1) top = o.l[i];
    else if (i == o.n - 2) second = o.l[i];
    else if (i < o.n - 2) rest |= o.l[i];
  }
  uint64_t v = ((uint64_t)top << 32) | second;
  uint64_t m53 = (v >> 11) + (((v & 0x7FFull) != 0 || rest != 0) ? 1 : 0);
  return (double)m53 * 0x1p-53;
}

template <int NS>
struct Window {
  uint32_t w[NS];
  uint32_t err;        // ulps of 2^lo
  uint32_t pt;         // terms that overlapped the window and lost bits
  uint32_t below_cnt;  // terms entirely below the window
  int below_max;       // largest top exponent among those
  bool bad;            // a truncated operand could not resolve this window
  ARB_HD void clear() {
#pragma unroll
    for (int i = 0; i < NS; ++i) w[i] = 0;
    err = pt = below_cnt = 0;
    below_max = -0x7FFFFFFF;
    bad = false;
  }
};

// Add bits [lo, lo + 32 NS) of (-1)^neg * a * b into the window, modulo
// 2^(32 NS).
template <int NS, int NA>
ARB_HD void add_term(Window<NS> &W, int lo, const Opnd<NA> &a, const Opnd<NA> &b, uint32_t neg) {
  const int top = lo + 32 * NS;
  const int et = a.e + b.e;
  if (et <= lo) {          // |term| < 2^et <= 2^lo
    W.err += 1;
    W.below_cnt += 1;
    W.below_max = et > W.below_max ? et : W.below_max;
    return;
  }
  uint32_t e_inc = 0;
  if (a.trunc || b.trunc) {
    // dropped operand limbs change the product by less than
    // 2^(et - 32 min(n_a, n_b) + 1); that must stay below one ulp
    int nmin = (a.trunc && b.trunc) ? (a.n < b.n ? a.n : b.n) : (a.trunc ? a.n : b.n);
    if (et - 32 * nmin + 1 > lo) W.bad = true;
    e_inc += 1;
  }
  const int base = et - 32 * (a.n + b.n);
  if (base >= top) {        // a multiple of 2^top: zero modulo the window
    if (e_inc) { W.pt += 1; W.err += e_inc; }
    return;
  }
  constexpr int L = NS + 2 * NA;
  uint32_t z[L];
#pragma unroll
  for (int i = 0; i < NS; ++i) z[i] = 0;
  // products of limb index sum below kc are left out: they sum below
  // kc 2^(32 kc + 32) (1 + 2^-31) 2^base < 2^(lo - 8 + log2 kc) <= 2^lo for
  // kc <= 2 NA <= 80, i.e. below one window unit
  const int kc = (lo - base - 40) >> 5;
  bool skipped;
  {
    uint32_t p[2 * NA];
    mul_limbs<NA>(a.l, a.n, b.l, b.n, p, kc < 0 ? 0 : kc, skipped);
#pragma unroll
    for (int i = 0; i < 2 * NA; ++i) z[NS + i] = p[i];
  }
  uint32_t x[NS];
  uint32_t sticky = 0;
  shr_sticky<L, NS>(z, (uint32_t)(top - base), x, sticky);
  // the window takes floor(P' 2^(base - lo)); the exact term lies within
  // one unit above it, or two when products were left out
  if (skipped) e_inc += 2;
  else if (sticky) e_inc += 1;
  if (e_inc) W.pt += 1;
  W.err += e_inc;
  const uint32_t inv = neg ? 0xFFFFFFFFu : 0u;
  madd_masked<NS>(W.w, x, inv, neg);
}

// Radius terms |m_a| r_b + |m_b| r_a + r_a r_b, added in the frame 2^F.
template <int NA>
ARB_HD double rad_term(const Opnd<NA> &a, const Opnd<NA> &b, int F) {
  double acc = 0.0;
  if (b.rm != 0.0 && a.n) acc = ru_add(acc, ru_scale_down(ru_mul(mag_upper(a), b.rm), a.e + b.re - F));
  if (a.rm != 0.0 && b.n) acc = ru_add(acc, ru_scale_down(ru_mul(mag_upper(b), a.rm), b.e + a.re - F));
  if (a.rm != 0.0 && b.rm != 0.0) acc = ru_add(acc, ru_scale_down(ru_mul(a.rm, b.rm), a.re + b.re - F));
  return acc;
}

// Exponent bound of the radius terms of one product (for the frame F).
template <int NA>
ARB_HD int rad_exp(const Opnd<NA> &a, const Opnd<NA> &b, bool &any) {
  int f = -0x7FFFFFFF;
  if (b.rm != 0.0 && a.n) { f = a.e + b.re > f ? a.e + b.re : f; any = true; }
  if (a.rm != 0.0 && b.n) { f = b.e + a.re > f ? b.e + a.re : f; any = true; }
  if (a.rm != 0.0 && b.rm != 0.0) { f = a.re + b.re > f ? a.re + b.re : f; any = true; }
  return f;
}

// Sum of the radius terms (Section 3.5) in fixed point: units of 2^-kRadQ
// of the frame 2^F, three 64-bit words (integer part below 2^42).  Each
// term, an upper bound as a double of at most 4, is rounded up to the grid
// and added exactly, so the sum does not depend on how the terms are split
// among lanes, waves or workgroups, nor on the order of the additions.
// Terms below 2^-kRadQ count as 2^-kRadQ: with the largest term at least
// 1/4 of the frame, that raises the sum by less than 2^-100 of itself for
// any count of terms the format allows.
constexpr int kRadQ = 150;
struct RadAcc {
  uint64_t w[3];
  ARB_HD void clear() { w[0] = w[1] = w[2] = 0; }
  ARB_HD void add_words(uint64_t a0, uint64_t a1, uint64_t a2) {
    const uint64_t s0 = w[0] + a0;
    const uint64_t c0 = s0 < a0 ? 1u : 0u;
    uint64_t s1 = w[1] + a1;
    uint64_t c1 = s1 < a1 ? 1u : 0u;
    s1 += c0;
    c1 += s1 < c0 ? 1u : 0u;
    w[0] = s0;
    w[1] = s1;
    w[2] = w[2] + a2 + c1;
  }
  ARB_HD void add(double x) {   // 0 <= x <= 4, zero or normal
    if (!(x > 0.0)) return;
    // x = m 2^(be - 1075) with m the 53-bit significand
    const uint64_t bits = (uint64_t)__builtin_bit_cast(int64_t, x);
    const int be = (int)(bits >> 52);
    const uint64_t m = (bits & 0xFFFFFFFFFFFFFull) | (1ull << 52);
    const int sh = be - 1075 + kRadQ;                              // x 2^Q = m 2^sh
    uint64_t v0 = 0, v1 = 0, v2 = 0;
    if (sh >= 128) {
      v2 = m << (sh - 128);
    } else if (sh >= 64) {
      const int r = sh - 64;
      v1 = m << r;
      v2 = r ? m >> (64 - r) : 0;
    } else if (sh >= 0) {
      v0 = m << sh;
      v1 = sh ? m >> (64 - sh) : 0;
    } else {   // below the grid: round up
      const int q = -sh;
      v0 = q >= 64 ? 1u : (m >> q) + ((m & ((1ull << q) - 1)) ? 1u : 0u);
    }
    add_words(v0, v1, v2);
  }
  ARB_HD void add(const RadAcc &o) { add_words(o.w[0], o.w[1], o.w[2]); }
  // The sum rounded up to m 2^e (m in [0.5, 1)) in units of the frame;
  // false when it is zero.
  ARB_HD bool get(double &m, int &e) const {
    int q = 2;
    while (q > 0 && w[q] == 0) --q;
    if (w[q] == 0) return false;
    const int L = 64 * q + (64 - __builtin_clzll(w[q]));   // bit length
    // the top 64 bits and whether any bit below them is set
    uint64_t t;
    bool sticky = false;
    const int lo = L - 64;
    if (lo <= 0) {
      t = w[0] << (-lo);
    } else {
      const int qw = lo >> 6, r = lo & 63;
      const uint64_t hi = qw + 1 <= 2 ? w[qw + 1] : 0;
      t = r ? (w[qw] >> r) | (hi << (64 - r)) : w[qw];
      for (int k = 0; k < qw; ++k) sticky |= w[k] != 0;
      if (r) sticky |= (w[qw] & ((1ull << r) - 1)) != 0;
    }
    uint64_t m53 = (t >> 11) + (((t & 0x7FFull) != 0 || sticky) ? 1u : 0u);
    int Lr = L;
    if (m53 >> 53) { m53 >>= 1; ++Lr; }   // rounded up to 2^53 (exact: it is even)
    m = (double)m53 * 0x1p-53;
    e = Lr - kRadQ;
    return true;
  }
};

// Setup-pass statistics (Section 3.3, steps 1-5).
struct Setup {
  int emax;       // max(e + e') over nonzero midpoint products
  uint32_t nnz;   // nonzero midpoint products
  int F;          // radius frame: max exponent bound of radius terms
  bool any_rad;
  bool erange;
  ARB_HD void clear() { emax = -0x7FFFFFFF; nnz = 0; F = -0x7FFFFFFF; any_rad = false; erange = false; }
};

template <int NA>
ARB_HD bool opnd_out_of_range(const Opnd<NA> &o) {
  if (o.n && (o.e >= kExpLimit || o.e <= -kExpLimit)) return true;
  if (o.rm != 0.0 && (o.re >= kExpLimit || o.re <= -kExpLimit)) return true;
  return false;
}

template <int NA>
ARB_HD void setup_term(Setup &S, const Opnd<NA> &a, const Opnd<NA> &b, bool want_rad) {
  if (opnd_out_of_range(a) || opnd_out_of_range(b)) S.erange = true;
  if (a.n && b.n) {
    int et = a.e + b.e;
    S.emax = et > S.emax ? et : S.emax;
    S.nnz += 1;
  }
  if (want_rad) {
    bool any = false;
    int f = rad_exp(a, b, any);
    if (any) { S.any_rad = true; S.F = f > S.F ? f : S.F; }
  }
}

// Refinement state and result of one output.
template <int NS>
struct Level {
  int top;
  bool have_g;
  uint32_t g_sign;
  int g_exp;
  // Y holds the grid point's p-bit magnitude (normalized to bit 32NS-1)
  // while have_g, and the result magnitude once done.
  uint32_t Y[NS];
  bool done, bad, zero, inexact;
  uint32_t r_sign;
  int r_exp;
  int levels;
};

// Keep-mask of the top p bits of a normalized NS-limb number, for limb i.
template <int NS>
ARB_HD uint32_t keep_mask(int i, int p) {
  const int cut = 32 * NS - p;      // lowest kept bit position
  const int q = cut >> 5, r = cut & 31;
  return i > q ? 0xFFFFFFFFu : (i == q ? (0xFFFFFFFFu << r) : 0u);
}

// Decide from the window value V (limbs at weight 2^lo) and the error
// state whether the truncation of the exact sum S to p bits is known.
// Invariant: S - g = V * 2^lo + eps with |eps| <= err * 2^lo, where g is the
// current grid point (0 when !have_g).
template <int NS>
ARB_HD void decide(Level<NS> &st, const Window<NS> &W, int lo, int p) {
  st.levels += 1;
  if (W.bad) {
    st.bad = true;
    st.done = true;
    return;
  }
  const uint32_t neg = W.w[NS - 1] >> 31;
  uint32_t mag[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) mag[i] = W.w[i];
  if (neg) mneg<NS>(mag);
  const bool magzero = miszero<NS>(mag);
  const uint32_t err = W.err;
  int new_top = 0;
  bool cont = false;

  if (err != 0 && magzero && W.pt == 0 && W.below_cnt > 0) {
    // only whole terms below the window are unknown: their sum is below
    // below_cnt * 2^below_max
    new_top = W.below_max + bitlen32(W.below_cnt) + 2;
    cont = true;
  } else if (!st.have_g) {
    if (err == 0) {
      if (magzero) {
        st.zero = true; st.inexact = false; st.done = true; return;
      }
      const int bl = mbitlen<NS>(mag);
      uint32_t Y[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) Y[i] = mag[i];
      shl_var<NS>(Y, (uint32_t)(32 * NS - bl));
      uint32_t lost = 0;
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        uint32_t k = keep_mask<NS>(i, p);
        lost |= Y[i] & ~k;
        st.Y[i] = Y[i] & k;
      }
      st.zero = false; st.r_sign = neg; st.r_exp = lo + bl; st.inexact = lost != 0;
      st.done = true;
      return;
    }
    uint32_t b[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) b[i] = mag[i];
    madd_small<NS>(b, err);
    if (!mgt_small<NS>(mag, err)) {          // sign unknown
      new_top = lo + mbitlen<NS>(b) + 2;
      cont = true;
    } else {
      uint32_t a[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) a[i] = mag[i];
      msub_small<NS>(a, err);
      const int bla = mbitlen<NS>(a), blb = mbitlen<NS>(b);
      const int need = bitlen32(2u * err) + 2;
      if (bla - p < need) {                   // window too coarse here
        new_top = lo + blb + 2;
        cont = true;
      } else {
        shl_var<NS>(a, (uint32_t)(32 * NS - bla));
        shl_var<NS>(b, (uint32_t)(32 * NS - blb));
        bool same = (bla == blb);
        uint32_t a_low = 0;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          uint32_t k = keep_mask<NS>(i, p);
          same = same && ((a[i] & k) == (b[i] & k));
          a_low |= a[i] & ~k;
        }
        if (same && a_low != 0) {             // certified
#pragma unroll
          for (int i = 0; i < NS; ++i) st.Y[i] = a[i] & keep_mask<NS>(i, p);
          st.zero = false; st.r_sign = neg; st.r_exp = lo + bla; st.inexact = true;
          st.done = true;
          return;
        }
        // the only p-bit grid point in [a, b] is trunc(b): recentre on it
        st.have_g = true;
        st.g_sign = neg;
        st.g_exp = lo + blb;
#pragma unroll
        for (int i = 0; i < NS; ++i) st.Y[i] = b[i] & keep_mask<NS>(i, p);
        new_top = lo + need;
        cont = true;
      }
    }
  } else {
    if (err == 0 && magzero) {                // S == g exactly
      st.zero = false; st.r_sign = st.g_sign; st.r_exp = st.g_exp; st.inexact = false;
      st.done = true;
      return;
    }
    if (err != 0 && !mgt_small<NS>(mag, err)) {  // sign of S - g unknown
      uint32_t b[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) b[i] = mag[i];
      madd_small<NS>(b, err);
      new_top = lo + mbitlen<NS>(b) + 2;
      cont = true;
    } else {
      st.zero = false; st.inexact = true; st.r_sign = st.g_sign;
      if (neg == st.g_sign) {                 // |S| > |g|
        st.r_exp = st.g_exp;
      } else {                                // |S| < |g|: predecessor of |g|
        bool pow2 = (st.Y[NS - 1] == 0x80000000u);
#pragma unroll
        for (int i = 0; i < NS - 1; ++i) pow2 = pow2 && (st.Y[i] == 0);
        if (pow2) {
#pragma unroll
          for (int i = 0; i < NS; ++i) st.Y[i] = keep_mask<NS>(i, p);
          st.r_exp = st.g_exp - 1;
        } else {
          const int cut = 32 * NS - p;
          uint32_t one[NS];
#pragma unroll
          for (int i = 0; i < NS; ++i) one[i] = (i == (cut >> 5)) ? (1u << (cut & 31)) : 0u;
          madd_masked<NS>(st.Y, one, 0xFFFFFFFFu, 1u);
          st.r_exp = st.g_exp;
        }
      }
      st.done = true;
      return;
    }
  }
  if (cont) {
    if (new_top >= st.top || st.levels >= kMaxLevels) {
      st.bad = true;
      st.done = true;
      return;
    }
    st.top = new_top;
  }
}

template <int NS>
ARB_HD void level_init(Level<NS> &st, int top) {
  st.top = top;
  st.have_g = false;
  st.g_sign = 0;
  st.g_exp = 0;
  st.done = st.bad = st.zero = st.inexact = false;
  st.r_sign = 0;
  st.r_exp = 0;
  st.levels = 0;
#pragma unroll
  for (int i = 0; i < NS; ++i) st.Y[i] = 0;
}

}  // namespace arb

namespace arb {

// An operand whose limbs stay in memory; any length.  Used by the exact
// fallback, which must never truncate an operand.
struct SOpnd {
  const ARB_GLOBAL uint32_t *l;   // limb planes, most significant first
  int64_t ld;          // plane distance
  int64_t idx;         // element index
  int n;
  bool trunc;          // always false
  int e;
  uint32_t sign;
  double rm;
  int re;
  ARB_HD uint32_t limb_ls(int i) const {   // i-th limb from the bottom
    return l[(int64_t)(n - 1 - i) * ld + idx];
  }
};

ARB_HD double mag_upper(const SOpnd &o) {
  if (o.n == 0) return 0.0;
  uint32_t top = o.limb_ls(o.n - 1), second = o.n > 1 ? o.limb_ls(o.n - 2) : 0u;
  uint32_t rest = 0;
  for (int i = 0; i < o.n - 2; ++i) rest |= o.limb_ls(i);
  uint64_t v = ((uint64_t)top << 32) | second;
  uint64_t m53 = (v >> 11) + (((v & 0x7FFull) != 0 || rest != 0) ? 1 : 0);
  return (double)m53 * 0x1p-53;
}

// Exact window update with the product formed column by column from the
// bottom (a running 96-bit column sum carries into the next column), so the
// operands may have any length.  The last NS+1 product limbs at or below
// the window top pass through a shift register with static indices.
template <int NS>
ARB_HD void add_term(Window<NS> &W, int lo, const SOpnd &a, const SOpnd &b, uint32_t neg) {
  const int top = lo + 32 * NS;
  const int et = a.e + b.e;
  if (et <= lo) {
    W.err += 1;
    W.below_cnt += 1;
    W.below_max = et > W.below_max ? et : W.below_max;
    return;
  }
  const int base = et - 32 * (a.n + b.n);
  if (base >= top) return;
  const int s = lo - base;                       // window start, in product bits
  const int qs = (s >= 0) ? (s >> 5) : -((31 - s) >> 5);
  const int rs = s - 32 * qs;
  const int np = a.n + b.n;
  const int cend = qs + NS;                      // last product limb needed
  uint32_t X[NS + 1];
#pragma unroll
  for (int i = 0; i <= NS; ++i) X[i] = 0;
  uint32_t sticky = 0;
  uint64_t clo = 0;   // running column sum, low 64 bits
  uint32_t chi = 0;   // bits 64..95
  const int c0 = qs < 0 ? qs : 0;
  for (int c = c0; c <= cend; ++c) {
    uint32_t limb = 0;
    if (c >= 0 && c < np) {
      int i0 = c - (b.n - 1);
      if (i0 < 0) i0 = 0;
      int i1 = c < a.n - 1 ? c : a.n - 1;
      for (int i = i0; i <= i1; ++i) {
        uint64_t pr = (uint64_t)a.limb_ls(i) * b.limb_ls(c - i);
        uint64_t t = clo + pr;
        chi += (t < clo) ? 1u : 0u;
        clo = t;
      }
      limb = (uint32_t)clo;
      clo = (clo >> 32) | ((uint64_t)chi << 32);
      chi = 0;
    } else if (c >= np) {
      limb = (uint32_t)clo;
      clo >>= 32;
    }
    if (c < qs) {
      sticky |= limb;
    } else {
#pragma unroll
      for (int i = 0; i < NS; ++i) X[i] = X[i + 1];
      X[NS] = limb;
    }
  }
  sticky |= rs ? (X[0] << (32u - rs)) : 0u;
  uint32_t x[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = funnel(X[i + 1], X[i], (uint32_t)rs);
  if (sticky) { W.pt += 1; W.err += 1; }
  const uint32_t inv = neg ? 0xFFFFFFFFu : 0u;
  madd_masked<NS>(W.w, x, inv, neg);
}

ARB_HD double rad_term(const SOpnd &a, const SOpnd &b, int F) {
  double acc = 0.0;
  if (b.rm != 0.0 && a.n) acc = ru_add(acc, ru_scale_down(ru_mul(mag_upper(a), b.rm), a.e + b.re - F));
  if (a.rm != 0.0 && b.n) acc = ru_add(acc, ru_scale_down(ru_mul(mag_upper(b), a.rm), b.e + a.re - F));
  if (a.rm != 0.0 && b.rm != 0.0) acc = ru_add(acc, ru_scale_down(ru_mul(a.rm, b.rm), a.re + b.re - F));
  return acc;
}

ARB_HD int rad_exp(const SOpnd &a, const SOpnd &b, bool &any) {
  int f = -0x7FFFFFFF;
  if (b.rm != 0.0 && a.n) { f = a.e + b.re > f ? a.e + b.re : f; any = true; }
  if (a.rm != 0.0 && b.n) { f = b.e + a.re > f ? b.e + a.re : f; any = true; }
  if (a.rm != 0.0 && b.rm != 0.0) { f = a.re + b.re > f ? a.re + b.re : f; any = true; }
  return f;
}

ARB_HD bool opnd_out_of_range(const SOpnd &o) {
  if (o.n && (o.e >= kExpLimit || o.e <= -kExpLimit)) return true;
  if (o.rm != 0.0 && (o.re >= kExpLimit || o.re <= -kExpLimit)) return true;
  return false;
}

ARB_HD void setup_term(Setup &S, const SOpnd &a, const SOpnd &b, bool want_rad) {
  if (opnd_out_of_range(a) || opnd_out_of_range(b)) S.erange = true;
  if (a.n && b.n) {
    int et = a.e + b.e;
    S.emax = et > S.emax ? et : S.emax;
    S.nnz += 1;
  }
  if (want_rad) {
    bool any = false;
    int f = rad_exp(a, b, any);
    if (any) { S.any_rad = true; S.F = f > S.F ? f : S.F; }
  }
}

// Result of one output as produced by run_dot.
template <int NS>
struct DotOut {
  Level<NS> st;
  double rin_m;   // propagated radius rho_in = rin_m * 2^rin_e (upper bound)
  int rin_e;
  bool erange;
  int p;          // precision of the midpoint (below the request after a cut)
};

// Reducer for a single lane per output (no cross-lane traffic).
struct SoloReducer {
  ARB_HD static int lane() { return 0; }
  ARB_HD static int group() { return 1; }
  ARB_HD static void setup(Setup &) {}
  template <int NS>
  ARB_HD static void window(Window<NS> &) {}
  ARB_HD static void rad(RadAcc &) {}
};

// The whole dot-product pipeline for one output.  `Src` supplies the terms:
//   int64_t nterms() const;
//   bool has_init() const;
//   void term(int64_t t, Op& a, Op& b, uint32_t& neg, bool limbs) const;
//   void init(Op& a, Op& one, bool limbs) const;
// `Op` is Opnd<NA> (limbs in registers) or SOpnd (limbs read in place).
// Lane `Red::lane()` of `Red::group()` handles terms t = lane (mod group);
// lane 0 also handles the initial term.
// With `reduce`, the precision is first cut to
// p' = max(2, min(p, e_max - e_rad + 30)) from the setup statistics
// (Section 3.3, step 7(a)); e_max and e_rad bound the exponents of the
// midpoint and radius products, and p' = 2 when every midpoint product is 0.
template <int NS, class Op, class Red, class Src>
ARB_HD void run_dot(const Src &src, int p, bool want_rad, DotOut<NS> &out, bool reduce = false) {
  const int lane = Red::lane(), group = Red::group();
  const int64_t nt = src.nterms();
  const bool hi = src.has_init() && lane == 0;
  Setup S;
  S.clear();
  for (int64_t t = lane; t < nt; t += group) {
    Op a, b;
    uint32_t neg;
    src.term(t, a, b, neg, false);
    setup_term(S, a, b, want_rad || reduce);
  }
  if (hi) {
    Op a, b;
    src.init(a, b, false);
    setup_term(S, a, b, want_rad || reduce);
  }
  Red::setup(S);
  if (reduce) {
    int64_t q = S.nnz ? p : 2;
    if (S.nnz && S.any_rad && (int64_t)S.emax - S.F + 30 < q) q = (int64_t)S.emax - S.F + 30;
    p = q < 2 ? 2 : (int)q;
  }
  out.p = p;
  out.erange = S.erange;
  out.rin_m = 0.0;
  out.rin_e = 0;
  level_init(out.st, S.nnz ? S.emax + bitlen32(S.nnz) + 1 : 0);
  if (S.erange) {
    out.st.done = true;
    out.st.zero = true;
    return;
  }
  RadAcc racc;
  racc.clear();
  bool rad_pending = want_rad && S.any_rad;
  if (S.nnz == 0) {
    out.st.zero = true;
    out.st.done = true;
  }
  while (!out.st.done) {
    Window<NS> W;
    W.clear();
    const int lo = out.st.top - 32 * NS;
    for (int64_t t = lane; t < nt; t += group) {
      Op a, b;
      uint32_t neg;
      src.term(t, a, b, neg, true);
      if (a.n && b.n) add_term(W, lo, a, b, neg);
      if (rad_pending) racc.add(rad_term(a, b, S.F));
    }
    if (hi) {
      Op a, b;
      src.init(a, b, true);
      if (a.n) add_term(W, lo, a, b, a.sign);
      if (rad_pending) racc.add(rad_term(a, b, S.F));
    }
    Red::template window<NS>(W);
    if (rad_pending) {
      Red::rad(racc);
      rad_pending = false;
    }
    decide<NS>(out.st, W, lo, p);
  }
  if (rad_pending) {   // no midpoint pass ran: radius-only pass
    for (int64_t t = lane; t < nt; t += group) {
      Op a, b;
      uint32_t neg;
      src.term(t, a, b, neg, true);
      racc.add(rad_term(a, b, S.F));
    }
    if (hi) {
      Op a, b;
      src.init(a, b, true);
      racc.add(rad_term(a, b, S.F));
    }
    Red::rad(racc);
  }
  if (want_rad && S.any_rad) {
    double m;
    int e;
    if (racc.get(m, e)) {
      out.rin_m = m;
      out.rin_e = S.F + e;
    }
  }
}

// Output radius: rho_in plus one ulp 2^(e_m - p) of the truncated midpoint
// when the truncation lost bits; rounded up to (m in [0.5,1), e).
template <int NS>
ARB_HD void total_radius(const DotOut<NS> &o, int p, double &rm, int &re) {
  double um = 0.0;
  int ue = 0;
  if (!o.st.zero && o.st.inexact) { um = 0.5; ue = o.st.r_exp - p + 1; }
  ru_add_ext(o.rin_m, o.rin_e, um, ue, rm, re);
}

}  // namespace arb
