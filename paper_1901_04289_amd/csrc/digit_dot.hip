// Dot products of moderate precision as one small exact integer product on
// the INT8 matrix cores.
//
// Every operand of a dot is scaled to an integer in a frame of B = 224 LB
// bits and cut into L = 32 LB digits of 7 bits, each carrying the
// operand's sign, so that a digit fits an int8 whatever the sign.  With the
// terms of the dot along the inner dimension, the digits of the x operands
// as the rows of one matrix and those of the y operands as the columns of
// the other, one INT8 matrix product gives, for every digit pair, its sum
// over all terms; the integer sum of the dot is the sum of the product's
// anti-diagonals d weighted by 2^(7 d).  This is the scaled-integer product
// of Section 4 (Algorithm 2) for a 1 x N by N x 1 product with the digit
// indices in the place of rows and columns.  Term t's x operands are scaled
// by 2^(B - E + ey_t) and its y operands by 2^(B - ey_t) (ey_t the term's
// largest y exponent, E the largest exponent sum of a term), so every
// product has the unit 2^(E - 2B) and no term needs an alignment of its
// own; a complex dot takes both parts from the same digits (Section 3.6:
// the real part pairs x_re with y_re and x_im with -y_im, the imaginary part
// x_re with y_im and x_im with y_re).
//
// Operand bits below the frame are dropped, as the truncated products of
// Section 3.4 drop theirs: a product with a cut operand is off by less than
// 2^(B+1) + 1 units, counted as 3 units of the window 2^(E - B).  The window
// value with that bound either decides the truncation of the exact sum to p
// bits (the limb engine's decision on one window level, in registers) or
// the part goes back to the limb kernel, which refines (the fast dot with a
// fallback of Section 2).  The frame needs
// p + (E - e_max) + bitlen(terms) + 24 bits; a dot whose exponents spread
// wider than its blocks allow goes back the same way.  The radius is the
// limb engine's: the same per-term bounds (Section 3.5) added exactly in
// fixed point (RadAcc).
#include "limb_kernels.hpp"

using namespace arb;

namespace arbgpu_impl {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kDT = 256;           // threads per workgroup
constexpr int kDW = kDT / 64;      // waves
constexpr int kDigitGuard = 24;    // frame bits beyond p, the spread and the term count

template <int LB, bool CPLX>
struct DCfg {
  static constexpr int L = 32 * LB;             // digits per operand
  static constexpr int B = 224 * LB;            // frame bits
  static constexpr int NOP = CPLX ? 4 : 2;      // operands per term: x_re, x_im, y_re, y_im | x, y
  static constexpr int NPL = NOP;               // digit planes
  static constexpr int KC = CPLX ? 64 : 128;    // terms per chunk
  static constexpr int RS = KC + 16;            // bytes per digit row (padding against bank conflicts)
  // 32 x 32 blocks of the digit product that are formed (bs + bu >= LB - 2)
  static constexpr int NPAIR = LB * LB - (LB >= 3 ? (LB - 2) * (LB - 1) / 2 : 0);
  static constexpr int PPW = (NPAIR + kDW - 1) / kDW;
  static constexpr int NCOL = 14 * LB + 2;      // limbs of the integer sum (2 L digits + 64 bits)
  static constexpr int C0 = 7 * LB;             // window bottom: limb C0 has weight 2^B
};

template <int LB, bool CPLX>
struct DLds {
  using C = DCfg<LB, CPLX>;
  union {
    int8_t dig[C::NPL][C::L][C::RS];   // digit s of a chunk's terms: row s, term k at byte k
    struct {
      int64_t diag[2][2 * C::L];       // anti-diagonal sums per part
      int64_t col[2][C::NCOL];         // the integer sum per part, 32 bits per column
    } f;
  } u;
  // per operand and term of the chunk: the radius bound's inputs and flags
  double mag[C::NOP][C::KC], rm[C::NOP][C::KC];
  int re[C::NOP][C::KC], ex[C::NOP][C::KC], fl[C::NOP][C::KC];   // fl: 1 nonzero, 2 cut by the frame
  int red[kDW][10];
  RadAcc rad[kDW];
  uint32_t ntr[kDW];
  int job;
};

// An operand's sign, exponent, limb count and radius, as the limb kernels
// load them (load_op), without the limbs.
struct Meta {
  int n;
  uint32_t sign;
  int e;
  double rm;
  int re;
};

// Branch-free: every load is issued whatever the values, so the loads of a
// term go out together (a load under a value-dependent branch would wait
// for the one before it).
__device__ __forceinline__ void load_meta(const arbgpu_arr &A, int64_t idx, Meta &m) {
  const int32_t nl = gp(A.nls)[idx];
  const int e = gp(A.exp)[idx];
  double r = 0.0;
  int rexp = 0;
  if (A.rad_m) {   // uniform
    r = gp(A.rad_m)[idx];
    rexp = gp(A.rad_e)[idx];
  }
  int n = nl & 0x7FFFFFFF;
  m.n = n > A.cap ? A.cap : n;
  m.sign = (uint32_t)nl >> 31;
  m.e = e;
  int ex = 0;
  const double fm = frexp(r, &ex);
  const bool fin = r > 0.0 && r < INFINITY;
  m.rm = fin ? fm : (r != 0.0 ? 1.0 : 0.0);
  m.re = fin ? rexp + ex : (r != 0.0 ? kExpLimit : 0);
}

__device__ __forceinline__ bool meta_out_of_range(const Meta &o) {
  if (o.n && (o.e >= kExpLimit || o.e <= -kExpLimit)) return true;
  if (o.rm != 0.0 && (o.re >= kExpLimit || o.re <= -kExpLimit)) return true;
  return false;
}

__device__ __forceinline__ int meta_rad_exp(const Meta &a, const Meta &b, bool &any) {
  int f = -0x7FFFFFFF;
  if (b.rm != 0.0 && a.n) { f = a.e + b.re > f ? a.e + b.re : f; any = true; }
  if (a.rm != 0.0 && b.n) { f = b.e + a.re > f ? b.e + a.re : f; any = true; }
  if (a.rm != 0.0 && b.rm != 0.0) { f = a.re + b.re > f ? a.re + b.re : f; any = true; }
  return f;
}

// rad_term of the limb engine on staged values (mag: mag_upper of the operand).
__device__ __forceinline__ double staged_rad_term(bool an, int ae, double amag, double arm, int are, bool bn, int be,
                                                  double bmag, double brm, int bre, int F) {
  double acc = 0.0;
  if (brm != 0.0 && an) acc = ru_add(acc, ru_scale_down(ru_mul(amag, brm), ae + bre - F));
  if (arm != 0.0 && bn) acc = ru_add(acc, ru_scale_down(ru_mul(bmag, arm), be + are - F));
  if (arm != 0.0 && brm != 0.0) acc = ru_add(acc, ru_scale_down(ru_mul(arm, brm), are + bre - F));
  return acc;
}

__device__ __forceinline__ void write_erange(const arbgpu_out &R, int64_t idx, int p, bool approx) {
  const int PL = (p + 31) >> 5;
  for (int k = 0; k < PL; ++k) gpw(R.limbs)[(int64_t)k * R.ld + idx] = 0u;
  gpw(R.exp)[idx] = 0;
  gpw(R.nls)[idx] = 0;
  if (!approx) {
    gpw(R.rad_m)[idx] = INFINITY;
    gpw(R.rad_e)[idx] = 0;
  }
  if (R.status) gpw(R.status)[idx] = ARBGPU_ST_ERANGE;
}

// Job parameters read from memory are the same in every lane: held in
// scalar registers (the compiler cannot prove that for a global load).
__device__ __forceinline__ int32_t uni32(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T *uniptr(T *p) {
  return reinterpret_cast<T *>(uni64(reinterpret_cast<int64_t>(p)));
}
__device__ __forceinline__ arbgpu_arr uni_arr(const arbgpu_arr &a) {
  arbgpu_arr r;
  r.limbs = uniptr(a.limbs);
  r.ld = uni64(a.ld);
  r.cap = uni32(a.cap);
  r.exp = uniptr(a.exp);
  r.nls = uniptr(a.nls);
  r.rad_m = uniptr(a.rad_m);
  r.rad_e = uniptr(a.rad_e);
  return r;
}

__device__ __forceinline__ int ifloor32(int v) { return v >= 0 ? (v >> 5) : -((31 - v) >> 5); }

// Bytewise negation of int8 digits in [-127, 127]: with b' = b xor 0x80 in
// [1, 255], -b xor 0x80 = 256 - b', and 0x01010100 - (b'3 b'2 b'1 b'0)
// forms 256 - b' in every byte (each borrow is taken by the 1 above it).
__device__ __forceinline__ v4i neg_digits(v4i a) {
  v4i r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = (int)((0x01010100u - ((uint32_t)a[k] ^ 0x80808080u)) ^ 0x80808080u);
  return r;
}

// One dot job on one workgroup.  P[q] is the task of part q (real part
// first).  fb(q, bool) is called once per part by one thread: true when the
// limb kernel must redo part q (nothing has been written for it then).
template <int LB, bool CPLX, class PP, class FB>
__device__ void digit_job(PP P0, PP P1, DLds<LB, CPLX> &S, const FB &fb) {
  using C = DCfg<LB, CPLX>;
  constexpr int NPART = CPLX ? 2 : 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t N = uni64(P0->N);
  const bool approx = uni32(P0->approx) != 0, want_rad = !approx, reduce = uni32(P0->reduce) != 0;
  const uint32_t sub = (uint32_t)uni32((int32_t)P0->sub);
  const int NA = uni32(P0->na);
  const int preq = uni32(P0->p);
  const arbgpu_arr Xr = uni_arr(P0->X[0]), Yr = uni_arr(P0->Y[0]);
  const arbgpu_arr Xi = CPLX ? uni_arr(P0->X[1]) : Xr, Yi = CPLX ? uni_arr(P0->Y[1]) : Yr;
  const int64_t xoff = uni64(P0->xoff), xstep = uni64(P0->xstep), yoff = uni64(P0->yoff), ystep = uni64(P0->ystep);

  // ---- setup pass (Section 3.3): per part e_max, nonzero products and the
  // radius frame; the job's exponent frame E and the range check
  int emax[2] = {-0x7FFFFFFF, -0x7FFFFFFF}, F[2] = {-0x7FFFFFFF, -0x7FFFFFFF};
  uint32_t nnz[2] = {0u, 0u};
  int anyr[2] = {0, 0};
  int erange = 0, E = -0x7FFFFFFF;
  for (int64_t t = tid; t < N; t += kDT) {
    Meta o[4];
    load_meta(Xr, xoff + t * xstep, o[0]);
    load_meta(Yr, yoff + t * ystep, o[2]);
    if (CPLX) {
      load_meta(Xi, xoff + t * xstep, o[1]);
      load_meta(Yi, yoff + t * ystep, o[3]);
    } else {
      o[1].n = 0; o[1].rm = 0.0; o[3].n = 0; o[3].rm = 0.0;
      o[1].e = o[3].e = 0; o[1].re = o[3].re = 0; o[1].sign = o[3].sign = 0;
    }
    // products (part, x operand, y operand)
    constexpr int NPR = CPLX ? 4 : 1;
    const int pa[4] = {0, 1, 0, 1}, pb[4] = {2, 3, 3, 2}, pp[4] = {0, 0, 1, 1};
#pragma unroll
    for (int r = 0; r < NPR; ++r) {
      const Meta &a = o[pa[r]], &b = o[pb[r]];
      const int q = pp[r];
      if (meta_out_of_range(a) || meta_out_of_range(b)) erange = 1;
      if (a.n && b.n) {
        const int et = a.e + b.e;
        emax[q] = et > emax[q] ? et : emax[q];
        nnz[q] += 1;
      }
      if (want_rad || reduce) {
        bool any = false;
        const int f = meta_rad_exp(a, b, any);
        if (any) { anyr[q] = 1; F[q] = f > F[q] ? f : F[q]; }
      }
    }
    int exm = -0x7FFFFFFF, eym = -0x7FFFFFFF;
    if (o[0].n) exm = o[0].e;
    if (o[1].n && o[1].e > exm) exm = o[1].e;
    if (o[2].n) eym = o[2].e;
    if (o[3].n && o[3].e > eym) eym = o[3].e;
    if (exm != -0x7FFFFFFF && eym != -0x7FFFFFFF && exm + eym > E) E = exm + eym;
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      int v = __shfl_xor(emax[q], m, 64);
      emax[q] = v > emax[q] ? v : emax[q];
      nnz[q] += (uint32_t)__shfl_xor((int)nnz[q], m, 64);
      v = __shfl_xor(F[q], m, 64);
      F[q] = v > F[q] ? v : F[q];
      anyr[q] |= __shfl_xor(anyr[q], m, 64);
    }
    erange |= __shfl_xor(erange, m, 64);
    const int v = __shfl_xor(E, m, 64);
    E = v > E ? v : E;
  }
  if (lane == 0) {
    int *r = S.red[wave];
    r[0] = emax[0]; r[1] = (int)nnz[0]; r[2] = F[0]; r[3] = anyr[0];
    r[4] = emax[1]; r[5] = (int)nnz[1]; r[6] = F[1]; r[7] = anyr[1];
    r[8] = erange; r[9] = E;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) { emax[q] = -0x7FFFFFFF; nnz[q] = 0; F[q] = -0x7FFFFFFF; anyr[q] = 0; }
  erange = 0;
  E = -0x7FFFFFFF;
  for (int w = 0; w < kDW; ++w) {
    const int *r = S.red[w];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      emax[q] = r[4 * q] > emax[q] ? r[4 * q] : emax[q];
      nnz[q] += (uint32_t)r[4 * q + 1];
      F[q] = r[4 * q + 2] > F[q] ? r[4 * q + 2] : F[q];
      anyr[q] |= r[4 * q + 3];
    }
    erange |= r[8];
    E = r[9] > E ? r[9] : E;
  }
  __syncthreads();

  // precision of each part (the radius-driven cut, Section 3.3 step 7(a))
  int prec[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    int pq = preq;
    if (reduce) {
      int64_t v = nnz[q] ? pq : 2;
      if (nnz[q] && anyr[q] && (int64_t)emax[q] - F[q] + 30 < v) v = (int64_t)emax[q] - F[q] + 30;
      pq = v < 2 ? 2 : (int)v;
    }
    prec[q] = pq;
  }
  if (erange) {
    if (tid == 0) write_erange(P0->R, P0->res_idx, P0->p, approx);
    if (CPLX && tid == 64) write_erange(P1->R, P1->res_idx, P1->p, approx);
    if (tid == 0) fb(0, false);
    if (CPLX && tid == 64) fb(1, false);
    __syncthreads();
    return;
  }
  {   // does the frame hold every part's p bits, spread and guard?
    const int64_t kp = N * (CPLX ? 2 : 1);
    const int bk = 64 - __builtin_clzll((uint64_t)kp | 1ull);
    bool fits = true;
#pragma unroll
    for (int q = 0; q < NPART; ++q)
      if (nnz[q] && (int64_t)prec[q] + ((int64_t)E - emax[q]) + bk + kDigitGuard > C::B) fits = false;
    if (!fits) {
      if (tid == 0) fb(0, true);
      if (CPLX && tid == 64) fb(1, true);
      __syncthreads();
      return;
    }
  }
  if (E == -0x7FFFFFFF) E = 0;   // no term has a nonzero x and a nonzero y: every digit product is 0

  // ---- main pass: digits of a chunk of terms, their product, the radius
  v16i acc[NPART][C::PPW];
#pragma unroll
  for (int q = 0; q < NPART; ++q)
#pragma unroll
    for (int i = 0; i < C::PPW; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[q][i][r] = 0;
  RadAcc racc;
  racc.clear();
  uint32_t ntr = 0;
  // conversion: thread (operand, term of the chunk)
  const int cop = CPLX ? wave : (wave & 1);
  const int ck = CPLX ? lane : lane + 64 * (wave >> 1);
  const bool isx = CPLX ? cop < 2 : cop == 0;
  const arbgpu_arr A = CPLX ? (cop == 0 ? Xr : cop == 1 ? Xi : cop == 2 ? Yr : Yi) : (cop == 0 ? Xr : Yr);
  // radius and cut counting: thread (product, term)
  const int rpa = CPLX ? (wave & 1) : 0;
  const int rpb = CPLX ? (wave == 0 ? 2 : wave == 1 ? 3 : wave == 2 ? 3 : 2) : 1;
  const int rpart = CPLX ? (wave >> 1) : 0;
  const int rk = CPLX ? lane : lane + 64 * (wave & 1);
  const bool ract = CPLX ? true : wave < 2;
  const bool rad_on = want_rad && (rpart ? anyr[1] : anyr[0]);
  const int Fr = rpart ? F[1] : F[0];
  // kept blocks of the digit product: (bs, bu) with bs + bu >= LB - 2; the
  // others add less than 2^-200 units of the window together (each block's
  // sum is below 2^(224 (bs + bu + 2 - LB)) K units, K < 2^18 products)
  int pbs[C::PPW], pbu[C::PPW];
#pragma unroll
  for (int i = 0; i < C::PPW; ++i) {
    pbs[i] = -1;
    pbu[i] = 0;
    int cnt = 0;
    for (int a = 0; a < LB; ++a)
      for (int b = 0; b < LB; ++b)
        if (a + b >= LB - 2) {
          if (cnt == wave + kDW * i) { pbs[i] = a; pbu[i] = b; }
          ++cnt;
        }
  }

  for (int64_t k0 = 0; k0 < N; k0 += C::KC) {
    {
      // every read below is from a valid index (term 0 stands in for terms
      // past the end, plane 0 or n - 1 for planes outside the operand) and
      // issued unconditionally, so the loads of a chunk go out together
      const int64_t t = k0 + ck;
      const bool live = t < N;
      const int64_t tt = live ? t : 0;
      const int64_t idx = isx ? xoff + tt * xstep : yoff + tt * ystep;
      const int64_t yix = yoff + tt * ystep;
      const ARB_GLOBAL uint32_t *LB0 = gp(A.limbs) + idx;
      const uint32_t ld32 = (uint32_t)A.ld;   // below 2^31 on this path
      Meta m;
      load_meta(A, idx, m);
      const int32_t n0 = gp(Yr.nls)[yix] & 0x7FFFFFFF;
      const int e0 = gp(Yr.exp)[yix];
      int32_t n1 = 0;
      int e1 = 0;
      if (CPLX) {
        n1 = gp(Yi.nls)[yix] & 0x7FFFFFFF;
        e1 = gp(Yi.exp)[yix];
      }
      const uint32_t top = LB0[0], second = LB0[A.cap > 1 ? (uint64_t)ld32 : 0];
      int ey = n0 ? e0 : -0x7FFFFFFF;
      ey = (n1 && e1 > ey) ? e1 : ey;
      m.n = live ? m.n : 0;
      const bool zero = m.n == 0 || ey == -0x7FFFFFFF;
      // leading zero bits of the operand in its frame
      const int z = zero ? 0 : (isx ? E - ey - m.e : ey - m.e);
      const bool cut = !zero && 32 * (int64_t)m.n > (int64_t)C::B - z;
      const int nc = m.n > 0 ? m.n - 1 : 0;
      // limbs JL .. JL + 7 LB (from the top) cover the frame; R aligns them
      constexpr int NL = 7 * LB + 1;
      const int JL = ifloor32(-z);
      const uint32_t R = (uint32_t)(-z - 32 * JL);
      uint32_t lim[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int j = JL + q;
        const uint32_t jc = (uint32_t)(j < 0 ? 0 : (j > nc ? nc : j));
        lim[q] = LB0[(uint64_t)jc * ld32];
      }
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int j = JL + q;
        lim[q] = (!zero && j >= 0 && j < m.n) ? lim[q] : 0u;
      }
      double mg = 0.0;
      if (want_rad && m.n) {   // mag_upper of the limb engine's operand (top min(n, NA) limbs)
        const int nt = m.n < NA ? m.n : NA;
        const uint64_t v = ((uint64_t)top << 32) | (nt > 1 ? second : 0u);
        bool rest = m.n > NA;
        if (!rest && (v & 0x7FFull) == 0)
          for (int j = 2; j < nt && !rest; ++j) rest = LB0[(uint64_t)j * ld32] != 0;
        const uint64_t m53 = (v >> 11) + (((v & 0x7FFull) != 0 || rest) ? 1 : 0);
        mg = (double)m53 * 0x1p-53;
      }
      S.mag[cop][ck] = mg;
      S.rm[cop][ck] = m.rm;
      S.re[cop][ck] = m.re;
      S.ex[cop][ck] = m.e;
      S.fl[cop][ck] = (m.n ? 1 : 0) | (cut ? 2 : 0);
      // the frame's bits from the top, 32 to a word
#pragma unroll
      for (int q = 0; q < NL - 1; ++q) lim[q] = R ? ((lim[q] << R) | (lim[q + 1] >> (32u - R))) : lim[q];
      lim[NL - 1] = 0;
      const int sg = ((m.sign ^ (isx ? sub : 0u)) & 1u) ? -1 : 1;
      // digit s (weight 2^(7 s)) is bits [7 (L - 1 - s), +7) from the top
      auto bits_of = [&](int s) -> int {
        const int o = 7 * (C::L - 1 - s), q = o >> 5, r = o & 31;
        return (int)(r <= 25 ? (lim[q] >> (25 - r)) & 0x7Fu : ((lim[q] << (r - 25)) | (lim[q + 1] >> (57 - r))) & 0x7Fu);
      };
      // (the empty asm after every 8 digits keeps the compiler from forming
      // every digit before the first store, a register each)
      int8_t *row0 = &S.u.dig[cop][0][ck];
#pragma unroll
      for (int s = 0; s < C::L; ++s) {
        row0[s * C::RS] = (int8_t)(bits_of(s) * sg);
        if ((s & 7) == 7) asm volatile("" ::: "memory");
      }
    }
    __syncthreads();
    // digit products: wave w takes the blocks w, w + 4, ...
#pragma unroll
    for (int i = 0; i < C::PPW; ++i) {
      if (pbs[i] >= 0) {
        const int bs = pbs[i], bu = pbu[i];
#pragma unroll
        for (int ks = 0; ks < C::KC / 32; ++ks) {
          const int cb = 32 * ks + 16 * (lane >> 5);
          const int ra = 32 * bs + (lane & 31), rb = 32 * bu + (lane & 31);
          if (CPLX) {
            const v4i ar = *reinterpret_cast<const v4i *>(&S.u.dig[0][ra][cb]);
            const v4i ai = *reinterpret_cast<const v4i *>(&S.u.dig[1][ra][cb]);
            const v4i br = *reinterpret_cast<const v4i *>(&S.u.dig[2][rb][cb]);
            const v4i bi = *reinterpret_cast<const v4i *>(&S.u.dig[3][rb][cb]);
            const v4i an = neg_digits(ai);
            acc[0][i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ar, br, acc[0][i], 0, 0, 0);
            acc[0][i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(an, bi, acc[0][i], 0, 0, 0);
            acc[NPART - 1][i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ar, bi, acc[NPART - 1][i], 0, 0, 0);
            acc[NPART - 1][i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ai, br, acc[NPART - 1][i], 0, 0, 0);
          } else {
            const v4i a = *reinterpret_cast<const v4i *>(&S.u.dig[0][ra][cb]);
            const v4i b = *reinterpret_cast<const v4i *>(&S.u.dig[1][rb][cb]);
            acc[0][i] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[0][i], 0, 0, 0);
          }
        }
      }
    }
    // radius terms and cut products of the chunk
    if (ract && k0 + rk < N) {
      const int fa = S.fl[rpa][rk], fbv = S.fl[rpb][rk];
      if ((fa & fbv & 1) && ((fa | fbv) & 2)) ++ntr;
      if (rad_on)
        racc.add(staged_rad_term(fa & 1, S.ex[rpa][rk], S.mag[rpa][rk], S.rm[rpa][rk], S.re[rpa][rk], fbv & 1,
                                 S.ex[rpb][rk], S.mag[rpb][rk], S.rm[rpb][rk], S.re[rpb][rk], Fr));
    }
    __syncthreads();
  }

  // ---- anti-diagonal sums, the integer sum, certification, output
  for (int w = tid; w < NPART * (2 * C::L + C::NCOL); w += kDT) {
    if (w < NPART * 2 * C::L) S.u.f.diag[w / (2 * C::L)][w % (2 * C::L)] = 0;
    else {
      const int v = w - NPART * 2 * C::L;
      S.u.f.col[v / C::NCOL][v % C::NCOL] = 0;
    }
  }
  WaveReducer::rad(racc);
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) ntr += (uint32_t)__shfl_xor((int)ntr, m, 64);
  if (lane == 0) {
    S.rad[wave] = racc;
    S.ntr[wave] = ract ? ntr : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < C::PPW; ++i) {
    if (pbs[i] >= 0) {
      const int bs = pbs[i], bu = pbu[i];
#pragma unroll
      for (int pt = 0; pt < NPART; ++pt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int s = 32 * bs + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), u = 32 * bu + (lane & 31);
          atomicAdd(reinterpret_cast<unsigned long long *>(&S.u.f.diag[pt][s + u]),
                    (unsigned long long)(int64_t)acc[pt][i][r]);
        }
    }
  }
  __syncthreads();
  for (int w = tid; w < NPART * 2 * C::L; w += kDT) {
    const int pt = w / (2 * C::L), d = w % (2 * C::L);
    const int64_t v = S.u.f.diag[pt][d];
    if (v) {
      const int b = 7 * d, c = b >> 5, r = b & 31;
      const uint64_t sl = ((uint64_t)v & 0xFFFFFFFFull) << r;
      const int64_t hv = (v >> 32) * ((int64_t)1 << r);
      atomicAdd(reinterpret_cast<unsigned long long *>(&S.u.f.col[pt][c]), sl & 0xFFFFFFFFull);
      atomicAdd(reinterpret_cast<unsigned long long *>(&S.u.f.col[pt][c + 1]),
                (unsigned long long)((int64_t)(sl >> 32) + hv));
    }
  }
  __syncthreads();
  // per part, one lane: the columns' carries in registers, then the limb
  // engine's decision (a single window level) and output; a part that the
  // window does not decide goes to the limb kernel
  if (lane == 0 && wave < NPART) {
    constexpr int NW = C::NCOL - C::C0;   // window limbs
    const int pt = wave;
    PP P = pt ? P1 : P0;
    const int64_t *col = S.u.f.col[pt];
    Window<NW> Wd;
    Wd.clear();
    int64_t cy = 0;
    bool lownz = false;
#pragma unroll
    for (int c = 0; c < C::NCOL; ++c) {
      const int64_t v = col[c] + cy;
      cy = v >> 32;
      if (c < C::C0) lownz |= (v & 0xFFFFFFFFll) != 0;
      else Wd.w[c - C::C0] = (uint32_t)v;
    }
    uint32_t nt = 0;
    RadAcc rt;
    rt.clear();
    for (int w = 0; w < kDW; ++w) {
      const int wp = CPLX ? (w >> 1) : 0;
      if (wp == pt) {
        nt += S.ntr[w];
        rt.add(S.rad[w]);
      }
    }
    // 3 units per product with a cut operand, 1 for the bits below the
    // window, 1 for the blocks left out
    Wd.err = 3u * nt + (lownz ? 1u : 0u) + (LB >= 3 ? 1u : 0u);
    Wd.pt = nt;
    const int p = pt ? prec[1] : prec[0];
    const int Fp = pt ? F[1] : F[0];
    const bool radp = want_rad && (pt ? anyr[1] : anyr[0]);
    const int lo = E - C::B;   // the window's unit 2^(E - B)
    DotOut<NW> out;
    level_init(out.st, lo + 32 * NW);
    decide<NW>(out.st, Wd, lo, p);
    const bool ok = out.st.done && !out.st.bad;
    if (ok) {
      out.rin_m = 0.0;
      out.rin_e = 0;
      if (radp) {
        double m;
        int e;
        if (rt.get(m, e)) {
          out.rin_m = m;
          out.rin_e = Fp + e;
        }
      }
      out.erange = false;
      out.p = p;
      store_out<NW>(P->R, P->res_idx, out, P->p, approx, ARBGPU_ST_OK);
    }
    fb(pt, !ok);
  }
  __syncthreads();
}

template <int LB, bool CPLX>
__global__ __launch_bounds__(kDT) void digit_dot_kernel(DotParams p0, DotParams p1, int32_t *flags) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  auto &S = *reinterpret_cast<DLds<LB, CPLX> *>(smem);
  auto fb = [&](int q, bool redo) { gpw(flags)[q] = redo ? 1 : 0; };
  digit_job<LB, CPLX>(&p0, &p1, S, fb);
}

// Persistent batch: each workgroup takes jobs from the run's counter; a
// part that needs the limb kernel is appended to its shape's list.
// Waves per SIMD the batch kernel is compiled for (its register budget;
// the complex kernel of 5 blocks holds 160 accumulators per lane and runs
// one wave per SIMD rather than spill them).
template <int LB, bool CPLX>
constexpr int digit_waves() {
  return LB <= 2 ? 4 : (LB == 3 ? 3 : (LB == 5 && CPLX ? 1 : 2));
}

template <int LB, bool CPLX>
__global__ __launch_bounds__(kDT) __attribute__((amdgpu_waves_per_eu(digit_waves<LB, CPLX>(), 8))) void digit_dot_batch_kernel(
    DigitBatchParams bp) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  auto &S = *reinterpret_cast<DLds<LB, CPLX> *>(smem);
  for (int64_t iter = 0; iter <= bp.count; ++iter) {
    if (threadIdx.x == 0) S.job = atomicAdd(bp.counter, 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(S.job);
    __syncthreads();
    if (t >= bp.count) break;   // uniform across the workgroup
    const int32_t e = __builtin_amdgcn_readfirstlane(gp(bp.order)[t]);
    const ARB_GLOBAL DotParams *P0 = gp(bp.tasks) + e;
    auto fb = [&](int q, bool redo) {
      if (!redo) return;
      const int32_t task = e + q;
      const int f = gp(bp.tasks)[task].fb;
      const int32_t slot = atomicAdd(bp.fb_count + f, 1);
      gpw(bp.fb_list)[gp(bp.fb_base)[f] + slot] = task;
    };
    digit_job<LB, CPLX>(P0, P0 + (CPLX ? 1 : 0), S, fb);
  }
}

template <int LB, bool CPLX>
size_t lds_of() {
  return sizeof(DLds<LB, CPLX>);
}

}  // namespace

int digit_blocks(const DotParams &prm, LimbShape sh) {
  if (prm.has_init || sh.ns == 0 || prm.N <= 0 || prm.N > 65536) return 0;
  for (int k = 0; k < prm.ct.ncomp; ++k)   // 32-bit plane offsets
    if (prm.X[k].ld >= ((int64_t)1 << 31) || prm.Y[k].ld >= ((int64_t)1 << 31)) return 0;
  // frame for p, the term count, the guard and the spread E - e_max: none
  // for a real dot (E is its largest product exponent), 40 bits allowed
  // for a complex one (E pairs each term's larger x and y parts)
  const int64_t kp = prm.N * prm.ct.ncomp;
  int bk = 0;
  for (int64_t v = kp; v; v >>= 1) ++bk;
  const int64_t need = (int64_t)prm.p + (prm.ct.ncomp == 2 ? 40 : 0) + bk + kDigitGuard;
  const int64_t lb = (need + 223) / 224;
  return lb <= kDigitMaxBlocks ? (int)lb : 0;
}

#define ARB_DIGIT_CASES(X) X(1) X(2) X(3) X(4) X(5)

hipError_t launch_digit_dot(const DotParams *prm, int lb, int32_t *flags, hipStream_t s) {
  const bool cplx = prm[0].ct.ncomp == 2;
  const DotParams &p1 = cplx ? prm[1] : prm[0];
#define X(b)                                                                                              \
  if (lb == b) {                                                                                          \
    if (cplx)                                                                                             \
      hipLaunchKernelGGL((digit_dot_kernel<b, true>), dim3(1), dim3(kDT), (lds_of<b, true>()), s, prm[0], p1, \
                         flags);                                                                          \
    else                                                                                                  \
      hipLaunchKernelGGL((digit_dot_kernel<b, false>), dim3(1), dim3(kDT), (lds_of<b, false>()), s, prm[0], \
                         p1, flags);                                                                      \
    return hipGetLastError();                                                                             \
  }
  ARB_DIGIT_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

const void *digit_dot_batch_kernel(int lb, bool cplx, size_t *lds_bytes) {
#define X(b)                                                                              \
  if (lb == b) {                                                                          \
    *lds_bytes = cplx ? lds_of<b, true>() : lds_of<b, false>();                          \
    return cplx ? reinterpret_cast<const void *>(&digit_dot_batch_kernel<b, true>)       \
                : reinterpret_cast<const void *>(&digit_dot_batch_kernel<b, false>);     \
  }
  ARB_DIGIT_CASES(X)
#undef X
  *lds_bytes = 0;
  return nullptr;
}

}  // namespace arbgpu_impl
