// Multimodular (residue number system) form of the scaled-integer block
// product.  The paper multiplies its integer matrices with FLINT, whose
// fast path works modulo word-size primes followed by Chinese remainder
// reconstruction (introduction of Section 4).  Here every scaled integer Y
// of a block is reduced modulo m odd primes p_j < 2^15, each residue
// (balanced, |r| < 2^14) is split into two int8 digits r = lo + 256 hi, and
// the digit products run on the INT8 MFMA kernel (mfma_rns.hip), which
// folds a prime's four digit products into one int16 residue per entry.
// The exact T is rebuilt per entry by the explicit Chinese remainder
// formula, exact whenever prod p_j > 4 |T|.  The MFMA work is 4 m digit
// products instead of L_A L_B base-256 slices.
//
// The per-prime tables are the same for every thread and are read through
// the constant address space, so they arrive by scalar loads; the digit
// tables of the two matrix products (weights 256^a mod p_j, quotients
// P / p_j) are MFMA operands.
#include "elements.hpp"
#include "finish.hpp"
#include "sliced.hpp"

namespace arbgpu_impl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cp(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

// x mod p for 0 <= x < 2^32 and 2^14 < p < 2^15 (Barrett with mu =
// floor(2^32 / p): the quotient estimate is short by at most one, so one
// correction suffices; it is below 2^18, so q p is an exact 24-bit product).
__device__ __forceinline__ uint32_t mod_u32(uint32_t x, uint32_t p, uint32_t mu) {
  const uint32_t q = __umulhi(x, mu);
  const uint32_t r = x - __umul24(q, p);
  return r >= p ? r - p : r;
}

// Scaled integer of one plane element: its limbs, shift and sign.
struct SliceElem {
  int n = 0, part = 0;
  int64_t idx = 0, s = 0;
  uint32_t sg = 0;
};

__device__ __forceinline__ SliceElem slice_elem(const RnsSliceParams &P, int64_t line, int64_t k) {
  SliceElem e;
  const int64_t len_total = (P.mode == 0) ? P.len : 2 * P.len;
  if (line < P.lines && k < len_total) {
    int64_t kk;
    uint32_t ng;
    inner_map(P.mode, P.len, k, e.part, kk, ng);
    const arbgpu_arr &A = part_of(P.part, e.part);
    e.idx = P.off + line * P.line_stride + (P.k0 + kk) * P.elem_stride;
    const int nn = elem_n(A, e.idx);
    if (nn) {
      e.n = nn;
      e.sg = ((uint32_t)A.nls[e.idx] >> 31) ^ ng;
      e.s = (int64_t)A.exp[e.idx] - 32 * (int64_t)nn - P.v2[line];
    }
  }
  return e;
}

// Words 4 g .. 4 g + 4 NG - 1 (4 balanced base-256 digits each, int8) of
// Y: the digits of Y + B, B = sum_{a<L} 128 * 256^a, are bytes; those of Y
// are the bytes minus 128.  cy carries between words.  The 4 NG + 1 limbs
// that hold bits [128 g - s, 128 (g + NG) - s) of the mantissa are read
// first, all at once, so a run of NG words costs one memory round trip.
template <int NG>
__device__ __forceinline__ void digit_words(const RnsSliceParams &P, const SliceElem &e, int g, uint32_t &cy,
                                            uint32_t (&x)[4 * NG]) {
  constexpr int NL = 4 * NG + 1;
  uint32_t lim[NL];
#pragma unroll
  for (int t = 0; t < NL; ++t) lim[t] = 0u;
  const int64_t o = 128 * (int64_t)g - e.s;   // bit offset of word 4 g into M (may be negative)
  const int64_t li = o >= 0 ? (o >> 5) : -((31 - o) >> 5);
  const uint32_t r = (uint32_t)(o - 32 * li);
  if (e.n) {
    const arbgpu_arr &A = part_of(P.part, e.part);
    uint32_t v[NL];
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      // limb li + t counted from the least significant; clamped reads stay
      // inside the element's limbs and are discarded outside
      const int64_t i = li + t;
      const int64_t ic = i < 0 ? 0 : (i >= e.n ? e.n - 1 : i);
      v[t] = A.limbs[(int64_t)(e.n - 1 - ic) * A.ld + e.idx];
    }
    // the values are taken unconditionally, so the reads are issued
    // together rather than each behind its own range test
#pragma unroll
    for (int t = 0; t < NL; ++t) asm volatile("" : "+v"(v[t]));
#pragma unroll
    for (int t = 0; t < NL; ++t) lim[t] = (li + t >= 0 && li + t < e.n) ? v[t] : 0u;
  }
#pragma unroll
  for (int u = 0; u < 4 * NG; ++u) {
    const int w = 4 * g + u;
    const int nbytes = P.L - 4 * w;
    const uint32_t bmask = nbytes >= 4 ? 0xFFFFFFFFu : (nbytes <= 0 ? 0u : ((1u << (8 * nbytes)) - 1u));
    const uint32_t Bc = 0x80808080u & bmask;
    const uint32_t xv = r ? ((lim[u] >> r) | (lim[u + 1] << (32u - r))) : lim[u];
    uint64_t v;
    if (!e.sg) {
      v = (uint64_t)Bc + xv + cy;
      cy = (uint32_t)(v >> 32);
    } else {
      v = (uint64_t)Bc - xv - cy;
      cy = (uint32_t)((v >> 63) & 1u);
    }
    x[u] = (((uint32_t)v) ^ 0x80808080u) & bmask;
  }
}

// Residues of a sum from those of its terms, for 4 consecutive elements of
// a prime's planes: the terms' balanced residues (lo + 256 hi, |r| <=
// (p - 1) / 2) are added, brought back into the balanced range and split
// again.  lo4 / hi4 hold 4 bytes each.
__device__ __forceinline__ void residue_sum4(uint32_t xl, uint32_t xh, uint32_t yl, uint32_t yh, int32_t p,
                                             uint32_t &lo4, uint32_t &hi4) {
  const int32_t half = (p - 1) >> 1;
  lo4 = 0u;
  hi4 = 0u;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int32_t a = (int32_t)(int8_t)(xl >> (8 * u)) + 256 * (int32_t)(int8_t)(xh >> (8 * u));
    const int32_t b = (int32_t)(int8_t)(yl >> (8 * u)) + 256 * (int32_t)(int8_t)(yh >> (8 * u));
    int32_t r = a + b;
    r = r > half ? r - p : (r < -half ? r + p : r);
    const int32_t lo = ((r + 128) & 255) - 128;
    lo4 |= ((uint32_t)lo & 0xFFu) << (8 * u);
    hi4 |= ((uint32_t)((r - lo) >> 8) & 0xFFu) << (8 * u);
  }
}

// Residue of S = sum_a d_a 256^a (the lo sum plus 256 times the hi sum of
// the weight digits) modulo p, balanced and split into its int8 digits
// (lo, hi), returned as the bytes lo | hi << 8.
// |S| < 2^30 (4 nw <= 508 digits of |d_a| <= 128 against weight digits of
// magnitude <= 128 and <= 64), so S + kp, kp = p ceil(2^30 / p), lies in
// [0, 2^32).
__device__ __forceinline__ uint32_t residue_digits(uint32_t p, uint32_t mu, uint32_t kp, int32_t sum) {
  const uint32_t r = mod_u32((uint32_t)sum + kp, p, mu);
  const int32_t rb = r > (p >> 1) ? (int32_t)r - (int32_t)p : (int32_t)r;   // balanced, |rb| < 2^14
  const int32_t lo = ((rb + 128) & 255) - 128;
  return ((uint32_t)lo & 0xFFu) | ((((uint32_t)(rb - lo) >> 8) & 0xFFu) << 8);
}

// Fragments of steps k0 .. k0 + 3 of a run of 32-byte steps (at a + 32 ks;
// steps past nks repeat step k0 and are not used).
__device__ __forceinline__ void frag_load4(v4i (&f)[4], const int8_t *a, int k0, int nks) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int ks = k0 + u < nks ? k0 + u : k0;
    f[u] = *reinterpret_cast<const v4i *>(a + 32 * ks);
  }
}

// Rounding of one entry's T (W two's-complement limbs, limb q at T[q EW])
// to the output, by the G threads of the entry (part 0 .. G - 1; every
// thread of the workgroup calls it, live or not): the result of
// finish_entry, with the limb scans split into G ranges of limbs and the
// output limbs dealt out in turn; partial results meet in xs (G EW ints of
// LDS).
template <int EW, int G>
__device__ void finish_entry_split(const uint32_t *T, int W, int64_t scale, const arbgpu_out &C, int64_t oidx, int p,
                                   int approx, double rin_m, int rin_e, bool live, int e, int part, int32_t *xs) {
  auto get = [&](int q) -> uint32_t { return T[q * EW]; };
  const bool neg = (get(W - 1) >> 31) != 0;
  const int per = (W + G - 1) / G, qa = min(W, part * per), qb = min(W, qa + per);
  int z = W;   // lowest nonzero limb
  for (int q = qa; q < qb; ++q)
    if (get(q)) { z = q; break; }
  xs[part * EW + e] = z;
  __syncthreads();
  z = W;
  for (int k = 0; k < G; ++k) z = min(z, xs[k * EW + e]);
  __syncthreads();
  auto mag = [&](int q) -> uint32_t {
    if (q < 0 || q >= W) return 0u;
    const uint32_t v = get(q);
    if (!neg) return v;
    return q > z ? ~v : (q == z ? (uint32_t)(0u - v) : 0u);
  };
  int qt = -1;   // top nonzero limb of |T|
  for (int q = qb - 1; q >= qa; --q)
    if (mag(q)) { qt = q; break; }
  xs[part * EW + e] = qt;
  __syncthreads();
  qt = -1;
  for (int k = 0; k < G; ++k) qt = max(qt, xs[k * EW + e]);
  __syncthreads();
  const int PL = (p + 31) >> 5;
  int nout = 0;
  bool inexact = false;
  int64_t bl = 0;
  if (qt >= 0) {
    bl = 32 * (int64_t)qt + (32 - __builtin_clz(mag(qt)));
    auto bits32 = [&](int64_t lo) -> uint32_t {   // bits [lo, lo + 32) of |T|
      const int64_t q0 = lo >= 0 ? (lo >> 5) : -((31 - lo) >> 5);
      const uint32_t r = (uint32_t)(lo - 32 * q0);
      const uint32_t a = mag((int)q0), b = mag((int)q0 + 1);
      return r ? ((a >> r) | (b << (32u - r))) : a;
    };
    for (int k = part; k < PL; k += G) {
      uint32_t v = bits32(bl - 32 * (int64_t)(k + 1));
      if (k == PL - 1) v &= 0xFFFFFFFFu << (32 * PL - p);
      if (live) C.limbs[(int64_t)k * C.ld + oidx] = v;
      if (v) nout = k + 1;
    }
    // bits of |T| below position bl - p, in this thread's limbs
    const int64_t cut = bl - p;
    if (cut > 0) {
      const int64_t qc = cut >> 5;
      const uint32_t rc = (uint32_t)(cut & 31);
      for (int q = qa; q < qb && q < qc && !inexact; ++q) inexact = mag(q) != 0;
      if (rc && qc >= qa && qc < qb) inexact = inexact || (mag((int)qc) & ((1u << rc) - 1u)) != 0;
    }
  } else if (live) {
    for (int k = part; k < PL; k += G) C.limbs[(int64_t)k * C.ld + oidx] = 0u;
  }
  xs[part * EW + e] = nout | (inexact ? (1 << 30) : 0);
  __syncthreads();
  if (part == 0 && live) {
    int no = 0;
    bool ix = false;
    for (int k = 0; k < G; ++k) {
      const int v = xs[k * EW + e];
      no = max(no, v & 0x3FFFFFFF);
      ix = ix || ((v >> 30) & 1);
    }
    if (qt < 0) {
      C.exp[oidx] = 0;
      C.nls[oidx] = 0;
      if (!approx) {
        C.rad_m[oidx] = rin_m;
        C.rad_e[oidx] = rin_m != 0.0 ? rin_e : 0;
      }
    } else {
      const int em = (int)(bl + scale);
      C.exp[oidx] = em;
      C.nls[oidx] = (int32_t)((uint32_t)no | (neg ? 0x80000000u : 0u));
      if (!approx) {
        double rm = 0.0;
        int re = 0;
        arb::ru_add_ext(rin_m, rin_e, ix ? 0.5 : 0.0, em - p + 1, rm, re);
        C.rad_m[oidx] = rm;
        C.rad_e[oidx] = re;
      }
    }
    if (C.status) C.status[oidx] = ARBGPU_ST_OK;
  }
}

}  // namespace

// Residues of the plane elements on INT8 MFMA: r_j = sum_a d_a (256^a mod
// p_j) is an integer matrix product of the balanced base-256 digits d_a
// of the scaled integers with the int8 digits (lo, hi) of the weights
// 256^a mod p_j.  Workgroup: 256 threads, EL consecutive elements of the
// padded plane.  Phase 1: one thread per element writes its digits into an
// LDS row of kd bytes (+16 so that 8 consecutive rows fall in distinct
// 16-byte bank groups).  Phase 2: each wave takes one or two blocks of 32
// elements and loads each tile of 16 primes' weight fragments once for
// them; per block and tile one 32 x 32 MFMA result (elements x weight
// digits), whose lane l holds the lo or hi sum of one prime for 16
// elements.  Lane pairs combine lo + 256 hi by DPP exchanges; each lane of
// the pair reduces 8 of the 16 elements (its prime's constants sit in
// registers, loaded a tile ahead) and puts the residue digits of 8
// consecutive elements (the LDS rows are permuted for that) into an LDS
// stage of the tile's 32 planes; the workgroup then stores each plane's
// row of EL bytes whole (the padded plane holds whole blocks of 32
// elements and starts 16-byte aligned).  SUM (the imaginary part of an
// operand of the three-product complex form): the store pass also adds
// the real part's residues (P.addend, same layout), requested at the
// tile's start, and stores the residues of re + im into P.sum.
//
// With the stage the 256-element form's LDS (about 37 KiB at p = 512)
// admits four workgroups per CU, so registers are capped for four waves
// per SIMD (no spill) rather than five.
template <int EL, bool SUM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void rns_slice_kernel(RnsSliceParams P) {
  extern __shared__ __attribute__((aligned(16))) uint8_t dl[];   // [EL][kd + 16], then [32][EL]
  const int tid = threadIdx.x;
  const int nw = P.tab.nw, kd = P.tab.kd, S = kd + 16, m = P.tab.m;
  const int64_t total = P.lines_pad * P.k_pad;
  const int64_t g0 = (int64_t)blockIdx.x * EL;
  if (tid < EL) {
    const int64_t gid = g0 + tid;
    SliceElem e;
    if (gid < total) {
      const int64_t line = gid / P.k_pad;
      e = slice_elem(P, line, gid - line * P.k_pad);
    }
    // element x of a block of 32 sits in LDS row 16 x2 + 8 x4 + 4 x3 + x%4
    // (x_b: bit b of x): the MFMA result row 8 G + 4 h + i then holds
    // element 16 (G % 2) + 8 h + 4 (G / 2) + i, so that each lane reduces
    // 8 consecutive elements
    const int x = tid & 31;
    const int row = (tid & ~31) | (((x >> 2) & 1) << 4) | ((x >> 4) << 3) | (((x >> 3) & 1) << 2) | (x & 3);
    uint32_t cy = 0;
    uint8_t *drow0 = dl + (size_t)row * S;
    int w4 = 0;
    // runs of eight and of four 16-byte groups (one memory round trip
    // each), then single groups; words past nw have no digits (bmask 0), so
    // no run reaches there
    for (; w4 + 8 <= kd / 16 && 4 * (w4 + 7) < nw; w4 += 8) {
      uint32_t x[32];
      digit_words<8>(P, e, w4, cy, x);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        *reinterpret_cast<uint4 *>(drow0 + 16 * (w4 + q)) = make_uint4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
    }
    for (; w4 + 4 <= kd / 16 && 4 * (w4 + 3) < nw; w4 += 4) {
      uint32_t x[16];
      digit_words<4>(P, e, w4, cy, x);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<uint4 *>(drow0 + 16 * (w4 + q)) = make_uint4(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3]);
    }
    for (; w4 < kd / 16; ++w4) {
      uint32_t x[4] = {0u, 0u, 0u, 0u};
      if (4 * w4 < nw) digit_words<1>(P, e, w4, cy, x);
      *reinterpret_cast<uint4 *>(drow0 + 16 * w4) = make_uint4(x[0], x[1], x[2], x[3]);
    }
  }
  __syncthreads();
  // D = (element digits) x (weight digits): lane l holds column c = l % 32
  // of each 32 x 32 result, the lo (even c) or hi (odd c) sum of prime
  // 16 rt + c / 2, for elements 8 G + 4 h + i in register 4 G + i
  const int lane = tid & 63, wave = tid >> 6, h = lane >> 5, c = lane & 31, d = c & 1;
  // blocks of 32 elements per wave (waves past EL / 32 have none but take
  // part in the stores); the weight fragments of a prime tile are loaded
  // once for all of them
  constexpr int NBW = EL >= 128 ? EL / 128 : 1;
  // runs of four weight fragments requested at a tile's start besides the
  // prefetched first (register budget: one with two blocks per wave)
  constexpr int NPRE = NBW > 1 ? 1 : 2;
  const bool act = wave < EL / 32;
  // a tile's 32 planes x EL elements, staged so that the stores write
  // whole plane rows of EL bytes
  uint8_t *stage = dl + (size_t)EL * S;
  const uint8_t *drow[NBW];
  int soff[NBW];
#pragma unroll
  for (int b = 0; b < NBW; ++b) {
    const int wv = NBW * wave + b;
    drow[b] = dl + (size_t)(32 * wv + c) * S + 16 * h;
    // this lane reduces elements 16 d + 8 h .. + 7 of its block for the two
    // planes of its prime (stage rows c - d and c - d + 1)
    soff[b] = (c - d) * EL + 32 * wv + 16 * d + 8 * h;
  }
  const int nrt = (m + 15) / 16, nks = kd / 32;
  const int8_t *wbase = P.tab.wd + (int64_t)c * kd + 16 * h;
  v4i fnext[4];
  if (act) frag_load4(fnext, wbase, 0, nks);
  // reduction constants of this lane's prime, loaded a tile ahead
  int jn = min(c >> 1, m - 1);
  uint32_t pn = (uint32_t)P.tab.prime[jn], mun = P.tab.mu[jn], kpn = P.tab.kp[jn];
  // with the residue sums: this thread's items of a tile's store (prime
  // rp of the tile, word wd of its plane rows: 4 elements) and the
  // addend's words for them, requested at the tile's start
  constexpr int NIT = SUM ? (4 * EL + 255) / 256 : 1;
  uint32_t ya[NIT][2], yp[NIT];
  auto item = [&](int i, int rt_, int &rp, int &wd, int &j) {
    const int t = tid + 256 * i;
    rp = t / (EL / 4);
    wd = t - rp * (EL / 4);
    j = 16 * rt_ + rp;
    return t < 4 * EL && j < m && g0 + 4 * wd < total;
  };
  for (int rt = 0; rt < nrt; ++rt) {
    if constexpr (SUM) {
#pragma unroll
      for (int i = 0; i < NIT; ++i) {
        int rp, wd, j;
        if (item(i, rt, rp, wd, j)) {
          const int64_t olo = (int64_t)(2 * j) * total + g0 + 4 * wd;
          ya[i][0] = *reinterpret_cast<const uint32_t *>(P.addend + olo);
          ya[i][1] = *reinterpret_cast<const uint32_t *>(P.addend + olo + total);
          yp[i] = (uint32_t)P.tab.prime[j];
        }
      }
    }
    if (act) {
      const int8_t *wrow = wbase + (int64_t)rt * 32 * kd;
      const uint32_t pj = pn, muj = mun, kpj = kpn;
      const int j = 16 * rt + (c >> 1);
      if (rt + 1 < nrt) {
        jn = min(j + 16, m - 1);
        pn = (uint32_t)P.tab.prime[jn];
        mun = P.tab.mu[jn];
        kpn = P.tab.kp[jn];
      }
      v16i acc[NBW];
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[b][r] = 0;
      auto products = [&](const v4i (&fa)[4], int k0) {
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
          v4i fb[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int ks = k0 + u < nks ? k0 + u : k0;
            fb[u] = *reinterpret_cast<const v4i *>(drow[b] + 32 * ks);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (k0 + u < nks) acc[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fb[u], fa[u], acc[b], 0, 0, 0);
        }
      };
      // the tile's next NPRE runs of four weight fragments are requested
      // together, then the next tile's first run, which loads during this
      // tile's products and residue arithmetic
      v4i fx[NPRE][4];
#pragma unroll
      for (int q = 0; q < NPRE; ++q)
        if (4 * (q + 1) < nks) frag_load4(fx[q], wrow, 4 * (q + 1), nks);
      v4i fa0[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) fa0[u] = fnext[u];
      frag_load4(fnext, rt + 1 < nrt ? wrow + 32 * kd : wbase, 0, nks);
      products(fa0, 0);
#pragma unroll
      for (int q = 0; q < NPRE; ++q)
        if (4 * (q + 1) < nks) products(fx[q], 4 * (q + 1));
      for (int k0 = 4 * (NPRE + 1); k0 < nks; k0 += 4) {
        v4i fa[4];
        frag_load4(fa, wrow, k0, nks);
        products(fa, k0);
      }
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        // lo + 256 hi per element from the lane pair (2u, 2u + 1): the even
        // lane reduces registers 8 g + i (elements 8 h + 4 g + i), the odd
        // lane registers 8 g + 4 + i (elements 16 + 8 h + 4 g + i); each
        // forms both candidates with one DPP exchange each and keeps its own
        uint32_t w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int re = 8 * (k >> 2) + (k & 3), ro = re + 4;
          const int32_t te = __builtin_amdgcn_mov_dpp(acc[b][re], 0xB1, 0xF, 0xF, false);
          const int32_t to = __builtin_amdgcn_mov_dpp(acc[b][ro], 0xB1, 0xF, 0xF, false);
          const int32_t se = acc[b][re] + (te << 8), so = to + (acc[b][ro] << 8);
          w[k] = residue_digits(pj, muj, kpj, d ? so : se);
        }
        // bytes (lo, hi) of the 8 consecutive elements into the stage rows
        // of the prime's two planes
        uint32_t lo[2], hi[2];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          const uint32_t x01 = __builtin_amdgcn_perm(w[4 * g + 1], w[4 * g], 0x05010400u);
          const uint32_t x23 = __builtin_amdgcn_perm(w[4 * g + 3], w[4 * g + 2], 0x05010400u);
          lo[g] = __builtin_amdgcn_perm(x23, x01, 0x05040100u);
          hi[g] = __builtin_amdgcn_perm(x23, x01, 0x07060302u);
        }
        *reinterpret_cast<uint2 *>(stage + soff[b]) = make_uint2(lo[0], lo[1]);
        *reinterpret_cast<uint2 *>(stage + soff[b] + EL) = make_uint2(hi[0], hi[1]);
      }
    }
    __syncthreads();
    if constexpr (!SUM) {
      // the tile's planes 32 rt .. 32 rt + 31 (those of real primes), one
      // word of a plane row per thread
      for (int t = tid; t < 32 * (EL / 4); t += 256) {
        const int r = t / (EL / 4), wd = t - r * (EL / 4);
        const int plane = 32 * rt + r;
        if (plane < 2 * m && g0 + 4 * wd < total)
          *reinterpret_cast<uint32_t *>(P.planes + (int64_t)plane * total + g0 + 4 * wd) =
              *reinterpret_cast<const uint32_t *>(stage + r * EL + 4 * wd);
      }
    } else {
      // the same per prime (its two planes' words for 4 elements), and the
      // residues of the sum with the addend's into the sum planes
#pragma unroll
      for (int i = 0; i < NIT; ++i) {
        int rp, wd, j;
        if (item(i, rt, rp, wd, j)) {
          const int64_t olo = (int64_t)(2 * j) * total + g0 + 4 * wd, ohi = olo + total;
          const uint32_t xl = *reinterpret_cast<const uint32_t *>(stage + 2 * rp * EL + 4 * wd);
          const uint32_t xh = *reinterpret_cast<const uint32_t *>(stage + (2 * rp + 1) * EL + 4 * wd);
          *reinterpret_cast<uint32_t *>(P.planes + olo) = xl;
          *reinterpret_cast<uint32_t *>(P.planes + ohi) = xh;
          uint32_t lo4, hi4;
          residue_sum4(xl, xh, ya[i][0], ya[i][1], (int32_t)yp[i], lo4, hi4);
          *reinterpret_cast<uint32_t *>(P.sum + olo) = lo4;
          *reinterpret_cast<uint32_t *>(P.sum + ohi) = hi4;
        }
      }
    }
    __syncthreads();
  }
}

// Explicit Chinese remainder formula per entry:
//   T = sum_j y_j (P / p_j) - k P,  y_j = r_j (P / p_j)^-1 mod p_j (balanced),
// with k the integer nearest to alpha = sum_j y_j / p_j (|T| < P / 4, so
// alpha lies within 1/4 of an integer and its double-precision value
// rounds to the right k).  The sum is an integer matrix product: the int8
// digits (lo, hi) of every y_j and of -k against the balanced base-256
// digits of P / p_j, 256 P / p_j, P and 256 P, on INT8 MFMA.
//
// Workgroup: 256 threads, EW entries.  Phase 1: 256 / EW threads per entry
// compute the y_j digits from the three partial planes of each prime into
// an LDS row of kc bytes (+16 so that 8 consecutive rows fall in distinct
// 16-byte bank groups), and k.  Phase 2: the waves split the blocks of 32
// entries and (for a single block, or for both blocks together when the
// limb count is large) their chunks of 32 digit columns (8 limbs) into
// runs of consecutive chunks: one 32 x 32 MFMA result per
// chunk, whose lane l holds limbs 4 (l / 32) .. +3 of entry l % 32 as four
// groups of 4 digit sums; the limbs are formed in 64-bit with the carry
// passed from the lower lane half to the upper and on along the run, and
// kept in LDS with the run's signed carry out.  Phase 3: every entry adds
// the runs' carries in limb order and is rounded.
template <int EW, bool PAIR>
__global__ __launch_bounds__(256) void rns_crt_kernel(RnsCrtParams P) {
  extern __shared__ __attribute__((aligned(16))) uint8_t ylds[];   // [EW][kc + 16], then T
  uint32_t *tl = reinterpret_cast<uint32_t *>(ylds + (size_t)EW * (P.tab.kc + 16));   // [W][EW]
  int32_t *cyl = reinterpret_cast<int32_t *>(tl + (size_t)P.W * EW);                  // [ncc][EW], with runs
  // phase 1's partial sums of alpha share the limbs' space: the limbs are
  // written only after the last read of the partials (and the host sizes
  // that space to hold at least 256 doubles)
  double *apart = reinterpret_cast<double *>(tl);
  constexpr int TPE = 256 / EW;
  const int tid = threadIdx.x;
  const int m = P.tab.m, kc = P.tab.kc, S = kc + 16, W = P.W;
  const int64_t MN = P.M * P.N;
  const int64_t e0 = (int64_t)blockIdx.x * EW;

  // phase 1: balanced y_j = lo + 256 hi as bytes 2j, 2j + 1 of the row
  {
    const int e = tid % EW;
    // part is the same across a wave when EW >= 64: per-prime constants
    // then come by scalar loads
    const int part = EW >= 64 ? __builtin_amdgcn_readfirstlane(tid / EW) : tid / EW;
    const int64_t ij = e0 + e;
    const bool live = ij < MN;
    double alpha = 0.0;
    // lanes past the end read entry 0 (in bounds) and contribute nothing
    const int64_t ij0 = live ? ij : 0;
    // the source planes' signs as masks (x ^ s) - s, s = 0 or -1
    int32_t sm[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) sm[c] = P.sgn[c] < 0 ? -1 : 0;
    for (int g = part; g < kc / 16; g += TPE) {
      // the residue reads of 8 primes (up to 3 products each) are issued
      // before any use, each from a uniform base plus the entry's offset
      // (planes past prime m - 1 repeat its plane and are not used)
      int32_t dv[8][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int16_t *yp = P.Y + ((int64_t)P.src[c < P.nsrc ? c : 0] * m + min(8 * g, m - 1)) * P.ds + ij0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          dv[u][c] = c < P.nsrc ? (int32_t)*yp : 0;
          if (8 * g + u + 1 < m) yp += P.ds;
        }
      }
      uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = 8 * g + u;
        if (j < m) {
          const auto *crp = cp(P.tab.crt) + j;
          struct { uint32_t p, mu; int32_t cb; uint32_t kp2; double rp; uint32_t half; } cr = {
              crp->p, crp->mu, crp->cb, crp->kp2, crp->rp, crp->half};
          // y = (sum of at most three residues in [-p, p)) times cb mod p:
          // |sum cb| < 1.5 p^2 < 1.5 2^30 (24-bit signed factors, so the
          // 24-bit product is exact), and 2 kp (a multiple of p in [2^31,
          // 2^31 + 2p)) keeps the value nonnegative and below 2^32, so one
          // reduction suffices; its quotient q < 2^18 and p < 2^15 again
          // multiply exactly in 24 bits
          int32_t rs = 0;
#pragma unroll
          for (int c = 0; c < 3; ++c) rs += (dv[u][c] ^ sm[c]) - sm[c];
          const uint32_t x = (uint32_t)__mul24(rs, cr.cb) + cr.kp2;
          const uint32_t q = __umulhi(x, cr.mu);
          uint32_t y = x - __umul24(q, cr.p);
          y = y >= cr.p ? y - cr.p : y;
          int32_t yb = y > cr.half ? (int32_t)y - (int32_t)cr.p : (int32_t)y;
          yb = live ? yb : 0;
          alpha += (double)yb * cr.rp;
          const int32_t lo = ((yb + 128) & 255) - 128;
          const int32_t hi = (yb - lo) >> 8;
          w[u >> 1] |= (((uint32_t)lo & 0xFFu) | (((uint32_t)hi & 0xFFu) << 8)) << (16 * (u & 1));
        }
      }
      *reinterpret_cast<uint4 *>(ylds + (size_t)e * S + 16 * g) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    apart[tid] = alpha;
    __syncthreads();
    if (part == 0) {
      double a = 0.0;
#pragma unroll
      for (int t = 0; t < TPE; ++t) a += apart[e + t * EW];
      const int32_t nk = live ? -__double2int_rn(a) : 0;   // |k| <= m / 2 + 1
      const int32_t lo = ((nk + 128) & 255) - 128;
      ylds[(size_t)e * S + 2 * m] = (uint8_t)lo;
      ylds[(size_t)e * S + 2 * m + 1] = (uint8_t)((nk - lo) >> 8);
    }
    __syncthreads();
  }

  // phase 2: digit sums on MFMA; each wave walks a run of consecutive limb
  // chunks of one or two entry blocks, passing the carries along the run,
  // and stores each chunk's 8 limbs and, at the end of its run, the signed
  // carry out (zero for the other chunks)
  {
    const int lane = tid & 63, wave = tid >> 6, h = lane >> 5;
    // entry blocks; runs per block: with 64 entries two runs of chunks per
    // block, one wave each (phase 3 adds the runs' carries), unless PAIR:
    // then each wave takes a quarter of the chunks of both blocks,
    // and every weight fragment feeds the products of both (for long
    // limb counts, where those fragments' traffic dominates); with 32
    // entries the four waves share the one block
    constexpr int NB = EW / 32, RB = (EW == 32 || PAIR) ? 4 : 2, NBW = PAIR ? 2 : 1;
    const int ncc = P.tab.ncc, rl = (ncc + RB - 1) / RB, nks = kc / 32;
    const int wv0 = PAIR ? 0 : wave % NB, run = PAIR ? wave : wave / NB;
    const int c0 = run * rl, c1 = min(c0 + rl, ncc);
    const uint8_t *yrow[NBW];
    int el[NBW];
    int64_t carry[NBW];
#pragma unroll
    for (int b = 0; b < NBW; ++b) {
      el[b] = 32 * (wv0 + b) + (lane & 31);
      yrow[b] = ylds + (size_t)el[b] * S + 16 * h;
      carry[b] = 0;
    }
    for (int cc = c0; cc < c1; ++cc) {
      const int8_t *qrow = P.tab.qd + ((int64_t)cc * 32 + (lane & 31)) * kc + 16 * h;
      v16i acc[NBW];
#pragma unroll
      for (int b = 0; b < NBW; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[b][r] = 0;
      for (int k0 = 0; k0 < nks; k0 += 4) {
        v4i fa[4];
        frag_load4(fa, qrow, k0, nks);
#pragma unroll
        for (int b = 0; b < NBW; ++b) {
          v4i fb[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int ks = k0 + u < nks ? k0 + u : k0;
            fb[u] = *reinterpret_cast<const v4i *>(yrow[b] + 32 * ks);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (k0 + u < nks) acc[b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[u], fb[u], acc[b], 0, 0, 0);
        }
      }
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        int64_t L[4];
#pragma unroll
        for (int g = 0; g < 4; ++g)
          L[g] = (int64_t)acc[b][4 * g] + ((int64_t)acc[b][4 * g + 1] << 8) + ((int64_t)acc[b][4 * g + 2] << 16) +
                 ((int64_t)acc[b][4 * g + 3] << 24);
        // lower half first (carry in from the previous chunk of the run),
        // then the upper half with the lower half's carry out; the carry
        // out of a run is below 2^22 in magnitude (every column sum is
        // below kc 2^14 < 2^25)
        uint32_t limb[4];
        int64_t v = h ? 0 : carry[b];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          v += L[g];
          limb[g] = (uint32_t)v;
          v >>= 32;
        }
        const int64_t vl = __shfl(v, lane & 31);
        if (h) {
          v = vl;
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            v += L[g];
            limb[g] = (uint32_t)v;
            v >>= 32;
          }
        }
        carry[b] = __shfl(v, (lane & 31) + 32);
        if (RB > 1 && h) cyl[cc * EW + el[b]] = cc + 1 == c1 ? (int32_t)carry[b] : 0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int q = 8 * cc + 4 * h + g;
          if (q < W) tl[q * EW + el[b]] = limb[g];
        }
      }
    }
  }
  __syncthreads();

  // phase 3: rounding of the entry to the output
  if constexpr (!PAIR) {
    if (tid < EW) {
      const int64_t ij = e0 + tid;
      if (ij >= MN) return;
      uint32_t *T = tl + tid;
      // the runs' carries, added in limb order (a chunk's 8 limbs are read
      // together; a chunk changes only where a carry reaches it)
      int64_t c = 0;
      for (int cc = 0; cc < P.tab.ncc; ++cc) {
        const int32_t co = cyl[cc * EW + tid];
        if (c != 0) {
          uint32_t t[8];
#pragma unroll
          for (int g = 0; g < 8; ++g) t[g] = 8 * cc + g < W ? T[(8 * cc + g) * EW] : 0u;
#pragma unroll
          for (int g = 0; g < 8; ++g) {
            const int64_t v = (int64_t)t[g] + c;
            if (8 * cc + g < W) T[(8 * cc + g) * EW] = (uint32_t)v;
            c = v >> 32;
          }
        }
        c += co;
      }
      if (P.t_out)
        for (int q = 0; q < W; ++q) P.t_out[(int64_t)q * P.t_ld + ij] = T[q * EW];
      if (!P.C.exp) return;   // the exact T only
      const int64_t i = ij / P.N, jj = ij - i * P.N;
      double m0 = 0.0;
      int e0r = 0;
      if (P.rin_m) { m0 = P.rin_m[ij]; e0r = P.rin_e[ij]; }
      finish_entry([&](int q) { return T[q * EW]; }, W, (int64_t)P.rowv2[i] + P.colv2[jj], P.C,
                   P.c_off + i * P.c_rs + jj * P.c_cs, P.p, P.approx, m0, e0r);
    }
  } else {
    // long T (from 8 limb chunks on): the runs' carries by one thread per
    // entry, then the rounding by all the entry's threads, its limb scans
    // split over them (the digit rows' LDS is free now)
    constexpr int G = 256 / EW;
    const int e3 = tid % EW, part3 = tid / EW;
    const int64_t ij = e0 + e3;
    const bool live = ij < MN;
    uint32_t *T = tl + e3;
    if (part3 == 0 && live) {
      // a chunk changes only where a carry reaches it (after a run's end,
      // until the carry is absorbed)
      int64_t c = 0;
      for (int cc = 0; cc < P.tab.ncc; ++cc) {
        const int32_t co = cyl[cc * EW + e3];
        if (c != 0) {
          uint32_t t[8];
#pragma unroll
          for (int g = 0; g < 8; ++g) t[g] = 8 * cc + g < W ? T[(8 * cc + g) * EW] : 0u;
#pragma unroll
          for (int g = 0; g < 8; ++g) {
            const int64_t v = (int64_t)t[g] + c;
            if (8 * cc + g < W) T[(8 * cc + g) * EW] = (uint32_t)v;
            c = v >> 32;
          }
        }
        c += co;
      }
    }
    __syncthreads();
    if (P.t_out && live)
      for (int q = part3; q < W; q += G) P.t_out[(int64_t)q * P.t_ld + ij] = T[q * EW];
    if (!P.C.exp) return;   // the exact T only (the same for every thread)
    int64_t scale = 0, oidx = 0;
    double m0 = 0.0;
    int e0r = 0;
    if (live) {
      const int64_t i = ij / P.N, jj = ij - i * P.N;
      scale = (int64_t)P.rowv2[i] + P.colv2[jj];
      oidx = P.c_off + i * P.c_rs + jj * P.c_cs;
      if (P.rin_m) { m0 = P.rin_m[ij]; e0r = P.rin_e[ij]; }
    }
    finish_entry_split<EW, G>(T, W, scale, P.C, oidx, P.p, P.approx, m0, e0r, live, e3, part3,
                              reinterpret_cast<int32_t *>(ylds));
  }
}

hipError_t launch_rns_slice(const RnsSliceParams &P, hipStream_t s) {
  const int64_t total = P.lines_pad * P.k_pad;
  if (total == 0) return hipSuccess;
  const size_t S = (size_t)P.tab.kd + 16;
  if (32 * (S + 32) > 65536 || 4 * P.tab.nw > P.tab.kd) return hipErrorInvalidValue;
  // whole blocks of 32 elements, 16-byte aligned plane rows
  if ((total & 31) != 0 || ((uintptr_t)P.planes & 15) != 0) return hipErrorInvalidValue;
  if (P.sum && (!P.addend || (((uintptr_t)P.addend | (uintptr_t)P.sum) & 15) != 0)) return hipErrorInvalidValue;
  // digit rows and a tile's staged planes (32 x el bytes)
  // (with the residue sums at most 128 elements: their addend words take
  // the registers of a second block per wave)
  int el = P.sum ? 128 : 256;
  while (el > 32 && (size_t)el * (S + 32) > 65536) el >>= 1;
  const dim3 grid((unsigned)((total + el - 1) / el));
  const size_t lds = (size_t)el * (S + 32);
  auto go = [&](auto sum) {
    constexpr bool SUM = decltype(sum)::value;
    if (el == 256) {
      if constexpr (!SUM) hipLaunchKernelGGL((rns_slice_kernel<256, false>), grid, dim3(256), lds, s, P);
    } else if (el == 128) hipLaunchKernelGGL((rns_slice_kernel<128, SUM>), grid, dim3(256), lds, s, P);
    else if (el == 64) hipLaunchKernelGGL((rns_slice_kernel<64, SUM>), grid, dim3(256), lds, s, P);
    else hipLaunchKernelGGL((rns_slice_kernel<32, SUM>), grid, dim3(256), lds, s, P);
  };
  if (P.sum) go(std::true_type{});
  else go(std::false_type{});
  return hipGetLastError();
}

size_t rns_crt_lds(int ew, int kc, int W) { return rns_crt_lds(ew, kc, W, ew == 32); }

size_t rns_crt_lds(int ew, int kc, int W, bool runs) {
  const size_t rows = (size_t)ew * ((size_t)kc + 16);
  const size_t rest = (size_t)ew * (4 * (size_t)W + (runs ? 4 * (size_t)((W + 7) / 8) : 0));
  return rows + std::max<size_t>(rest, 256 * sizeof(double));
}

hipError_t launch_rns_crt(const RnsCrtParams &P, hipStream_t s) {
  const int64_t MN = P.M * P.N;
  if (MN == 0) return hipSuccess;
  if (rns_crt_lds(32, P.tab.kc, P.W) > kRnsCrtLds || P.tab.ncc * 8 < P.W || P.tab.ncc != (P.W + 7) / 8)
    return hipErrorInvalidValue;
  // 64 entries per workgroup (four threads per entry in phase 1) measured
  // faster than 128 and than fewer threads.  From 8 limb chunks on, the
  // waves pair the two 32-entry blocks (up to 80 KiB of LDS; with 9 chunks
  // 1.49 -> 1.38 ms at 1024^2 complex p = 1024, with 5 slower, 1.12 ->
  // 1.25 ms at 2048^2 p = 512); below, two waves walk a block each (up to
  // 64 KiB); else 32 entries, also when the launch would leave compute
  // units idle
  const bool many = (MN + 63) / 64 >= 1024;
  const int kc = P.tab.kc, W = P.W;
  if (many && P.tab.ncc >= 8 && rns_crt_lds(64, kc, W, true) <= 81920) {
    hipLaunchKernelGGL((rns_crt_kernel<64, true>), dim3((unsigned)((MN + 63) / 64)), dim3(256),
                       rns_crt_lds(64, kc, W, true), s, P);
  } else if (many && rns_crt_lds(64, kc, W, true) <= 65536) {
    hipLaunchKernelGGL((rns_crt_kernel<64, false>), dim3((unsigned)((MN + 63) / 64)), dim3(256),
                       rns_crt_lds(64, kc, W, true), s, P);
  } else {
    hipLaunchKernelGGL((rns_crt_kernel<32, false>), dim3((unsigned)((MN + 31) / 32)), dim3(256),
                       rns_crt_lds(32, kc, W, true), s, P);
  }
  return hipGetLastError();
}

}  // namespace arbgpu_impl
