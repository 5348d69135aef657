// Scaled-integer block product on INT8 MFMA (Algorithm 2 of Johansson 2019,
// Section 4.1; FLINT's integer product replaced by an exact sliced product).
//
// For a block of inner indices, row i of A is scaled by 2^-v2_i and column
// j of B by 2^-v2_j (the lowest set bit over the line, Section 4.1) so that
// both become integer matrices X, Y.  Each integer is written in balanced
// base 256, x = sum_a d_a 256^a with d_a in [-128, 127], as L int8 digit
// planes.  Then
//     T = X Y = sum_c 256^c D_c,   D_c = sum_{a+b=c} X_a Y_b,
// where every X_a Y_b is an int8 GEMM with int32 accumulation.  A diagonal
// group of at most P pairs keeps |D| < P K 2^14 < 2^31, so the int32 planes
// are exact.  The recombination streams the diagonals from c = 0 upward with
// one int64 carry per entry and emits the bytes of T, which is exact; the
// entry C_ij = T_ij 2^(v2_i + v2_j) is then truncated to p bits once.
//
// Radii (Section 4.1, last paragraph): |A| R_B + R_A (|B| + R_B) in FP64
// with upward rounding, each row and column scaled into the double range.
//
// This unit holds the line statistics, the base-256 slicer, the carry
// recombination and the radius frames; the INT8 MFMA product is in
// mfma.hip, the FP64 radius product in radius.hip, the residue form in
// rns.hip.
#include <math.h>

#include "engine.hpp"
#include "sliced.hpp"
#include "finish.hpp"
#include "elements.hpp"

using namespace arb;

namespace arbgpu_impl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// statistics: top exponent and lowest set bit per line
// ---------------------------------------------------------------------------

__device__ __forceinline__ void stats_elem(const StatsParams &P, int64_t line, int64_t k, int &top, int &v2,
                                          int &prec, int &bad, int &amax) {
  for (int q = 0; q < P.nparts; ++q) {
    const arbgpu_arr &A = part_of(P.part, q);
    const int64_t idx = P.off + line * P.line_stride + (P.k0 + k) * P.elem_stride;
    const int n = elem_n(A, idx);
    if (n == 0) continue;
    const int e = A.exp[idx];
    if (e >= kExpLimit || e <= -kExpLimit) { bad = 1; continue; }
    const int lb = low_bit(A, idx, n, e);
    if (lb == 0x7FFFFFFF) continue;
    top = e > top ? e : top;
    v2 = lb < v2 ? lb : v2;
    prec = (e - lb) > prec ? (e - lb) : prec;
    const int ae = e < 0 ? -e : e, al = lb < 0 ? -lb : lb;
    amax = ae > amax ? ae : amax;
    amax = al > amax ? al : amax;
  }
}

// Atomic max / min that first reads the stored value and skips the atomic
// when it cannot change it (the stored value only moves one way, so a
// stale read costs at most a needless atomic): most partial results of a
// line or of the whole product lose, and atomics on one address serialize.
__device__ __forceinline__ void max_into(int32_t *p, int v) {
  if (v > *reinterpret_cast<volatile int32_t *>(p)) atomicMax(p, v);
}
__device__ __forceinline__ void min_into(int32_t *p, int v) {
  if (v < *reinterpret_cast<volatile int32_t *>(p)) atomicMin(p, v);
}

// Rows: one wave per (row, chunk of row_chunk inner indices), lanes along
// the inner index (coalesced for row-major A); partial results merge with
// atomics.  Chunks keep enough waves in flight to hide the dependent
// count, exponent and low-limb loads of each element.
constexpr int kRowChunk = 256;
constexpr int kColChunk = 16;

// Inner indices per wave of the row (column) kernels: kRowChunk
// (kColChunk), halved while the product is too small to give about 2048
// waves, down to one index per lane (per wave).
__host__ __device__ inline int64_t row_chunk(int64_t lines, int64_t lt) {
  int64_t c = kRowChunk;
  while (c > 64 && lines * ((lt + c - 1) / c) < 2048) c >>= 1;
  return c;
}
__host__ __device__ inline int64_t col_chunk(int64_t lines, int64_t lt) {
  const int64_t tiles = (lines + 63) / 64;
  int64_t c = kColChunk;
  while (c > 1 && tiles * ((lt + c - 1) / c) < 2048) c >>= 1;
  return c;
}
__global__ __launch_bounds__(256) void stats_rows_kernel(StatsParams P) {
  const int64_t ch = row_chunk(P.lines, P.len), nch = (P.len + ch - 1) / ch;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t line = w / nch, k0 = (w - line * nch) * ch;
  const int lane = threadIdx.x & 63;
  if (line >= P.lines) return;
  const int64_t k1 = k0 + ch < P.len ? k0 + ch : P.len;
  int top = -0x7FFFFFFF - 1, v2 = 0x7FFFFFFF, prec = 0, bad = 0, amax = 0;
  for (int64_t k = k0 + lane; k < k1; k += 64) stats_elem(P, line, k, top, v2, prec, bad, amax);
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    int t = __shfl_xor(top, m, 64); top = t > top ? t : top;
    int v = __shfl_xor(v2, m, 64); v2 = v < v2 ? v : v2;
    int q = __shfl_xor(prec, m, 64); prec = q > prec ? q : prec;
    bad |= __shfl_xor(bad, m, 64);
    int a = __shfl_xor(amax, m, 64); amax = a > amax ? a : amax;
  }
  if (lane == 0) {
    if (top != -0x7FFFFFFF - 1) max_into(&P.out.top[line], top);
    if (v2 != 0x7FFFFFFF) min_into(&P.out.v2[line], v2);
    if (prec) max_into(&P.gmax[1], prec);
    if (bad) max_into(&P.gmax[2], 1);
    if (amax) max_into(&P.gmax[3], amax);
  }
}

// Columns: lane = column (coalesced for row-major B), one wave per chunk of
// col_chunk inner indices; partial results merge with atomics.
__global__ __launch_bounds__(256) void stats_cols_kernel(StatsParams P) {
  const int64_t nct = (P.lines + 63) >> 6;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t ct = w % nct, kc = w / nct;
  const int64_t line = ct * 64 + (threadIdx.x & 63);
  const int64_t ch = col_chunk(P.lines, P.len), k0 = kc * ch;
  if (k0 >= P.len) return;   // uniform across the wave
  const int64_t k1 = k0 + ch < P.len ? k0 + ch : P.len;
  int top = -0x7FFFFFFF - 1, v2 = 0x7FFFFFFF, prec = 0, bad = 0, amax = 0;
  if (line < P.lines) {
    for (int64_t k = k0; k < k1; ++k) stats_elem(P, line, k, top, v2, prec, bad, amax);
    if (top != -0x7FFFFFFF - 1) max_into(&P.out.top[line], top);
    if (v2 != 0x7FFFFFFF) min_into(&P.out.v2[line], v2);
  }
  // the whole-product maxima: one atomic (at most) per wave
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    int q = __shfl_xor(prec, m, 64); prec = q > prec ? q : prec;
    bad |= __shfl_xor(bad, m, 64);
    int a = __shfl_xor(amax, m, 64); amax = a > amax ? a : amax;
  }
  if ((threadIdx.x & 63) == 0) {
    if (prec) max_into(&P.gmax[1], prec);
    if (bad) max_into(&P.gmax[2], 1);
    if (amax) max_into(&P.gmax[3], amax);
  }
}

__global__ __launch_bounds__(256) void stats_init_kernel(LineStats S, int64_t lines) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < lines) {
    S.top[i] = -0x7FFFFFFF - 1;
    S.v2[i] = 0x7FFFFFFF;
  }
}

// Largest integer height top - v2 over nonzero lines.
__global__ __launch_bounds__(256) void stats_height_kernel(LineStats S, int64_t lines, int32_t *gmax) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int h = 0;
  if (i < lines && S.v2[i] != 0x7FFFFFFF) h = S.top[i] - S.v2[i];
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    int o = __shfl_xor(h, m, 64);
    h = o > h ? o : h;
  }
  if ((threadIdx.x & 63) == 0 && h > 0) atomicMax(&gmax[0], h);
}

// ---------------------------------------------------------------------------
// slicing into balanced base-256 digit planes
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void slice_kernel(SliceParams P) {
  const int64_t kq = P.k_pad >> 2;
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= P.lines_pad * kq) return;
  const int64_t line = gid / kq;
  const int64_t q = gid - line * kq;
  const int64_t len_total = (P.mode == 0) ? P.len : 2 * P.len;
  const int L = P.L;
  const int nw = (L + 3) >> 2;
  // per-element state
  int64_t idx[4];
  int part[4], n[4];
  int64_t s[4];
  uint32_t sg[4];
  uint32_t cy[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t k = 4 * q + t;
    n[t] = 0; s[t] = 0; sg[t] = 0; cy[t] = 0; idx[t] = 0; part[t] = 0;
    if (line < P.lines && k < len_total) {
      int64_t kk;
      uint32_t ng;
      inner_map(P.mode, P.len, k, part[t], kk, ng);
      const arbgpu_arr &A = part_of(P.part, part[t]);
      idx[t] = P.off + line * P.line_stride + (P.k0 + kk) * P.elem_stride;
      const int nn = elem_n(A, idx[t]);
      if (nn) {
        const int32_t nl = A.nls[idx[t]];
        n[t] = nn;
        sg[t] = ((uint32_t)nl >> 31) ^ ng;
        s[t] = (int64_t)A.exp[idx[t]] - 32 * (int64_t)nn - P.v2[line];
      }
    }
  }
  const int64_t plane = P.lines_pad * P.k_pad;
  uint32_t *base = reinterpret_cast<uint32_t *>(P.planes + line * P.k_pad + 4 * q);
  for (int w = 0; w < nw; ++w) {
    // offset B = sum_{a<L} 128 * 256^a, restricted to this 32-bit chunk
    const int nbytes = (L - 4 * w) >= 4 ? 4 : (L - 4 * w);
    const uint32_t bmask = nbytes == 4 ? 0xFFFFFFFFu : ((1u << (8 * nbytes)) - 1u);
    const uint32_t Bc = 0x80808080u & bmask;
    uint32_t y[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      uint32_t x = 0;
      if (n[t]) x = mant_chunk(part_of(P.part, part[t]), idx[t], n[t], 32 * (int64_t)w - s[t]);
      uint64_t v;
      if (!sg[t]) {
        v = (uint64_t)Bc + x + cy[t];
        cy[t] = (uint32_t)(v >> 32);
      } else {
        v = (uint64_t)Bc - x - cy[t];
        cy[t] = (uint32_t)((v >> 63) & 1u);
      }
      y[t] = ((uint32_t)v) ^ 0x80808080u;   // byte u - 128 as int8 is u ^ 0x80
    }
    // transpose 4 elements x 4 digits into 4 plane words
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int a = 4 * w + b;
      if (a < L) {
        const uint32_t word = ((y[0] >> (8 * b)) & 0xFFu) | (((y[1] >> (8 * b)) & 0xFFu) << 8) |
                              (((y[2] >> (8 * b)) & 0xFFu) << 16) | (((y[3] >> (8 * b)) & 0xFFu) << 24);
        base[(a * plane) >> 2] = word;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// carry recombination and truncation to p bits
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void recombine_kernel(RecombParams P) {
  const int64_t MN = P.M * P.N;
  const int64_t ij = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (ij >= MN) return;
  const int64_t i = ij / P.N, j = ij - i * P.N;
  uint32_t *T = P.T + ij;
  const int nq = (P.Lc + 3) >> 2;
  int64_t carry = 0;
  for (int w = 0; w < nq; ++w) {
    uint32_t limb = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = 4 * w + b;
      if (c < P.Lc) {
        int64_t s = 0;
        for (int sl = P.slot_of[c]; sl < P.slot_of[c + 1]; ++sl) s += P.D[(int64_t)sl * P.ds + ij];
        carry += s;
      }
      limb |= ((uint32_t)carry & 0xFFu) << (8 * b);
      carry >>= 8;
    }
    T[(int64_t)w * MN] = limb;
  }
  T[(int64_t)nq * MN] = (uint32_t)carry;
  T[(int64_t)(nq + 1) * MN] = (uint32_t)((uint64_t)carry >> 32);
  const int nT = nq + 2;
  if (!P.C.exp) return;   // the exact T only
  if (P.ebits >= 0 && !certify_truncation([&](int q) { return T[(int64_t)q * MN]; }, nT, P.p, P.ebits)) {
    P.fb_list[atomicAdd(P.fb_count, 1)] = ij;   // recomputed exactly by the limb kernel
    return;
  }

  double m0 = 0.0;
  int e0 = 0;
  if (P.rin_m) { m0 = P.rin_m[ij]; e0 = P.rin_e[ij]; }
  finish_entry([&](int q) { return T[(int64_t)q * MN]; }, nT, (int64_t)P.rowv2[i] + P.colv2[j], P.C,
               P.c_off + i * P.c_rs + j * P.c_cs, P.p, P.approx, m0, e0);
}

// ---------------------------------------------------------------------------
// radius matrices (FP64, rounded up, per-line exponent frames)
// ---------------------------------------------------------------------------

// Upper bound of |m| (mantissa in [0.5, 1]): the top 64 bits rounded up to
// 53 bits, with a sticky bit for the limbs below them.  The lowest limb is
// read first: when it is nonzero (operands of full precision) it settles
// the sticky bit without a pass over the middle limbs.
__device__ __forceinline__ double mag_upper_mem(const arbgpu_arr &A, int64_t idx, int n) {
  const uint32_t top = A.limbs[idx];
  const uint32_t second = n > 1 ? A.limbs[A.ld + idx] : 0u;
  uint32_t rest = n > 2 ? A.limbs[(int64_t)(n - 1) * A.ld + idx] : 0u;
  if (rest == 0)
    for (int q = 2; q < n - 1; ++q) rest |= A.limbs[(int64_t)q * A.ld + idx];
  const uint64_t v = ((uint64_t)top << 32) | second;
  const uint64_t m53 = (v >> 11) + (((v & 0x7FFull) != 0 || rest != 0) ? 1 : 0);
  return (double)m53 * 0x1p-53;
}

// x * 2^d (x >= 0, d <= 0) exactly, for the radius products.  Values that
// would land below 2^-480 raise the tiny flag instead (the products of two
// such values could leave the normal range) and read as 0: the exact
// per-entry kernel then recomputes every radius.
__device__ __forceinline__ double rad_scaled(double x, int d, int32_t *tiny) {
  if (x == 0.0) return 0.0;
  int ex;
  (void)frexp(x, &ex);
  if (ex + d < -480) {
    atomicOr(tiny, 1);
    return 0.0;
  }
  return ldexp(x, d);
}

// (|b| + r) * 2^-F rounded up: an r too small to matter at the precision of
// |b| bumps |b| by one ulp instead.
__device__ __forceinline__ double rad_scaled_sum(double m, int dm, double r, int dr, int32_t *tiny) {
  const double ms = rad_scaled(m, dm, tiny);
  if (r == 0.0) return ms;
  int ex;
  (void)frexp(r, &ex);
  if (ex + dr < -480 && ms >= 0x1p-420) return next_up(ms);   // r * 2^dr < ulp(ms)
  return ru_add(ms, rad_scaled(r, dr, tiny));
}

__device__ __forceinline__ void rad_elem(const arbgpu_arr &A, int64_t idx, double &m, int &e, double &r, int &re) {
  const int n = elem_n(A, idx);
  m = 0.0;
  e = 0;
  r = 0.0;
  re = 0;
  if (n) {
    m = mag_upper_mem(A, idx, n);
    e = A.exp[idx];
  }
  if (A.rad_m) {
    const double rr = A.rad_m[idx];
    if (rr != 0.0) {
      int ex;
      r = frexp(rr, &ex);
      re = A.rad_e[idx] + ex;
    }
  }
}

// Exponent frames per line, one for each value array (A side: |a| and
// r_a; B side: |b| + r_b, bounded by 2^(max(e, re) + 1), and r_b), then
// the values scaled into their frames (A side writes [line][k], B side
// [k][line]).  The frames are maxima over a line, merged from chunks with
// atomics into arrays preset to kNoFrame; lines without a value get frame
// 0 afterwards.
constexpr int kNoFrame = -0x7FFFFFFF - 1;

__device__ __forceinline__ void rad_frame_elem(const RadPrepParams &P, int64_t line, int64_t k, int &F0,
                                               int &F1) {
  int part;
  int64_t kk;
  uint32_t ng;
  inner_map(P.mode, P.len, k, part, kk, ng);
  const arbgpu_arr &A = part_of(P.part, part);
  const int64_t idx = P.off + line * P.line_stride + kk * P.elem_stride;
  int f0 = elem_n(A, idx) ? A.exp[idx] : kNoFrame;
  int f1 = kNoFrame;
  if (A.rad_m) {
    const double rr = A.rad_m[idx];
    if (rr != 0.0) {
      int ex;
      (void)frexp(rr, &ex);
      f1 = A.rad_e[idx] + ex;
    }
  }
  if (P.side == 1) {
    f0 = f1 > f0 ? f1 : f0;
    if (f0 != kNoFrame) f0 += 1;
  }
  F0 = f0 > F0 ? f0 : F0;
  F1 = f1 > F1 ? f1 : F1;
}

// A side: one wave per (line, chunk of row_chunk inner indices), lanes
// along the inner index.
__global__ __launch_bounds__(256) void rad_frames_rows_kernel(RadPrepParams P) {
  const int64_t lt = (P.mode == 0) ? P.len : 2 * P.len;
  const int64_t ch = row_chunk(P.lines, lt), nch = (lt + ch - 1) / ch;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t line = w / nch, k0 = (w - line * nch) * ch;
  const int lane = threadIdx.x & 63;
  if (line >= P.lines) return;
  const int64_t k1 = k0 + ch < lt ? k0 + ch : lt;
  int F0 = kNoFrame, F1 = kNoFrame;
  for (int64_t k = k0 + lane; k < k1; k += 64) rad_frame_elem(P, line, k, F0, F1);
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    int o = __shfl_xor(F0, m, 64);
    F0 = o > F0 ? o : F0;
    o = __shfl_xor(F1, m, 64);
    F1 = o > F1 ? o : F1;
  }
  if (lane == 0) {
    if (F0 != kNoFrame) max_into(&P.scale0[line], F0);
    if (F1 != kNoFrame) max_into(&P.scale1[line], F1);
  }
}

// B side: lane = line (consecutive in a row-major B), one wave per chunk of
// col_chunk inner indices.
__global__ __launch_bounds__(256) void rad_frames_cols_kernel(RadPrepParams P) {
  const int64_t lt = (P.mode == 0) ? P.len : 2 * P.len;
  const int64_t nct = (P.lines + 63) >> 6;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t ct = w % nct, kc = w / nct;
  const int64_t line = ct * 64 + (threadIdx.x & 63);
  const int64_t ch = col_chunk(P.lines, lt), k0 = kc * ch;
  if (line >= P.lines || k0 >= lt) return;
  const int64_t k1 = k0 + ch < lt ? k0 + ch : lt;
  int F0 = kNoFrame, F1 = kNoFrame;
  for (int64_t k = k0; k < k1; ++k) rad_frame_elem(P, line, k, F0, F1);
  if (F0 != kNoFrame) max_into(&P.scale0[line], F0);
  if (F1 != kNoFrame) max_into(&P.scale1[line], F1);
}

// One thread per value: consecutive threads along the inner index (A side)
// or along the lines (B side), the direction its output is contiguous in.
template <int SIDE>
__global__ __launch_bounds__(256) void rad_values_kernel(RadPrepParams P) {
  const int64_t lt = (P.mode == 0) ? P.len : 2 * P.len;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= P.lines * lt) return;
  int64_t line, k;
  if (SIDE == 0) {
    line = t / lt;
    k = t - line * lt;
  } else {
    k = t / P.lines;
    line = t - k * P.lines;
  }
  int F0 = P.scale0[line], F1 = P.scale1[line];
  F0 = F0 == kNoFrame ? 0 : F0;
  F1 = F1 == kNoFrame ? 0 : F1;
  int part;
  int64_t kk;
  uint32_t ng;
  inner_map(P.mode, P.len, k, part, kk, ng);
  const arbgpu_arr &A = part_of(P.part, part);
  double m, r;
  int e, re;
  rad_elem(A, P.off + line * P.line_stride + kk * P.elem_stride, m, e, r, re);
  // t is the output index: [line][k] on the A side, [k][line] on the B side
  P.v0[t] = (SIDE == 0) ? rad_scaled(m, e - F0, P.tiny) : rad_scaled_sum(m, e - F0, r, re - F0, P.tiny);
  P.v1[t] = rad_scaled(r, re - F1, P.tiny);
}

__global__ __launch_bounds__(256) void rad_frames_finish_kernel(RadPrepParams P) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= P.lines) return;
  if (P.scale0[i] == kNoFrame) P.scale0[i] = 0;
  if (P.scale1[i] == kNoFrame) P.scale1[i] = 0;
}

// Radius of one entry with its own frame (the largest term bound), as in
// the limb kernel: used when the per-line frames could not hold a value.
__global__ __launch_bounds__(256) void rad_exact_kernel(RadExactParams P) {
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= P.M || j >= P.N || !*P.tiny) return;
  constexpr int kNone = -0x7FFFFFFF - 1;
  int F = kNone;
  for (int pass = 0; pass < 2; ++pass) {
    double acc = 0.0;
    for (int64_t k = 0; k < P.Kt; ++k) {
      int pa, pb;
      int64_t ka, kb;
      uint32_t ng;
      inner_map(P.a_mode, P.len, k, pa, ka, ng);
      inner_map(P.b_mode, P.len, k, pb, kb, ng);
      double am, ar, bm, br;
      int ae, are, be, bre;
      rad_elem(part_of(P.A, pa), P.a_off + i * P.a_rs + ka * P.a_cs, am, ae, ar, are);
      rad_elem(part_of(P.B, pb), P.b_off + kb * P.b_rs + j * P.b_cs, bm, be, br, bre);
      if (pass == 0) {
        if (am != 0.0 && br != 0.0) F = ae + bre > F ? ae + bre : F;
        if (ar != 0.0 && bm != 0.0) F = are + be > F ? are + be : F;
        if (ar != 0.0 && br != 0.0) F = are + bre > F ? are + bre : F;
      } else {
        if (am != 0.0 && br != 0.0) acc = ru_add(acc, ru_scale_down(ru_mul(am, br), ae + bre - F));
        if (ar != 0.0 && bm != 0.0) acc = ru_add(acc, ru_scale_down(ru_mul(ar, bm), are + be - F));
        if (ar != 0.0 && br != 0.0) acc = ru_add(acc, ru_scale_down(ru_mul(ar, br), are + bre - F));
      }
    }
    if (pass == 0 && F == kNone) break;
    if (pass == 1) {
      double m = 0.0;
      int e = 0;
      if (acc != 0.0) {
        int ex;
        m = frexp(acc, &ex);
        e = F + ex;
      }
      P.out_m[i * P.N + j] = m;
      P.out_e[i * P.N + j] = e;
      return;
    }
  }
  P.out_m[i * P.N + j] = 0.0;
  P.out_e[i * P.N + j] = 0;
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline unsigned nblk(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_stats_rows(const StatsParams &P, hipStream_t s) {
  if (P.lines == 0) return hipSuccess;
  hipLaunchKernelGGL(stats_init_kernel, dim3(nblk(P.lines, 256)), dim3(256), 0, s, P.out, P.lines);
  if (P.len > 0) {
    const int64_t ch = row_chunk(P.lines, P.len), waves = P.lines * ((P.len + ch - 1) / ch);
    hipLaunchKernelGGL(stats_rows_kernel, dim3(nblk(waves, 4)), dim3(256), 0, s, P);
  }
  hipLaunchKernelGGL(stats_height_kernel, dim3(nblk(P.lines, 256)), dim3(256), 0, s, P.out, P.lines, P.gmax);
  return hipGetLastError();
}
hipError_t launch_stats_cols(const StatsParams &P, hipStream_t s) {
  if (P.lines == 0) return hipSuccess;
  hipLaunchKernelGGL(stats_init_kernel, dim3(nblk(P.lines, 256)), dim3(256), 0, s, P.out, P.lines);
  if (P.len > 0) {
    const int64_t ch = col_chunk(P.lines, P.len), waves = ((P.lines + 63) / 64) * ((P.len + ch - 1) / ch);
    hipLaunchKernelGGL(stats_cols_kernel, dim3(nblk(waves, 4)), dim3(256), 0, s, P);
  }
  hipLaunchKernelGGL(stats_height_kernel, dim3(nblk(P.lines, 256)), dim3(256), 0, s, P.out, P.lines, P.gmax);
  return hipGetLastError();
}
hipError_t launch_slice(const SliceParams &P, hipStream_t s) {
  const int64_t n = P.lines_pad * (P.k_pad >> 2);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(slice_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_recombine(const RecombParams &P, hipStream_t s) {
  const int64_t n = P.M * P.N;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(recombine_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, P);
  return hipGetLastError();
}
__global__ __launch_bounds__(256) void t_copy_kernel(const uint32_t *src, int n, int64_t mn, uint32_t *dst,
                                                     int64_t ld, int cap) {
  const int64_t ij = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (ij >= mn) return;
  uint32_t top = 0u;
  for (int k = 0; k < cap; ++k) {
    const uint32_t v = k < n ? src[(int64_t)k * mn + ij] : (uint32_t)((int32_t)top >> 31);
    dst[(int64_t)k * ld + ij] = v;
    top = v;
  }
}
__global__ __launch_bounds__(256) void v2_out_kernel(const int32_t *v2, int64_t n, int32_t *out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = v2[i] == INT32_MAX ? 0 : v2[i];
}
hipError_t launch_v2_out(const int32_t *v2, int64_t n, int32_t *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(v2_out_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, v2, n, out);
  return hipGetLastError();
}
hipError_t launch_t_copy(const uint32_t *src, int n, int64_t mn, uint32_t *dst, int64_t ld, int cap, hipStream_t s) {
  if (mn == 0 || cap == 0) return hipSuccess;
  hipLaunchKernelGGL(t_copy_kernel, dim3(nblk(mn, 256)), dim3(256), 0, s, src, n, mn, dst, ld, cap);
  return hipGetLastError();
}
hipError_t launch_rad_prep(const RadPrepParams &P, hipStream_t s) {
  if (P.lines == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(P.lines, 256)), dim3(256), 0, s, P.scale0, kNoFrame, P.lines);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(P.lines, 256)), dim3(256), 0, s, P.scale1, kNoFrame, P.lines);
  const int64_t lt = (P.mode == 0) ? P.len : 2 * P.len;
  if (lt > 0) {
    if (P.side == 0) {
      const int64_t ch = row_chunk(P.lines, lt), waves = P.lines * ((lt + ch - 1) / ch);
      hipLaunchKernelGGL(rad_frames_rows_kernel, dim3(nblk(waves, 4)), dim3(256), 0, s, P);
      hipLaunchKernelGGL(rad_values_kernel<0>, dim3(nblk(P.lines * lt, 256)), dim3(256), 0, s, P);
    } else {
      const int64_t ch = col_chunk(P.lines, lt), waves = ((P.lines + 63) / 64) * ((lt + ch - 1) / ch);
      hipLaunchKernelGGL(rad_frames_cols_kernel, dim3(nblk(waves, 4)), dim3(256), 0, s, P);
      hipLaunchKernelGGL(rad_values_kernel<1>, dim3(nblk(P.lines * lt, 256)), dim3(256), 0, s, P);
    }
  }
  hipLaunchKernelGGL(rad_frames_finish_kernel, dim3(nblk(P.lines, 256)), dim3(256), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_rad_exact(const RadExactParams &P, hipStream_t s) {
  if (P.M == 0 || P.N == 0) return hipSuccess;
  hipLaunchKernelGGL(rad_exact_kernel, dim3(nblk(P.N, 64), nblk(P.M, 4)), dim3(256), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
