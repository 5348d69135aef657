// Radius matrix products of the scaled-integer block product (Section 4.1,
// last paragraph): |A| R_B + R_A (|B| + R_B) on FP64 MFMA, the operands
// already scaled into per-line exponent frames.  Built with the matrix
// cores writing ordinary vector registers: with accumulation registers the
// loop-carried accumulators were copied to and from them at every chunk.
#include <math.h>

#include "engine.hpp"
#include "sliced.hpp"

using namespace arb;

namespace arbgpu_impl {

// rho_in(i, j) = sum_k a_m[i][k] b_r[k][j]    (frame 2^(a_s0[i] + b_s1[j]))
//              + sum_k a_r[i][k] b_mr[k][j]   (frame 2^(a_s1[i] + b_s0[j])),
// rounded up.  Skipped when a value was too small for its frame.
//
// The two sums run on FP64 MFMA in round-to-nearest and are then raised to
// upper bounds: every term is a nonnegative product of scaled values in
// [2^-481, 1] (or zero), so no subnormal arises, and each term passes
// through at most Kt + 1 roundings of relative error below 2^-52.  The
// computed sum s' therefore satisfies s <= s' (1 - 2^-52)^-(Kt+1) <=
// s' (1 + (Kt + 2) 2^-50), which is applied with upward rounding.  With
// the inner dimension split S ways (ranges of at least 64, S <= Kt / 64),
// a term meets at most ceil(Kt / S) + 1 roundings in its split and S - 1
// in the sum of the splits' partials, fewer than Kt + 1, so the same
// factor holds; the partials are added in split order, so the result does
// not depend on scheduling.
//
// Workgroup: 256 threads, 64 x 64 output tile, inner chunks of 16 staged
// in LDS k-major ([16][64] for every operand, so the 16 rows or columns of
// a fragment are consecutive doubles); the next chunk's values are loaded
// into registers while the current chunk's products run.  Wave w computes
// the 32 x 32 quarter (w / 2, w % 2) as 2 x 2 blocks of
// v_mfma_f64_16x16x4_f64 per sum: operand lane l holds row (column) l % 16
// at inner index l / 16; result lane l, register r holds row l / 16 + 4 r,
// column l % 16.
typedef double v4d __attribute__((ext_vector_type(4)));

// Upper bound of entry (i, j) from its two round-to-nearest sums.
__device__ __forceinline__ void rad_gemm_store(const RadGemmParams &P, int64_t i, int64_t j, double s1, double s2) {
  const double infl = 1.0 + ldexp((double)(P.Kt + 2), -50);
  double m1 = 0.0, m2 = 0.0;
  int e1 = 0, e2 = 0, ex;
  if (s1 != 0.0) { m1 = frexp(ru_mul(s1, infl), &ex); e1 = P.a_s0[i] + P.b_s1[j] + ex; }
  if (s2 != 0.0) { m2 = frexp(ru_mul(s2, infl), &ex); e2 = P.a_s1[i] + P.b_s0[j] + ex; }
  double m = 0.0;
  int e = 0;
  if (m1 != 0.0 && m2 != 0.0) ru_add_ext(m1, e1, m2, e2, m, e);
  else if (m1 != 0.0) { m = m1; e = e1; }
  else if (m2 != 0.0) { m = m2; e = e2; }
  P.out_m[i * P.N + j] = m;
  P.out_e[i * P.N + j] = e;
}

__global__ __launch_bounds__(256) void rad_gemm_kernel(RadGemmParams P) {
  constexpr int T = 64, KC = 16;
  __shared__ double sa[2][KC][T], sb[2][KC][T];   // [a_m | a_r], [b_r | b_mr]
  if (*P.tiny) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * T, j0 = (int64_t)blockIdx.x * T;
  const int wm = wave >> 1, wn = wave & 1;
  v4d acc[2][2][2];   // [sum][row block][column block]
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[q][bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
  // staging: A rows (i0 + r, r = tid / 4) at inner offsets 4 (tid % 4) .. +3;
  // B inner row k0 + tid / 16 at columns 4 (tid % 16) .. +3
  const int ar = tid >> 2, ak = 4 * (tid & 3);
  const int bk = tid >> 4, bc = 4 * (tid & 15);
  const int64_t ai = i0 + ar;
  // this split's inner range [kb, ke)
  const int64_t kb = (int64_t)blockIdx.z * P.kchunk;
  const int64_t ke = kb + P.kchunk < P.Kt ? kb + P.kchunk : P.Kt;
  double ra[2][4], rb[2][4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + ak + u;
      const bool ok = ai < P.M && k < ke;
      ra[0][u] = ok ? P.a_m[ai * P.Kt + k] : 0.0;
      ra[1][u] = ok ? P.a_r[ai * P.Kt + k] : 0.0;
    }
    const int64_t k = k0 + bk;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = j0 + bc + u;
      const bool ok = k < ke && j < P.N;
      rb[0][u] = ok ? P.b_r[k * P.N + j] : 0.0;
      rb[1][u] = ok ? P.b_mr[k * P.N + j] : 0.0;
    }
  };
  load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sa[0][ak + u][ar] = ra[0][u];
      sa[1][ak + u][ar] = ra[1][u];
      sb[0][bk][bc + u] = rb[0][u];
      sb[1][bk][bc + u] = rb[1][u];
    }
    __syncthreads();
    if (k0 + KC < ke) load(k0 + KC);
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        double fa[2], fb[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) fa[bi] = sa[q][kk][wm * 32 + bi * 16 + (lane & 15)];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) fb[bj] = sb[q][kk][wn * 32 + bj * 16 + (lane & 15)];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[q][bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[bi], fb[bj], acc[q][bi][bj], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int64_t MN = P.M * P.N;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wm * 32 + bi * 16 + (lane >> 4) + 4 * r;
        const int64_t j = j0 + wn * 32 + bj * 16 + (lane & 15);
        if (i >= P.M || j >= P.N) continue;
        if (P.splits > 1) {
          P.part[(2 * (int64_t)blockIdx.z) * MN + i * P.N + j] = acc[0][bi][bj][r];
          P.part[(2 * (int64_t)blockIdx.z + 1) * MN + i * P.N + j] = acc[1][bi][bj][r];
        } else {
          rad_gemm_store(P, i, j, acc[0][bi][bj][r], acc[1][bi][bj][r]);
        }
      }
}

// Sums of the splits' partials in split order, then the upper bound.
__global__ __launch_bounds__(256) void rad_gemm_finish_kernel(RadGemmParams P) {
  const int64_t MN = P.M * P.N;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (*P.tiny || t >= MN) return;
  double s1 = 0.0, s2 = 0.0;
  for (int z = 0; z < P.splits; ++z) {
    s1 += P.part[(2 * (int64_t)z) * MN + t];
    s2 += P.part[(2 * (int64_t)z + 1) * MN + t];
  }
  const int64_t i = t / P.N;
  rad_gemm_store(P, i, t - i * P.N, s1, s2);
}

int rad_gemm_splits(int64_t M, int64_t N, int64_t Kt) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int64_t sp = 1;
  while (sp < 16 && tiles * sp < 2048 && Kt / (2 * sp) >= 64) sp *= 2;
  return (int)sp;
}

hipError_t launch_rad_gemm(const RadGemmParams &P, hipStream_t s) {
  if (P.M == 0 || P.N == 0) return hipSuccess;
  if (P.splits < 1 || P.kchunk < 16 || P.kchunk % 16 != 0 || (int64_t)P.splits * P.kchunk < P.Kt ||
      (P.splits > 1 && !P.part))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((P.N + 63) / 64), (unsigned)((P.M + 63) / 64), (unsigned)P.splits);
  hipLaunchKernelGGL(rad_gemm_kernel, grid, dim3(256), 0, s, P);
  if (P.splits > 1)
    hipLaunchKernelGGL(rad_gemm_finish_kernel, dim3((unsigned)((P.M * P.N + 255) / 256)), dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
