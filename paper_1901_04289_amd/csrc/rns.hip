// Multimodular (residue number system) form of the scaled-integer block
// product.  The paper multiplies its integer matrices with FLINT, whose
// fast path works modulo word-size primes followed by Chinese remainder
// reconstruction (introduction of Section 4).  Here every scaled integer Y
// of a block is reduced modulo m odd primes p_j < 2^15, each residue
// (balanced, |r| < 2^14) is split into two int8 digits r = lo + 256 hi, and
// the digit products run on the INT8 MFMA kernel as three partial planes
// per prime (weights 1, 256, 65536).  The exact T is rebuilt per entry by
// Garner's mixed-radix conversion with balanced digits,
// T = v_0 + p_0 (v_1 + p_1 (v_2 + ...)), exact whenever prod p_j > 2 |T|.
// The MFMA work is 4 m digit products instead of L_A L_B base-256 slices.
#include "elements.hpp"
#include "finish.hpp"
#include "sliced.hpp"

namespace arbgpu_impl {

namespace {

// x mod p for 0 <= x < 2^32 (Barrett with mu = floor(2^32 / p)).
__device__ __forceinline__ uint32_t mod_u32(uint32_t x, uint32_t p, uint32_t mu) {
  const uint32_t q = __umulhi(x, mu);
  uint32_t r = x - q * p;
  r = r >= p ? r - p : r;
  r = r >= p ? r - p : r;
  return r;
}

// x mod p in [0, p) for signed x.
__device__ __forceinline__ uint32_t mod_s32(int32_t x, uint32_t p, uint32_t mu) {
  const uint32_t ax = x < 0 ? (uint32_t)0 - (uint32_t)x : (uint32_t)x;
  const uint32_t r = mod_u32(ax, p, mu);
  return (x < 0 && r) ? p - r : r;
}

}  // namespace

// One thread per element (line, k) of the padded plane: the balanced
// base-256 digits of the scaled integer (4 per word, staged in LDS), then
// for every prime the residue sum_a d_a (256^a mod p) by 4-way int8 dot
// products, reduced and split into two int8 digits.
template <bool STAGE>
__global__ __launch_bounds__(256) void rns_slice_kernel(RnsSliceParams P) {
  extern __shared__ uint32_t dig[];   // [nw][blockDim], then (if staged) the weights [2][m][nw]
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * nt + tid;
  const int nwm = P.tab.m * P.tab.nw;
  int32_t *wl_lds = reinterpret_cast<int32_t *>(dig + (size_t)P.tab.nw * nt);
  if (STAGE) {
    // the weights are read by every thread in the same order: one copy in LDS
    for (int u = tid; u < nwm; u += nt) {
      wl_lds[u] = P.tab.wlo[u];
      wl_lds[nwm + u] = P.tab.whi[u];
    }
    __syncthreads();
  }
  const int64_t total = P.lines_pad * P.k_pad;
  const int64_t line = gid / P.k_pad;
  const int64_t k = gid - line * P.k_pad;
  const int64_t len_total = (P.mode == 0) ? P.len : 2 * P.len;
  int n = 0, part = 0;
  int64_t idx = 0, s = 0;
  uint32_t sg = 0;
  if (gid < total && line < P.lines && k < len_total) {
    int64_t kk;
    uint32_t ng;
    inner_map(P.mode, P.len, k, part, kk, ng);
    const arbgpu_arr &A = part_of(P.part, part);
    idx = P.off + line * P.line_stride + (P.k0 + kk) * P.elem_stride;
    const int nn = elem_n(A, idx);
    if (nn) {
      n = nn;
      sg = ((uint32_t)A.nls[idx] >> 31) ^ ng;
      s = (int64_t)A.exp[idx] - 32 * (int64_t)nn - P.v2[line];
    }
  }
  const int nw = P.tab.nw;
  uint32_t cy = 0;
  for (int w = 0; w < nw; ++w) {
    // offset B = sum_{a<L} 128 * 256^a restricted to this word; the digits
    // of Y + B are bytes, those of Y the bytes minus 128
    const int nbytes = P.L - 4 * w;
    const uint32_t bmask = nbytes >= 4 ? 0xFFFFFFFFu : (nbytes <= 0 ? 0u : ((1u << (8 * nbytes)) - 1u));
    const uint32_t Bc = 0x80808080u & bmask;
    uint32_t x = 0;
    if (n) x = mant_chunk(part_of(P.part, part), idx, n, 32 * (int64_t)w - s);
    uint64_t v;
    if (!sg) {
      v = (uint64_t)Bc + x + cy;
      cy = (uint32_t)(v >> 32);
    } else {
      v = (uint64_t)Bc - x - cy;
      cy = (uint32_t)((v >> 63) & 1u);
    }
    dig[w * nt + tid] = (((uint32_t)v) ^ 0x80808080u) & bmask;
  }
  if (gid >= total) return;
  const int64_t plane = total;
  int8_t *out = P.planes + line * P.k_pad + k;
  for (int j = 0; j < P.tab.m; ++j) {
    int32_t slo = 0, shi = 0;
    if (STAGE) {
      const int32_t *wl = wl_lds + j * nw, *wh = wl_lds + nwm + j * nw;
      for (int w = 0; w < nw; ++w) {
        const int d = (int)dig[w * nt + tid];
        slo = __builtin_amdgcn_sdot4(d, wl[w], slo, false);
        shi = __builtin_amdgcn_sdot4(d, wh[w], shi, false);
      }
    } else {
      const int32_t *wl = P.tab.wlo + (int64_t)j * nw, *wh = P.tab.whi + (int64_t)j * nw;
      for (int w = 0; w < nw; ++w) {
        const int d = (int)dig[w * nt + tid];
        slo = __builtin_amdgcn_sdot4(d, wl[w], slo, false);
        shi = __builtin_amdgcn_sdot4(d, wh[w], shi, false);
      }
    }
    const uint32_t p = (uint32_t)P.tab.prime[j], mu = P.tab.mu[j];
    // S = 256 shi + slo, |S| < 2^31 for L <= 512
    uint32_t r = mod_s32(shi, p, mu);
    r = mod_u32((r << 8) + mod_s32(slo, p, mu), p, mu);
    const int32_t rb = r > (p >> 1) ? (int32_t)r - (int32_t)p : (int32_t)r;   // balanced, |rb| < 2^14
    const int32_t lo = ((rb + 128) & 255) - 128;
    const int32_t hi = (rb - lo) >> 8;
    out[(2 * j) * plane] = (int8_t)lo;
    out[(2 * j + 1) * plane] = (int8_t)hi;
  }
}

// One thread per output entry.  Residues r_j from the three digit-product
// planes of every prime; then the explicit Chinese remainder formula
//   T = sum_j y_j (P / p_j) - k P,  y_j = r_j (P / p_j)^-1 mod p_j,
// with k the integer nearest to alpha = sum_j y_j / p_j (|T| < P / 4, so
// alpha lies within 1/4 of an integer and its double-precision value
// rounds to the right k).  The sum runs in 64-bit carry-save columns over
// blocks of 16 limbs (the y_j staged in LDS); T, in W two's-complement
// limbs (LDS), is rounded to the output.
template <bool STAGE>
__global__ void rns_crt_kernel(RnsCrtParams P) {
  extern __shared__ uint32_t sh[];
  const int nt = blockDim.x, tid = threadIdx.x;
  const int m = P.tab.m, wq = P.tab.wq;
  uint16_t *y = reinterpret_cast<uint16_t *>(sh) + tid;          // y[j * nt]
  uint32_t *T = sh + ((m * nt + 1) >> 1) + tid;                  // T[q * nt]
  // staged copy of the limbs of P / p_j, [m][wq4] with wq4 = wq rounded to 4
  const int wq4 = (wq + 3) & ~3;
  uint32_t *qs = sh + ((m * nt + 1) >> 1) + (size_t)P.W * nt;
  if (STAGE) {
    for (int u = tid; u < m * wq4; u += nt) {
      const int j = u / wq4, q = u - j * wq4;
      qs[u] = q < wq ? P.tab.q[(int64_t)j * wq + q] : 0u;
    }
    __syncthreads();
  }
  const int64_t MN = P.M * P.N;
  const int64_t ij = (int64_t)blockIdx.x * nt + tid;
  if (ij >= MN) return;
  double alpha = 0.0;
  for (int k = 0; k < m; ++k) {
    const uint32_t p = (uint32_t)P.tab.prime[k], mu = P.tab.mu[k];
    const uint32_t d0 = mod_s32(P.D[(int64_t)(3 * k) * MN + ij], p, mu);
    const uint32_t d1 = mod_s32(P.D[(int64_t)(3 * k + 1) * MN + ij], p, mu);
    const uint32_t d2 = mod_s32(P.D[(int64_t)(3 * k + 2) * MN + ij], p, mu);
    const uint32_t r = mod_u32((mod_u32((d2 << 8) + d1, p, mu) << 8) + d0, p, mu);
    const uint32_t yk = mod_u32(r * (uint32_t)P.tab.c[k], p, mu);
    y[k * nt] = (uint16_t)yk;
    alpha += (double)yk * P.tab.rp[k];
  }
  const uint32_t kq = (uint32_t)__double2int_rn(alpha);   // 0 <= k <= m
  // S - k P in W limbs: columns accumulate y_j Q_j[q] (< m 2^47 < 2^64)
  const int W = P.W;
  uint64_t carry = 0;      // carry of S into the next block
  uint64_t borrow = 0;     // of the subtraction of k P (0 or 1)
  uint64_t kcarry = 0;     // carry of the product k P
  for (int q0 = 0; q0 < W; q0 += 16) {
    uint64_t col[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) col[u] = 0;
    if (STAGE) {
      for (int j = 0; j < m; ++j) {
        const uint64_t yj = y[j * nt];
        const uint32_t *Q = qs + j * wq4 + q0;
#pragma unroll
        for (int u = 0; u < 16; u += 4) {
          if (q0 + u < wq4) {
            const uint4 v = *reinterpret_cast<const uint4 *>(Q + u);
            col[u] += yj * v.x;
            col[u + 1] += yj * v.y;
            col[u + 2] += yj * v.z;
            col[u + 3] += yj * v.w;
          }
        }
      }
    } else {
      for (int j = 0; j < m; ++j) {
        const uint64_t yj = y[j * nt];
        const uint32_t *Q = P.tab.q + (int64_t)j * wq;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int q = q0 + u;
          if (q < wq) col[u] += yj * Q[q];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int q = q0 + u;
      if (q >= W) break;
      // limb q of S
      const uint64_t sv = col[u] + carry;
      const uint32_t s_limb = (uint32_t)sv;
      carry = (sv >> 32) + (sv < col[u] ? ((uint64_t)1 << 32) : 0);
      // limb q of k P
      const uint64_t kp = (uint64_t)(q < wq ? P.tab.pp[q] : 0u) * kq + kcarry;
      const uint32_t kp_limb = (uint32_t)kp;
      kcarry = kp >> 32;
      // limb q of S - k P (two's complement modulo 2^(32 W))
      const uint64_t dv = (uint64_t)s_limb - kp_limb - borrow;
      borrow = (dv >> 63) & 1u;
      T[q * nt] = (uint32_t)dv;
    }
  }
  const int64_t i = ij / P.N, j = ij - i * P.N;
  double m0 = 0.0;
  int e0 = 0;
  if (P.rin_m) { m0 = P.rin_m[ij]; e0 = P.rin_e[ij]; }
  finish_entry([&](int q) { return T[q * nt]; }, W, (int64_t)P.rowv2[i] + P.colv2[j], P.C,
               P.c_off + i * P.c_rs + j * P.c_cs, P.p, P.approx, m0, e0);
}

hipError_t launch_rns_slice(const RnsSliceParams &P, hipStream_t s) {
  const int64_t total = P.lines_pad * P.k_pad;
  if (total == 0) return hipSuccess;
  const int nt = P.tab.nw <= 64 ? 256 : 64;
  size_t lds = sizeof(uint32_t) * nt * (size_t)P.tab.nw;
  if (lds > 65536) return hipErrorInvalidValue;
  const size_t wbytes = 2 * sizeof(int32_t) * (size_t)P.tab.m * P.tab.nw;
  const dim3 grid((unsigned)((total + nt - 1) / nt));
  if (lds + wbytes <= 65536)
    hipLaunchKernelGGL(rns_slice_kernel<true>, grid, dim3(nt), lds + wbytes, s, P);
  else
    hipLaunchKernelGGL(rns_slice_kernel<false>, grid, dim3(nt), lds, s, P);
  return hipGetLastError();
}

hipError_t launch_rns_crt(const RnsCrtParams &P, hipStream_t s) {
  const int64_t MN = P.M * P.N;
  if (MN == 0) return hipSuccess;
  // per entry: m 16-bit digits and W limbs in LDS; at most 64 KiB a block
  const size_t per = 2 * (size_t)P.tab.m + 4 * (size_t)P.W;
  const size_t qbytes = 4 * (size_t)P.tab.m * ((P.tab.wq + 3) & ~3);
  int nt = 256;
  while (nt > 32 && per * nt + 4 + qbytes > 65536) nt >>= 1;
  if (per * nt + 4 + qbytes <= 65536 && nt >= 64) {
    hipLaunchKernelGGL(rns_crt_kernel<true>, dim3((unsigned)((MN + nt - 1) / nt)), dim3(nt), per * nt + 4 + qbytes,
                       s, P);
    return hipGetLastError();
  }
  nt = 256;
  while (nt > 32 && per * nt + 4 > 65536) nt >>= 1;
  const size_t lds = per * nt + 4;
  if (lds > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rns_crt_kernel<false>, dim3((unsigned)((MN + nt - 1) / nt)), dim3(nt), lds, s, P);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
