// Multimodular (residue number system) form of the scaled-integer block
// product.  The paper multiplies its integer matrices with FLINT, whose
// fast path works modulo word-size primes followed by Chinese remainder
// reconstruction (introduction of Section 4).  Here every scaled integer Y
// of a block is reduced modulo m odd primes p_j < 2^15, each residue
// (balanced, |r| < 2^14) is split into two int8 digits r = lo + 256 hi, and
// the digit products run on the INT8 MFMA kernel as three partial planes
// per prime (weights 1, 256, 65536).  The exact T is rebuilt per entry by
// the explicit Chinese remainder formula, exact whenever prod p_j > 4 |T|.
// The MFMA work is 4 m digit products instead of L_A L_B base-256 slices.
//
// The tables (primes, digit weights, quotients P / p_j) are the same for
// every thread and are read through the constant address space, so they
// arrive by scalar loads.
#include "elements.hpp"
#include "finish.hpp"
#include "sliced.hpp"

namespace arbgpu_impl {

namespace {

template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *cp(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

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

// Word w (4 balanced base-256 digits, int8 each) of Y: the digits of
// Y + B, B = sum_{a<L} 128 * 256^a, are bytes; those of Y are the bytes
// minus 128.  cy carries between words.
__device__ __forceinline__ uint32_t digit_word(const RnsSliceParams &P, const SliceElem &e, int w, uint32_t &cy) {
  const int nbytes = P.L - 4 * w;
  const uint32_t bmask = nbytes >= 4 ? 0xFFFFFFFFu : (nbytes <= 0 ? 0u : ((1u << (8 * nbytes)) - 1u));
  const uint32_t Bc = 0x80808080u & bmask;
  uint32_t x = 0;
  if (e.n) x = mant_chunk(part_of(P.part, e.part), e.idx, e.n, 32 * (int64_t)w - e.s);
  uint64_t v;
  if (!e.sg) {
    v = (uint64_t)Bc + x + cy;
    cy = (uint32_t)(v >> 32);
  } else {
    v = (uint64_t)Bc - x - cy;
    cy = (uint32_t)((v >> 63) & 1u);
  }
  return (((uint32_t)v) ^ 0x80808080u) & bmask;
}

// Residue of sum_a d_a 256^a modulo prime j from the two int8 dot-product
// sums, balanced and split into int8 digits (lo, hi).
__device__ __forceinline__ void store_residue(const RnsSliceParams &P, int j, int32_t slo, int32_t shi,
                                              int8_t *out, int64_t plane) {
  const uint32_t p = (uint32_t)cp(P.tab.prime)[j], mu = cp(P.tab.mu)[j];
  // S = 256 shi + slo, |S| < 2^31 for L <= 512
  uint32_t r = mod_s32(shi, p, mu);
  r = mod_u32((r << 8) + mod_s32(slo, p, mu), p, mu);
  const int32_t rb = r > (p >> 1) ? (int32_t)r - (int32_t)p : (int32_t)r;   // balanced, |rb| < 2^14
  const int32_t lo = ((rb + 128) & 255) - 128;
  const int32_t hi = (rb - lo) >> 8;
  out[(2 * j) * plane] = (int8_t)lo;
  out[(2 * j + 1) * plane] = (int8_t)hi;
}

}  // namespace

// One thread per element (line, k) of the padded plane: the balanced
// base-256 digits of the scaled integer, then for every prime the residue
// sum_a d_a (256^a mod p) by 4-way int8 dot products.  NW > 0: at most NW
// digit words, held in registers; NW = 0: any number, staged in LDS.
template <int NW>
__global__ __launch_bounds__(256) void rns_slice_kernel(RnsSliceParams P) {
  extern __shared__ uint32_t dig[];   // NW = 0: [nw][blockDim]
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * nt + tid;
  const int64_t total = P.lines_pad * P.k_pad;
  if (gid >= total) return;
  const int64_t line = gid / P.k_pad;
  const int64_t k = gid - line * P.k_pad;
  const SliceElem e = slice_elem(P, line, k);
  const int nw = P.tab.nw;
  int8_t *out = P.planes + line * P.k_pad + k;
  uint32_t cy = 0;
  if (NW > 0) {
    uint32_t d[NW > 0 ? NW : 1];
#pragma unroll
    for (int w = 0; w < NW; ++w) d[w] = w < nw ? digit_word(P, e, w, cy) : 0u;
    for (int j = 0; j < P.tab.m; ++j) {
      const __attribute__((address_space(4))) int32_t *wl = cp(P.tab.wlo) + (int64_t)j * nw;
      const __attribute__((address_space(4))) int32_t *wh = cp(P.tab.whi) + (int64_t)j * nw;
      int32_t slo = 0, shi = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        if (w < nw) {
          slo = __builtin_amdgcn_sdot4((int)d[w], wl[w], slo, false);
          shi = __builtin_amdgcn_sdot4((int)d[w], wh[w], shi, false);
        }
      }
      store_residue(P, j, slo, shi, out, total);
    }
  } else {
    for (int w = 0; w < nw; ++w) dig[w * nt + tid] = digit_word(P, e, w, cy);
    for (int j = 0; j < P.tab.m; ++j) {
      const __attribute__((address_space(4))) int32_t *wl = cp(P.tab.wlo) + (int64_t)j * nw;
      const __attribute__((address_space(4))) int32_t *wh = cp(P.tab.whi) + (int64_t)j * nw;
      int32_t slo = 0, shi = 0;
      for (int w = 0; w < nw; ++w) {
        const int dw = (int)dig[w * nt + tid];
        slo = __builtin_amdgcn_sdot4(dw, wl[w], slo, false);
        shi = __builtin_amdgcn_sdot4(dw, wh[w], shi, false);
      }
      store_residue(P, j, slo, shi, out, total);
    }
  }
}

namespace {

// Residue r_j = T mod p_j of entry ij from the three digit-product planes.
__device__ __forceinline__ uint32_t entry_residue(const RnsCrtParams &P, int j, int64_t ij, int64_t MN,
                                                  uint32_t p, uint32_t mu) {
  const uint32_t d0 = mod_s32(P.D[(int64_t)(3 * j) * MN + ij], p, mu);
  const uint32_t d1 = mod_s32(P.D[(int64_t)(3 * j + 1) * MN + ij], p, mu);
  const uint32_t d2 = mod_s32(P.D[(int64_t)(3 * j + 2) * MN + ij], p, mu);
  return mod_u32((mod_u32((d2 << 8) + d1, p, mu) << 8) + d0, p, mu);
}

}  // namespace

// One thread per output entry: the explicit Chinese remainder formula
//   T = sum_j y_j (P / p_j) - k P,  y_j = r_j (P / p_j)^-1 mod p_j,
// with k the integer nearest to alpha = sum_j y_j / p_j (|T| < P / 4, so
// alpha lies within 1/4 of an integer and its double-precision value
// rounds to the right k).  The products y_j (P / p_j)[q] add up in 64-bit
// carry-save columns.  WB > 0: the W <= 16 WB columns stay in registers;
// WB = 0: any W, in blocks of 16 limbs with the y_j staged in LDS.  T, in
// W two's-complement limbs (LDS), is then rounded to the output.
template <int WB>
__global__ __launch_bounds__(256) void rns_crt_kernel(RnsCrtParams P) {
  extern __shared__ uint32_t sh[];
  const int nt = blockDim.x, tid = threadIdx.x;
  const int m = P.tab.m, wq = P.tab.wq, W = P.W;
  uint32_t *T = sh + tid;                                      // T[q * nt]
  uint16_t *y = reinterpret_cast<uint16_t *>(sh + (size_t)W * nt) + tid;   // WB = 0: y[j * nt]
  const int64_t MN = P.M * P.N;
  const int64_t ij = (int64_t)blockIdx.x * nt + tid;
  if (ij >= MN) return;
  const __attribute__((address_space(4))) uint32_t *Qt = cp(P.tab.q);
  const __attribute__((address_space(4))) uint32_t *PP = cp(P.tab.pp);
  double alpha = 0.0;
  constexpr int NC = WB > 0 ? 16 * WB : 16;
  uint64_t col[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) col[u] = 0;
  for (int j = 0; j < m; ++j) {
    const uint32_t p = (uint32_t)cp(P.tab.prime)[j], mu = cp(P.tab.mu)[j];
    const uint32_t r = entry_residue(P, j, ij, MN, p, mu);
    const uint32_t yj = mod_u32(r * (uint32_t)cp(P.tab.c)[j], p, mu);
    alpha += (double)yj * cp(P.tab.rp)[j];
    if (WB > 0) {
      const __attribute__((address_space(4))) uint32_t *Q = Qt + (int64_t)j * wq;
#pragma unroll
      for (int u = 0; u < NC; ++u)
        if (u < wq) col[u] += (uint64_t)yj * Q[u];
    } else {
      y[j * nt] = (uint16_t)yj;
    }
  }
  const uint32_t kq = (uint32_t)__double2int_rn(alpha);   // 0 <= k <= m
  // S - k P in W limbs (two's complement modulo 2^(32 W))
  uint64_t carry = 0, kcarry = 0, borrow = 0;
  auto emit = [&](int q, uint64_t c) {
    const uint64_t sv = c + carry;   // < 2^58
    carry = sv >> 32;
    const uint64_t kp = (uint64_t)(q < wq ? PP[q] : 0u) * kq + kcarry;
    kcarry = kp >> 32;
    const uint64_t dv = (uint64_t)(uint32_t)sv - (uint32_t)kp - borrow;
    borrow = (dv >> 63) & 1u;
    T[q * nt] = (uint32_t)dv;
  };
  if (WB > 0) {
#pragma unroll
    for (int u = 0; u < NC; ++u)
      if (u < W) emit(u, col[u]);
  } else {
    for (int q0 = 0; q0 < W; q0 += 16) {
#pragma unroll
      for (int u = 0; u < 16; ++u) col[u] = 0;
      for (int j = 0; j < m; ++j) {
        const uint64_t yj = y[j * nt];
        const __attribute__((address_space(4))) uint32_t *Q = Qt + (int64_t)j * wq + q0;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (q0 + u < wq) col[u] += yj * Q[u];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (q0 + u < W) emit(q0 + u, col[u]);
    }
  }
  const int64_t i = ij / P.N, jj = ij - i * P.N;
  double m0 = 0.0;
  int e0 = 0;
  if (P.rin_m) { m0 = P.rin_m[ij]; e0 = P.rin_e[ij]; }
  finish_entry([&](int q) { return T[q * nt]; }, W, (int64_t)P.rowv2[i] + P.colv2[jj], P.C,
               P.c_off + i * P.c_rs + jj * P.c_cs, P.p, P.approx, m0, e0);
}

hipError_t launch_rns_slice(const RnsSliceParams &P, hipStream_t s) {
  const int64_t total = P.lines_pad * P.k_pad;
  if (total == 0) return hipSuccess;
  const int nw = P.tab.nw;
  const dim3 grid((unsigned)((total + 255) / 256));
#define ARB_SLICE(nwmax)                                                                  \
  if (nw <= nwmax) {                                                                      \
    hipLaunchKernelGGL(rns_slice_kernel<nwmax>, grid, dim3(256), 0, s, P);                \
    return hipGetLastError();                                                             \
  }
  ARB_SLICE(8) ARB_SLICE(16) ARB_SLICE(24) ARB_SLICE(32)
#undef ARB_SLICE
  const int nt = nw <= 64 ? 256 : 64;
  const size_t lds = sizeof(uint32_t) * nt * (size_t)nw;
  if (lds > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rns_slice_kernel<0>, dim3((unsigned)((total + nt - 1) / nt)), dim3(nt), lds, s, P);
  return hipGetLastError();
}

hipError_t launch_rns_crt(const RnsCrtParams &P, hipStream_t s) {
  const int64_t MN = P.M * P.N;
  if (MN == 0) return hipSuccess;
  const int W = P.W;
  auto blocks = [&](int nt) { return dim3((unsigned)((MN + nt - 1) / nt)); };
#define ARB_CRT(wb)                                                                       \
  if (W <= 16 * wb) {                                                                     \
    hipLaunchKernelGGL(rns_crt_kernel<wb>, blocks(256), dim3(256), 4 * (size_t)W * 256, s, P); \
    return hipGetLastError();                                                             \
  }
  ARB_CRT(1) ARB_CRT(2) ARB_CRT(3) ARB_CRT(4)
#undef ARB_CRT
  // per entry: W limbs and m 16-bit digits in LDS; at most 64 KiB a block
  const size_t per = 4 * (size_t)W + 2 * (size_t)P.tab.m;
  int nt = 256;
  while (nt > 32 && per * nt + 4 > 65536) nt >>= 1;
  const size_t lds = per * nt + 4;
  if (lds > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rns_crt_kernel<0>, blocks(nt), dim3(nt), lds, s, P);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
