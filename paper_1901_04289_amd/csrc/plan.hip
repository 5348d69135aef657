// Greedy block extraction of Algorithm 2 (Johansson 2019, Section 4.1):
// starting at the lowest unused inner index, append indices in increasing
// order while every row of A_s and every column of B_s keeps integer height
// (highest exponent minus lowest set bit over its nonzero entries) at most
// h; a block shorter than the basecase length is extended to
// min(basecase, remaining) indices and evaluated with dot products.
//
// One workgroup walks the inner indices; each candidate index is tested
// against all rows and columns in parallel and then committed.
#include "sliced.hpp"
#include "engine.hpp"

using namespace arb;

namespace arbgpu_impl {

namespace {

__device__ __forceinline__ const arbgpu_arr &part_at(const arbgpu_arr *p, int i) { return i ? p[1] : p[0]; }

// (top exponent, lowest set bit) of one element over its parts; top =
// INT_MIN when every part is zero
__device__ __forceinline__ void elem_top_low(const arbgpu_arr *parts, int nparts, int64_t idx, int &top, int &low) {
  top = -0x7FFFFFFF - 1;
  low = 0x7FFFFFFF;
  for (int q = 0; q < nparts; ++q) {
    const arbgpu_arr &A = part_at(parts, q);
    int n = A.nls[idx] & 0x7FFFFFFF;
    if (n > A.cap) n = A.cap;
    if (n == 0) continue;
    const int e = A.exp[idx];
    int lb = 0x7FFFFFFF;
    for (int k = n - 1; k >= 0; --k) {
      const uint32_t v = A.limbs[(int64_t)k * A.ld + idx];
      if (v) { lb = e - 32 * (k + 1) + __builtin_ctz(v); break; }
    }
    if (lb == 0x7FFFFFFF) continue;
    top = e > top ? e : top;
    low = lb < low ? lb : low;
  }
}

constexpr int kPlanThreads = 1024;

__device__ int block_max(int v, int *red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const int o = __shfl_xor(v, m, 64);
    v = o > v ? o : v;
  }
  if (lane == 0) red[w] = v;
  __syncthreads();
  int r = red[0];
  for (int i = 1; i < kPlanThreads / 64; ++i) r = red[i] > r ? red[i] : r;
  __syncthreads();
  return r;
}

}  // namespace

__global__ __launch_bounds__(kPlanThreads) void plan_blocks_kernel(PlanParams P) {
  __shared__ int red[kPlanThreads / 64];
  const int tid = threadIdx.x;
  int64_t start = 0;
  int nb = 0;
  while (start < P.inner) {
    for (int64_t i = tid; i < P.M; i += kPlanThreads) { P.rtop[i] = -0x7FFFFFFF - 1; P.rlow[i] = 0x7FFFFFFF; }
    for (int64_t j = tid; j < P.N; j += kPlanThreads) { P.ctop[j] = -0x7FFFFFFF - 1; P.clow[j] = 0x7FFFFFFF; }
    __syncthreads();
    int64_t end = start;
    while (end < P.inner) {
      // heights with index `end` added
      int h = 0;
      for (int64_t i = tid; i < P.M; i += kPlanThreads) {
        int t, l;
        elem_top_low(P.A, P.nparts, P.a_off + i * P.a_rs + end * P.a_cs, t, l);
        if (t == -0x7FFFFFFF - 1) continue;
        const int nt = t > P.rtop[i] ? t : P.rtop[i];
        const int nl = l < P.rlow[i] ? l : P.rlow[i];
        h = (nt - nl) > h ? (nt - nl) : h;
      }
      for (int64_t j = tid; j < P.N; j += kPlanThreads) {
        int t, l;
        elem_top_low(P.B, P.nparts, P.b_off + end * P.b_rs + j * P.b_cs, t, l);
        if (t == -0x7FFFFFFF - 1) continue;
        const int nt = t > P.ctop[j] ? t : P.ctop[j];
        const int nl = l < P.clow[j] ? l : P.clow[j];
        h = (nt - nl) > h ? (nt - nl) : h;
      }
      const int H = block_max(h, red);
      if (H > P.hmax) break;
      for (int64_t i = tid; i < P.M; i += kPlanThreads) {
        int t, l;
        elem_top_low(P.A, P.nparts, P.a_off + i * P.a_rs + end * P.a_cs, t, l);
        if (t == -0x7FFFFFFF - 1) continue;
        if (t > P.rtop[i]) P.rtop[i] = t;
        if (l < P.rlow[i]) P.rlow[i] = l;
      }
      for (int64_t j = tid; j < P.N; j += kPlanThreads) {
        int t, l;
        elem_top_low(P.B, P.nparts, P.b_off + end * P.b_rs + j * P.b_cs, t, l);
        if (t == -0x7FFFFFFF - 1) continue;
        if (t > P.ctop[j]) P.ctop[j] = t;
        if (l < P.clow[j]) P.clow[j] = l;
      }
      __syncthreads();
      ++end;
    }
    int kind = 0;
    if (end - start < P.basecase) {
      end = start + (P.inner - start < P.basecase ? P.inner - start : P.basecase);
      kind = 1;
    }
    if (tid == 0 && nb < P.max_blocks) {
      P.bounds[2 * nb] = start;
      P.bounds[2 * nb + 1] = end;
      P.kinds[nb] = kind;
    }
    ++nb;
    start = end;
    __syncthreads();
  }
  if (tid == 0) *P.nblocks = nb;
}

hipError_t launch_plan(const PlanParams &P, hipStream_t s) {
  hipLaunchKernelGGL(plan_blocks_kernel, dim3(1), dim3(kPlanThreads), 0, s, P);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
