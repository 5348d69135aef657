// Greedy block extraction of Algorithm 2 (Johansson 2019, Section 4.1):
// starting at the lowest unused inner index, append indices in increasing
// order while every row of A_s and every column of B_s keeps integer height
// (highest exponent minus lowest set bit over its nonzero entries) at most
// h; a block shorter than the basecase length is extended to
// min(basecase, remaining) indices and evaluated with dot products.
//
// A parallel pass takes every element's top exponent and lowest set bit;
// then one workgroup walks the blocks, each line scanning forward from the
// block's start for the index that would lift its height above h.
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
constexpr int kNone = -0x7FFFFFFF - 1;

}  // namespace

// (top, lowest set bit) of every element of A and B over the inner range,
// one thread per element; the faster-varying index follows the smaller
// stride so that the limb reads coalesce.
__global__ __launch_bounds__(256) void plan_elements_kernel(PlanParams P) {
  const int64_t na = P.M * P.inner, nb = P.N * P.inner;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int top, low;
  if (t < na) {
    const bool k_fast = (P.a_cs < 0 ? -P.a_cs : P.a_cs) <= (P.a_rs < 0 ? -P.a_rs : P.a_rs);
    const int64_t i = k_fast ? t / P.inner : t % P.M, k = k_fast ? t % P.inner : t / P.M;
    elem_top_low(P.A, P.nparts, P.a_off + i * P.a_rs + k * P.a_cs, top, low);
    P.hlA[k * P.M + i] = make_int2(top, low);
  } else if (t < na + nb) {
    const int64_t u = t - na;
    const bool k_fast = (P.b_rs < 0 ? -P.b_rs : P.b_rs) <= (P.b_cs < 0 ? -P.b_cs : P.b_cs);
    const int64_t j = k_fast ? u / P.inner : u % P.N, k = k_fast ? u % P.inner : u / P.N;
    elem_top_low(P.B, P.nparts, P.b_off + k * P.b_rs + j * P.b_cs, top, low);
    P.hlB[k * P.N + j] = make_int2(top, low);
  }
}

// The greedy walk: from `start`, every line (row of A or column of B)
// finds the first inner index whose addition lifts its height above hmax;
// the block ends at the smallest of these (heights only grow as indices
// are added, so this is where the index-by-index greedy stops).  Lines
// stop scanning once they pass the smallest end found so far.
__global__ __launch_bounds__(kPlanThreads) void plan_walk_kernel(PlanParams P) {
  __shared__ int64_t end_min;
  const int tid = threadIdx.x;
  const int64_t lines = P.M + P.N;
  int64_t start = 0;
  int nb = 0;
  while (start < P.inner) {
    if (tid == 0) end_min = P.inner;
    __syncthreads();
    for (int64_t L = tid; L < lines; L += kPlanThreads) {
      const bool row = L < P.M;
      const int2 *hl = row ? P.hlA + L : P.hlB + (L - P.M);
      const int64_t stride = row ? P.M : P.N;
      int top = kNone, low = 0x7FFFFFFF;
      int64_t e = start, stop = -1;
      // eight indices per round, their loads issued together
      while (stop < 0 && e < *(volatile int64_t *)&end_min) {
        const int64_t lim = *(volatile int64_t *)&end_min;
        int2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = e + u < lim ? hl[(e + u) * stride] : make_int2(kNone, 0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (stop >= 0 || e + u >= lim || v[u].x == kNone) continue;
          top = v[u].x > top ? v[u].x : top;
          low = v[u].y < low ? v[u].y : low;
          if (top - low > P.hmax) stop = e + u;
        }
        e += 8;
      }
      if (stop >= 0 && stop < *(volatile int64_t *)&end_min)
        atomicMin((unsigned long long *)&end_min, (unsigned long long)stop);
    }
    __syncthreads();
    int64_t end = end_min;
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

// Line statistics of every block of the partition, one thread per (block,
// line): top exponent and lowest set bit over the block's range, and the
// block's largest row and column heights (atomic maxima into gA[0] and
// gB[0], which the host clears before the launch).
__global__ __launch_bounds__(256) void block_stats_kernel(BlockStatsParams P) {
  const int64_t lines = P.M + P.N;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t b = t / lines, L = t - b * lines;
  int h = 0;
  bool row = true;
  int32_t *st = nullptr;
  if (b < *P.nblocks && b < P.max_blocks) {
    const int64_t k0 = P.bounds[2 * b], k1 = P.bounds[2 * b + 1];
    row = L < P.M;
    const int2 *hl = row ? P.hlA + L : P.hlB + (L - P.M);
    const int64_t stride = row ? P.M : P.N;
    int top = kNone, low = 0x7FFFFFFF;
    for (int64_t k = k0; k < k1; k += 8) {   // eight loads in flight
      int2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = k + u < k1 ? hl[(k + u) * stride] : make_int2(kNone, 0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (v[u].x == kNone) continue;
        top = v[u].x > top ? v[u].x : top;
        low = v[u].y < low ? v[u].y : low;
      }
    }
    st = P.out + b * P.stride;
    if (row) {
      st[L] = top;
      st[P.M + L] = low;
    } else {
      st[2 * P.M + (L - P.M)] = top;
      st[2 * P.M + P.N + (L - P.M)] = low;
    }
    if (low != 0x7FFFFFFF) h = top - low;
  }
  if (st && h > 0) atomicMax(&st[2 * P.M + 2 * P.N + (row ? 0 : 4)], h);
}

hipError_t launch_block_stats(const BlockStatsParams &P, hipStream_t s) {
  const int64_t n = P.max_blocks * (P.M + P.N);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(block_stats_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_plan(const PlanParams &P, hipStream_t s) {
  const int64_t n = (P.M + P.N) * P.inner;
  if (n > 0)
    hipLaunchKernelGGL(plan_elements_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P);
  hipLaunchKernelGGL(plan_walk_kernel, dim3(1), dim3(kPlanThreads), 0, s, P);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
