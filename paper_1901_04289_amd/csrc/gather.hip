// Line-major copy of an operand whose inner index is strided (a row-major B
// read along its columns): element (line, k) of the block [k0, k0 + len)
// goes to index line * len + k, so the slicing kernels read consecutive
// inner indices from consecutive addresses.  Each workgroup transposes one
// 64 x 64 tile of one limb plane (or of the exponents or counts) through
// LDS; the planes are the third grid dimension, so that the tiles of all
// planes are in flight together.
#include "sliced.hpp"

namespace arbgpu_impl {

__global__ __launch_bounds__(256) void gather_lines_kernel(GatherParams P) {
  __shared__ uint32_t tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t k_base = (int64_t)blockIdx.x * 64, l_base = (int64_t)blockIdx.y * 64;
  const int q = blockIdx.z;   // limb plane, then exponents (cap), counts (cap + 1)
  // read: lanes along the line index (consecutive in the source)
  uint32_t v[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t k = k_base + ty + 4 * u, line = l_base + tx;
    v[u] = 0;
    if (k < P.len && line < P.lines) {
      const int64_t idx = P.off + line * P.line_stride + (P.k0 + k) * P.elem_stride;
      v[u] = q < P.src.cap ? P.src.limbs[(int64_t)q * P.src.ld + idx]
                           : (q == P.src.cap ? (uint32_t)P.src.exp[idx] : (uint32_t)P.src.nls[idx]);
    }
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) tile[ty + 4 * u][tx] = v[u];
  __syncthreads();
  // write: lanes along the inner index (consecutive in the copy)
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int64_t line = l_base + ty + 4 * u, k = k_base + tx;
    if (k < P.len && line < P.lines) {
      const int64_t o = line * P.len + k;
      const uint32_t w = tile[tx][ty + 4 * u];
      if (q < P.src.cap) P.limbs[(int64_t)q * P.lines * P.len + o] = w;
      else if (q == P.src.cap) P.exp[o] = (int32_t)w;
      else P.nls[o] = (int32_t)w;
    }
  }
}

hipError_t launch_gather(const GatherParams &P, hipStream_t s) {
  if (P.lines == 0 || P.len == 0) return hipSuccess;
  if (P.src.cap + 2 > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((P.len + 63) / 64), (unsigned)((P.lines + 63) / 64), (unsigned)(P.src.cap + 2));
  hipLaunchKernelGGL(gather_lines_kernel, grid, dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
