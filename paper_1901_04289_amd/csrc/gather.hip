// Line-major copy of an operand whose inner index is strided (a row-major B
// read along its columns): element (line, k) of the block [k0, k0 + len)
// goes to index line * len + k, so the slicing kernels read consecutive
// inner indices from consecutive addresses.  64 x 64 tiles are transposed
// through LDS, one limb plane (then exponents and counts) at a time.
#include "sliced.hpp"

namespace arbgpu_impl {

__global__ __launch_bounds__(256) void gather_lines_kernel(GatherParams P) {
  __shared__ uint32_t tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t k_base = (int64_t)blockIdx.x * 64, l_base = (int64_t)blockIdx.y * 64;
  const int nplanes = P.src.cap + 2;
  for (int q = 0; q < nplanes; ++q) {
    // read: lanes along the line index (consecutive in the source)
    for (int r = ty; r < 64; r += 4) {
      const int64_t k = k_base + r, line = l_base + tx;
      uint32_t v = 0;
      if (k < P.len && line < P.lines) {
        const int64_t idx = P.off + line * P.line_stride + (P.k0 + k) * P.elem_stride;
        v = q < P.src.cap ? P.src.limbs[(int64_t)q * P.src.ld + idx]
                          : (q == P.src.cap ? (uint32_t)P.src.exp[idx] : (uint32_t)P.src.nls[idx]);
      }
      tile[r][tx] = v;
    }
    __syncthreads();
    // write: lanes along the inner index (consecutive in the copy)
    for (int r = ty; r < 64; r += 4) {
      const int64_t line = l_base + r, k = k_base + tx;
      if (k < P.len && line < P.lines) {
        const int64_t o = line * P.len + k;
        const uint32_t v = tile[tx][r];
        if (q < P.src.cap) P.limbs[(int64_t)q * P.lines * P.len + o] = v;
        else if (q == P.src.cap) P.exp[o] = (int32_t)v;
        else P.nls[o] = (int32_t)v;
      }
    }
    __syncthreads();
  }
}

hipError_t launch_gather(const GatherParams &P, hipStream_t s) {
  if (P.lines == 0 || P.len == 0) return hipSuccess;
  const dim3 grid((unsigned)((P.len + 63) / 64), (unsigned)((P.lines + 63) / 64));
  hipLaunchKernelGGL(gather_lines_kernel, grid, dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
