// One (window limbs, operand limbs) instantiation of the limb kernels.
// Built once per shape with -DARB_NS=<window limbs> -DARB_NA=<operand limbs>
// so the shapes compile in parallel.
#include <algorithm>

#include "limb_kernels.hpp"

#if !defined(ARB_NS) || !defined(ARB_NA)
#error "build with -DARB_NS=... -DARB_NA=..."
#endif

namespace arbgpu_impl {

template <>
hipError_t launch_mm_shape<ARB_NS, ARB_NA>(const MmParams &prm, hipStream_t s) {
  const int64_t entries = prm.M * prm.K;
  if (entries == 0) return hipSuccess;
  if (entries < kMmWaveEntries) {   // a wave per entry
    hipLaunchKernelGGL((limb_mm_wave_kernel<ARB_NS, ARB_NA>), dim3((unsigned)((entries + 3) / 4)), dim3(256), 0, s,
                       prm);
    return hipGetLastError();
  }
  const int64_t blocks = ((prm.K + 63) / 64) * ((prm.M + 3) / 4);
  hipLaunchKernelGGL((limb_mm_kernel<ARB_NS, ARB_NA>), dim3((unsigned)blocks), dim3(256), 0, s, prm);
  return hipGetLastError();
}

template <>
hipError_t launch_mm_list_shape<ARB_NS, ARB_NA>(const MmParams &prm, const int64_t *list, const int32_t *count,
                                                int64_t max_count, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((max_count + 3) / 4, 1024);   // four entries (waves) per workgroup
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((limb_mm_list_kernel<ARB_NS, ARB_NA>), dim3((unsigned)blocks), dim3(256), 0, s, prm, list, count);
  return hipGetLastError();
}

template <>
hipError_t launch_dot_shape<ARB_NS, ARB_NA>(const DotParams &prm, hipStream_t s, const int32_t *gate) {
  if (prm.N * prm.ct.ncomp >= kDotBlockTerms)   // four waves share the terms
    hipLaunchKernelGGL((limb_dot_block_kernel<ARB_NS, ARB_NA>), dim3(1), dim3(256), 0, s, prm, gate);
  else
    hipLaunchKernelGGL((limb_dot_kernel<ARB_NS, ARB_NA>), dim3(1), dim3(64), 0, s, prm, gate);
  return hipGetLastError();
}

template <>
const void *dot_batch_kernel_shape<ARB_NS, ARB_NA>(bool block) {
  return block ? reinterpret_cast<const void *>(&limb_dot_batch_block_kernel<ARB_NS, ARB_NA>)
               : reinterpret_cast<const void *>(&limb_dot_batch_kernel<ARB_NS, ARB_NA>);
}

}  // namespace arbgpu_impl
