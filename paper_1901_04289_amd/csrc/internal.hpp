// Internal interfaces between the C-ABI front end (api.hip) and the kernel
// translation units.  Not installed; the public interface is arbgpu.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/arbgpu.h"

namespace arbgpu_impl {

// Which operand parts form the terms of one real output (Section 3.6: the
// real part of a complex dot is the 2N-term real dot of a c and -(b d), the
// imaginary part that of a d and b c).
struct CompTab {
  int ncomp;          // 1 (real) or 2 (complex)
  int pa[2], pb[2];   // part index (0 re, 1 im) of the x / y operand
  uint32_t ng[2];     // 1 negates the term
};

inline CompTab comp_real() { return CompTab{1, {0, 0}, {0, 0}, {0u, 0u}}; }
inline CompTab comp_re() { return CompTab{2, {0, 1}, {0, 1}, {0u, 1u}}; }
inline CompTab comp_im() { return CompTab{2, {0, 1}, {1, 0}, {0u, 0u}}; }

struct MmParams {
  arbgpu_arr A[2], B[2];
  arbgpu_out C;             // the output part this launch writes
  int64_t M, N, K;          // C is M x K, inner dimension N
  int64_t a_off, a_rs, a_cs;
  int64_t b_off, b_rs, b_cs;
  int64_t c_off, c_rs, c_cs;
  int p;
  int approx;
  CompTab ct;
};

struct DotParams {
  arbgpu_arr X[2], Y[2], I[2];
  int has_init;
  int64_t init_idx;
  arbgpu_out R;             // the output part this launch writes
  int64_t res_idx;
  int64_t xoff, xstep, yoff, ystep, N;
  int p;
  int approx;
  uint32_t sub;
  int init_part;            // which part of the initial value feeds this output
  CompTab ct;
};

// Window / operand-limb template choice for the limb kernels.
struct LimbShape {
  int ns;   // window limbs
  int na;   // operand limbs held in registers
};

bool limb_shape_for(int p, int64_t nterms, int cap, LimbShape *out);
template <int NS, int NA>
hipError_t launch_mm_shape(const MmParams &prm, hipStream_t s);
template <int NS, int NA>
hipError_t launch_dot_shape(const DotParams &prm, hipStream_t s);
hipError_t launch_limb_mm(const MmParams &prm, LimbShape sh, hipStream_t s);
hipError_t launch_limb_dot(const DotParams &prm, LimbShape sh, hipStream_t s);

}  // namespace arbgpu_impl
