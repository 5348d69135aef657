// Choice of the limb-kernel shape (window limbs NS, operand limbs NA) and
// dispatch to the per-shape instantiations.
#include "internal.hpp"
#include "limb_shapes.def"

namespace arbgpu_impl {

static const int kShapes[][2] = {
#define X(a, b) {a, b},
    ARB_LIMB_SHAPES(X)
#undef X
};

bool limb_shape_for(int p, int64_t nterms, int cap, LimbShape *out) {
  // window: p bits, extend = bc(nonzero terms) + 1 leading bits (Section
  // 3.3, steps 9-10) and 40 guard bits for the exact decision
  int bc = 0;
  for (int64_t v = nterms + 1; v; v >>= 1) ++bc;
  const int64_t need_bits = (int64_t)p + bc + 1 + 40;
  const int64_t ns_min = (need_bits + 31) / 32;
  int best = -1;
  for (unsigned k = 0; k < sizeof(kShapes) / sizeof(kShapes[0]); ++k) {
    const int ns = kShapes[k][0], na = kShapes[k][1];
    if (ns < ns_min) continue;
    // operand limbs: all of them, or at least NS + 1, the most a term can
    // contribute to a window whose top it does not exceed
    const int na_need = cap < ns + 1 ? cap : ns + 1;
    if (na < na_need) continue;
    if (best < 0 || ns < kShapes[best][0] || (ns == kShapes[best][0] && na < kShapes[best][1])) best = (int)k;
  }
  if (best < 0) return false;
  out->ns = kShapes[best][0];
  out->na = kShapes[best][1];
  return true;
}

hipError_t launch_limb_mm(const MmParams &prm, LimbShape sh, hipStream_t s) {
#define X(a, b) \
  if (sh.ns == a && sh.na == b) return launch_mm_shape<a, b>(prm, s);
  ARB_LIMB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_limb_mm_list(const MmParams &prm, LimbShape sh, const int64_t *list, const int32_t *count,
                               int64_t max_count, hipStream_t s) {
#define X(a, b) \
  if (sh.ns == a && sh.na == b) return launch_mm_list_shape<a, b>(prm, list, count, max_count, s);
  ARB_LIMB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

const void *dot_batch_kernel(LimbShape sh, bool block) {
#define X(a, b) \
  if (sh.ns == a && sh.na == b) return dot_batch_kernel_shape<a, b>(block);
  ARB_LIMB_SHAPES(X)
#undef X
  return nullptr;
}

hipError_t launch_limb_dot(const DotParams &prm, LimbShape sh, hipStream_t s, const int32_t *gate) {
#define X(a, b) \
  if (sh.ns == a && sh.na == b) return launch_dot_shape<a, b>(prm, s, gate);
  ARB_LIMB_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace arbgpu_impl
