// Final step of the multi-block product (Algorithm 2, Johansson 2019,
// Section 4.1): every output entry is the exact sum of its block results
// T_s 2^(-e_i - f_j) (exact floats from the INT8-MFMA products) and of the
// basecase chunks' products a_ik b_kj, truncated once to p bits by the
// window engine with exact refinement.  Operands are read in place (any
// length), one lane per entry.
#include "limb_kernels.hpp"
#include "sliced.hpp"

using namespace arb;

namespace arbgpu_impl {

namespace {

struct MergeSrc {
  const MergeParams *P;
  int64_t ij, abase, bbase;
  __device__ __forceinline__ int64_t nterms() const { return P->nS + P->nbk * P->ct.ncomp; }
  __device__ __forceinline__ bool has_init() const { return false; }
  __device__ __forceinline__ void term(int64_t t, SOpnd &a, SOpnd &b, uint32_t &neg, bool limbs) const {
    if (t < P->nS) {
      load_op(P->T, t * P->M * P->N + ij, a, limbs);
      make_one(b);
      neg = a.sign;
      return;
    }
    const int64_t u = t - P->nS;
    const int s = P->ct.ncomp == 2 ? (int)(u & 1) : 0;
    const int64_t k = P->bk[P->ct.ncomp == 2 ? (u >> 1) : u];
    load_op(pick(P->A, P->ct.pa[s]), abase + k * P->a_cs, a, limbs);
    load_op(pick(P->B, P->ct.pb[s]), bbase + k * P->b_rs, b, limbs);
    neg = a.sign ^ b.sign ^ P->ct.ng[s];
  }
  __device__ __forceinline__ void init(SOpnd &, SOpnd &, bool) const {}
};

}  // namespace

template <int NS>
__global__ __launch_bounds__(256) void merge_kernel(MergeParams prm) {
  const int64_t ij = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (ij >= prm.M * prm.N) return;
  const int64_t i = ij / prm.N, j = ij - i * prm.N;
  MergeSrc src{&prm, ij, prm.a_off + i * prm.a_rs, prm.b_off + j * prm.b_cs};
  DotOut<NS> out;
  run_dot<NS, SOpnd, SoloReducer>(src, prm.p, false, out);
  if (!out.erange && prm.rin_m) {
    out.rin_m = prm.rin_m[ij];
    out.rin_e = prm.rin_e[ij];
  }
  store_out<NS>(prm.C, prm.c_off + i * prm.c_rs + j * prm.c_cs, out, prm.p, prm.approx,
                status_of(out, false));
}

hipError_t launch_merge(const MergeParams &P, int ns, hipStream_t s) {
  const int64_t n = P.M * P.N;
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
#define X(a)                                                                          \
  if (ns == a) {                                                                      \
    hipLaunchKernelGGL((merge_kernel<a>), dim3(blocks), dim3(256), 0, s, P);          \
    return hipGetLastError();                                                         \
  }
  X(4) X(6) X(8) X(10) X(12) X(14) X(18) X(22) X(26) X(30) X(34) X(38)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace arbgpu_impl
