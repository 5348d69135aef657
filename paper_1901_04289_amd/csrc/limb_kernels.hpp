// Limb-window kernels: Algorithm 1 (Johansson 2019, Section 3) per output.
//
// limb_mm_kernel: one lane per output entry of a matrix product (the
//   classical product as M*K dot products, Section 4); lanes of a wave take
//   neighbouring columns, so the B operand reads are coalesced and the A
//   operand is a broadcast.
// limb_dot_kernel: one wave per dot product; the 64 lanes split the terms,
//   and windows, error counts and radius sums are reduced across the wave
//   with exact (modular) additions, so the result does not depend on the
//   split.
//
// Both keep the window and the operand limbs in registers (NS and NA are
// compile-time).  When a refinement level needs more operand limbs than
// were loaded, the lane redoes the output with the streaming exact operand
// path (SOpnd), which reads limbs in place and never truncates.
#pragma once

#include <math.h>

#include "internal.hpp"
#include "engine.hpp"

using namespace arb;

namespace arbgpu_impl {

// The arrays behind arbgpu_arr / arbgpu_out live in device global memory.
template <class T>
__device__ __forceinline__ const ARB_GLOBAL T *gp(const T *p) {
  return (const ARB_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ ARB_GLOBAL T *gpw(T *p) {
  return (ARB_GLOBAL T *)p;
}

template <int NA>
__device__ __forceinline__ void load_op(const arbgpu_arr &A, int64_t idx, Opnd<NA> &o, bool limbs) {
  const int32_t nl = gp(A.nls)[idx];
  int n = nl & 0x7FFFFFFF;
  if (n > A.cap) n = A.cap;
  o.sign = (uint32_t)nl >> 31;
  o.e = gp(A.exp)[idx];
  const int nt = n < NA ? n : NA;
  o.trunc = n > NA;
  o.n = nt;
  const ARB_GLOBAL uint32_t *L = gp(A.limbs);
#pragma unroll
  for (int i = 0; i < NA; ++i)
    o.l[i] = (limbs && i < nt) ? L[(int64_t)(nt - 1 - i) * A.ld + idx] : 0u;
  o.rm = 0.0;
  o.re = 0;
  if (A.rad_m) {
    const double r = gp(A.rad_m)[idx];
    if (r != 0.0) {
      if (r > 0.0 && r < INFINITY) {
        int ex;
        o.rm = frexp(r, &ex);
        o.re = gp(A.rad_e)[idx] + ex;
      } else {
        o.rm = 1.0;
        o.re = kExpLimit;   // reported as out of range
      }
    }
  }
}

__device__ __forceinline__ void load_op(const arbgpu_arr &A, int64_t idx, SOpnd &o, bool) {
  const int32_t nl = gp(A.nls)[idx];
  int n = nl & 0x7FFFFFFF;
  if (n > A.cap) n = A.cap;
  o.l = gp(A.limbs);
  o.ld = A.ld;
  o.idx = idx;
  o.n = n;
  o.trunc = false;
  o.sign = (uint32_t)nl >> 31;
  o.e = gp(A.exp)[idx];
  o.rm = 0.0;
  o.re = 0;
  if (A.rad_m) {
    const double r = gp(A.rad_m)[idx];
    if (r != 0.0) {
      if (r > 0.0 && r < INFINITY) {
        int ex;
        o.rm = frexp(r, &ex);
        o.re = gp(A.rad_e)[idx] + ex;
      } else {
        o.rm = 1.0;
        o.re = kExpLimit;
      }
    }
  }
}

static __device__ const uint32_t kOneLimb[1] = {0x80000000u};

template <int NA>
__device__ __forceinline__ void make_one(Opnd<NA> &o) {
#pragma unroll
  for (int i = 0; i < NA; ++i) o.l[i] = 0;
  o.l[0] = 0x80000000u;
  o.n = 1; o.trunc = false; o.e = 1; o.sign = 0; o.rm = 0.0; o.re = 0;
}
__device__ __forceinline__ void make_one(SOpnd &o) {
  o.l = gp(kOneLimb); o.ld = 1; o.idx = 0;
  o.n = 1; o.trunc = false; o.e = 1; o.sign = 0; o.rm = 0.0; o.re = 0;
}

template <class AP>
__device__ __forceinline__ arbgpu_arr pick(const AP &arr, int i) { return i ? arr[1] : arr[0]; }

// Terms of output (i, j) of a matrix product.
template <class Op, class PP = const MmParams *>
struct MmSrc {
  PP P;
  int64_t abase, bbase;
  __device__ __forceinline__ int64_t nterms() const { return P->N * P->ct.ncomp; }
  __device__ __forceinline__ bool has_init() const { return false; }
  __device__ __forceinline__ void term(int64_t t, Op &a, Op &b, uint32_t &neg, bool limbs) const {
    const int s = P->ct.ncomp == 2 ? (int)(t & 1) : 0;
    const int64_t k = P->ct.ncomp == 2 ? (t >> 1) : t;
    load_op(pick(P->A, P->ct.pa[s]), abase + k * P->a_cs, a, limbs);
    load_op(pick(P->B, P->ct.pb[s]), bbase + k * P->b_rs, b, limbs);
    neg = a.sign ^ b.sign ^ P->ct.ng[s];
  }
  __device__ __forceinline__ void init(Op &, Op &, bool) const {}
};

// Terms of one dot product.
template <class Op, class PP = const DotParams *>
struct DotSrc {
  PP P;
  __device__ __forceinline__ int64_t nterms() const { return P->N * P->ct.ncomp; }
  __device__ __forceinline__ bool has_init() const { return P->has_init != 0; }
  __device__ __forceinline__ void term(int64_t t, Op &a, Op &b, uint32_t &neg, bool limbs) const {
    const int s = P->ct.ncomp == 2 ? (int)(t & 1) : 0;
    const int64_t k = P->ct.ncomp == 2 ? (t >> 1) : t;
    load_op(pick(P->X, P->ct.pa[s]), P->xoff + k * P->xstep, a, limbs);
    load_op(pick(P->Y, P->ct.pb[s]), P->yoff + k * P->ystep, b, limbs);
    neg = a.sign ^ b.sign ^ P->ct.ng[s] ^ P->sub;
  }
  __device__ __forceinline__ void init(Op &a, Op &one, bool limbs) const {
    load_op(pick(P->I, P->init_part), P->init_idx, a, limbs);
    make_one(one);
  }
};

// Cross-lane reductions for one wave per output.  Butterfly exchanges give
// every lane the same totals; window additions are exact modulo 2^(32 NS)
// and the upward FP64 sum is order-independent in its error test.
struct WaveReducer {
  __device__ __forceinline__ static int lane() { return threadIdx.x & 63; }
  __device__ __forceinline__ static int group() { return 64; }
  __device__ __forceinline__ static void setup(Setup &S) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      int e = __shfl_xor(S.emax, m, 64);
      S.emax = e > S.emax ? e : S.emax;
      S.nnz += (uint32_t)__shfl_xor((int)S.nnz, m, 64);
      int f = __shfl_xor(S.F, m, 64);
      S.F = f > S.F ? f : S.F;
      S.any_rad = __shfl_xor((int)S.any_rad, m, 64) | S.any_rad;
      S.erange = __shfl_xor((int)S.erange, m, 64) | S.erange;
    }
  }
  template <int NS>
  __device__ __forceinline__ static void window(Window<NS> &W) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      uint32_t o[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) o[i] = (uint32_t)__shfl_xor((int)W.w[i], m, 64);
      madd<NS>(W.w, o);
      W.err += (uint32_t)__shfl_xor((int)W.err, m, 64);
      W.pt += (uint32_t)__shfl_xor((int)W.pt, m, 64);
      W.below_cnt += (uint32_t)__shfl_xor((int)W.below_cnt, m, 64);
      int bm = __shfl_xor(W.below_max, m, 64);
      W.below_max = bm > W.below_max ? bm : W.below_max;
      W.bad = __shfl_xor((int)W.bad, m, 64) | W.bad;
    }
  }
  __device__ __forceinline__ static void rad(RadAcc &r) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
      uint64_t o[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) o[k] = (uint64_t)__shfl_xor((long long)r.w[k], m, 64);
      r.add_words(o[0], o[1], o[2]);
    }
  }
};

// Cross-wave reductions for NW waves per output (one workgroup): each wave
// reduces with WaveReducer, the wave totals meet in LDS and every lane adds
// them in wave order.  Window sums are modular, counts are integers and the
// radius sum is exact, so the result is the one-wave result bit for bit.
template <int NW>
struct BlockReducer {
  __device__ __forceinline__ static int lane() { return threadIdx.x; }
  __device__ __forceinline__ static int group() { return 64 * NW; }
  __device__ __forceinline__ static void setup(Setup &S) {
    __shared__ Setup sh[NW];
    WaveReducer::setup(S);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = S;
    __syncthreads();
    Setup T = sh[0];
    for (int w = 1; w < NW; ++w) {
      const Setup o = sh[w];
      T.emax = o.emax > T.emax ? o.emax : T.emax;
      T.nnz += o.nnz;
      T.F = o.F > T.F ? o.F : T.F;
      T.any_rad = T.any_rad || o.any_rad;
      T.erange = T.erange || o.erange;
    }
    __syncthreads();
    S = T;
  }
  template <int NS>
  __device__ __forceinline__ static void window(Window<NS> &W) {
    __shared__ Window<NS> sh[NW];
    WaveReducer::window<NS>(W);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = W;
    __syncthreads();
    Window<NS> T = sh[0];
    for (int w = 1; w < NW; ++w) {
      uint32_t o[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) o[i] = sh[w].w[i];
      madd<NS>(T.w, o);
      T.err += sh[w].err;
      T.pt += sh[w].pt;
      T.below_cnt += sh[w].below_cnt;
      T.below_max = sh[w].below_max > T.below_max ? sh[w].below_max : T.below_max;
      T.bad = T.bad || sh[w].bad;
    }
    __syncthreads();
    W = T;
  }
  __device__ __forceinline__ static void rad(RadAcc &r) {
    __shared__ RadAcc sh[NW];
    WaveReducer::rad(r);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = r;
    __syncthreads();
    RadAcc T = sh[0];
    for (int w = 1; w < NW; ++w) T.add(sh[w]);
    __syncthreads();
    r = T;
  }
};

template <int NS>
__device__ __forceinline__ void store_out(const arbgpu_out &o, int64_t idx, const DotOut<NS> &r, int p, int approx,
                          uint8_t status) {
  const int PL = (p + 31) >> 5;
  int n = 0;
#pragma unroll
  for (int i = NS - 1; i >= 0; --i) {
    const int k = NS - 1 - i;
    if (k < PL) {
      const uint32_t v = r.st.zero ? 0u : r.st.Y[i];
      gpw(o.limbs)[(int64_t)k * o.ld + idx] = v;
      if (v) n = k + 1;
    }
  }
  gpw(o.exp)[idx] = r.st.zero ? 0 : r.st.r_exp;
  gpw(o.nls)[idx] = r.st.zero ? 0 : (int32_t)((uint32_t)n | (r.st.r_sign << 31));
  if (!approx) {
    double rm;
    int re;
    if (r.erange) {
      rm = INFINITY;
      re = 0;
    } else {
      total_radius(r, r.p, rm, re);
    }
    gpw(o.rad_m)[idx] = rm;
    gpw(o.rad_e)[idx] = re;
  }
  if (o.status) gpw(o.status)[idx] = status;
}

template <int NS>
__device__ __forceinline__ uint8_t status_of(const DotOut<NS> &r, bool fell_back) {
  if (r.erange) return ARBGPU_ST_ERANGE;
  return (fell_back || r.st.levels > 1) ? ARBGPU_ST_REFINED : ARBGPU_ST_OK;
}

template <int NS, int NA>
__global__ __launch_bounds__(256) void limb_mm_kernel(MmParams prm) {
  const int64_t tiles_j = (prm.K + 63) >> 6;
  const int64_t bid = blockIdx.x;
  const int64_t j = (bid % tiles_j) * 64 + (threadIdx.x & 63);
  const int64_t i = (bid / tiles_j) * 4 + (threadIdx.x >> 6);
  if (i >= prm.M || j >= prm.K) return;
  const int64_t abase = prm.a_off + i * prm.a_rs;
  const int64_t bbase = prm.b_off + j * prm.b_cs;
  DotOut<NS> out;
  MmSrc<Opnd<NA>> src{&prm, abase, bbase};
  run_dot<NS, Opnd<NA>, SoloReducer>(src, prm.p, !prm.approx, out);
  bool fell_back = false;
  if (out.st.bad) {
    MmSrc<SOpnd> s2{&prm, abase, bbase};
    run_dot<NS, SOpnd, SoloReducer>(s2, prm.p, !prm.approx, out);
    fell_back = true;
  }
  store_out<NS>(prm.C, prm.c_off + i * prm.c_rs + j * prm.c_cs, out, prm.p, prm.approx,
                status_of(out, fell_back));
}

// One wave per output entry, the entry's terms split over the lanes and
// merged as in limb_dot_kernel: for products with few entries, where one
// lane per entry would leave most of the machine idle and run each entry's
// terms one after another.  Four entries per workgroup.
template <int NS, int NA>
__global__ __launch_bounds__(256) void limb_mm_wave_kernel(MmParams prm) {
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= prm.M * prm.K) return;   // whole waves leave together
  const int64_t i = e / prm.K, j = e - i * prm.K;
  const int64_t abase = prm.a_off + i * prm.a_rs;
  const int64_t bbase = prm.b_off + j * prm.b_cs;
  DotOut<NS> out;
  MmSrc<Opnd<NA>> src{&prm, abase, bbase};
  run_dot<NS, Opnd<NA>, WaveReducer>(src, prm.p, !prm.approx, out);
  bool fell_back = false;
  if (out.st.bad) {   // uniform across the wave
    MmSrc<SOpnd> s2{&prm, abase, bbase};
    run_dot<NS, SOpnd, WaveReducer>(s2, prm.p, !prm.approx, out);
    fell_back = true;
  }
  if ((threadIdx.x & 63) == 0)
    store_out<NS>(prm.C, prm.c_off + i * prm.c_rs + j * prm.c_cs, out, prm.p, prm.approx,
                  status_of(out, fell_back));
}

// Listed entries (index i K + j) of a matrix product, one wave each, as
// limb_mm_wave_kernel: the exact recomputation of the entries whose
// truncation a truncated integer product could not certify (a few entries
// of a large product, each with its whole inner length: a wave per entry
// keeps one such entry from taking a single lane through all its terms).
// The waves stride over the list, whose length the device holds.
template <int NS, int NA>
__global__ __launch_bounds__(256) void limb_mm_list_kernel(MmParams prm, const int64_t *list, const int32_t *count) {
  const int64_t n = *gp(count);
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); t < n; t += nw) {   // uniform across the wave
    const int64_t ij = gp(list)[t];
    const int64_t i = ij / prm.K, j = ij - i * prm.K;
    const int64_t abase = prm.a_off + i * prm.a_rs;
    const int64_t bbase = prm.b_off + j * prm.b_cs;
    DotOut<NS> out;
    MmSrc<Opnd<NA>> src{&prm, abase, bbase};
    run_dot<NS, Opnd<NA>, WaveReducer>(src, prm.p, !prm.approx, out);
    bool fell_back = false;
    if (out.st.bad) {   // uniform across the wave
      MmSrc<SOpnd> s2{&prm, abase, bbase};
      run_dot<NS, SOpnd, WaveReducer>(s2, prm.p, !prm.approx, out);
      fell_back = true;
    }
    if ((threadIdx.x & 63) == 0)
      store_out<NS>(prm.C, prm.c_off + i * prm.c_rs + j * prm.c_cs, out, prm.p, prm.approx,
                    status_of(out, fell_back));
  }
}

template <int NS, int NA>
__global__ __launch_bounds__(64) void limb_dot_kernel(DotParams prm, const int32_t *gate) {
  if (gate && *gp(gate) == 0) return;   // the digit product certified this dot
  DotOut<NS> out;
  DotSrc<Opnd<NA>> src{&prm};
  run_dot<NS, Opnd<NA>, WaveReducer>(src, prm.p, !prm.approx, out, prm.reduce != 0);
  bool fell_back = false;
  if (out.st.bad) {   // uniform across the wave: every lane holds the same state
    DotSrc<SOpnd> s2{&prm};
    run_dot<NS, SOpnd, WaveReducer>(s2, prm.p, !prm.approx, out, prm.reduce != 0);
    fell_back = true;
  }
  if (threadIdx.x == 0) store_out<NS>(prm.R, prm.res_idx, out, prm.p, prm.approx, status_of(out, fell_back));
}

// One workgroup of four waves per dot product: the terms split over 256
// lanes, the waves' windows, error counts and radius sums added in LDS.
// The result is limb_dot_kernel's bit for bit.
template <int NS, int NA>
__global__ __launch_bounds__(256) void limb_dot_block_kernel(DotParams prm, const int32_t *gate) {
  if (gate && *gp(gate) == 0) return;
  DotOut<NS> out;
  DotSrc<Opnd<NA>> src{&prm};
  run_dot<NS, Opnd<NA>, BlockReducer<4>>(src, prm.p, !prm.approx, out, prm.reduce != 0);
  bool fell_back = false;
  if (out.st.bad) {   // uniform across the workgroup
    DotSrc<SOpnd> s2{&prm};
    run_dot<NS, SOpnd, BlockReducer<4>>(s2, prm.p, !prm.approx, out, prm.reduce != 0);
    fell_back = true;
  }
  if (threadIdx.x == 0) store_out<NS>(prm.R, prm.res_idx, out, prm.p, prm.approx, status_of(out, fell_back));
}

// Persistent batch: waves take tasks from a work counter until the list
// of this shape is exhausted.  A task is one dot output as in
// limb_dot_kernel (order entry e >= 0: dot task e), or a tile of 64
// entries of one row of a matrix product (e < 0: tile -e - 1), one entry
// per lane as in limb_mm_kernel or, for products that run a wave per
// entry alone, entry by entry as in limb_mm_wave_kernel.  Four independent
// waves per workgroup.
template <int NS, int NA>
__global__ __launch_bounds__(256) void limb_dot_batch_kernel(BatchShapeParams bp) {
  const int lane = threadIdx.x & 63;
  int64_t count = bp.count;
  if (bp.dcount) {
    const int64_t d = *gp(bp.dcount);
    count = d < count ? d : count;
  }
  if (count == 0) return;   // an empty list: no wave touches the counter
  // the counter only grows, so a wave takes at most `count` tasks
  for (int64_t iter = 0; iter <= count; ++iter) {
    int t = 0;
    if (lane == 0) t = atomicAdd(bp.counter, 1);
    t = __shfl(t, 0, 64);
    if (t >= count) break;   // uniform across the wave
    // uniform task index: the parameters are read with scalar loads
    const int tu = __builtin_amdgcn_readfirstlane(t);
    const int32_t e = __builtin_amdgcn_readfirstlane(gp(bp.order)[tu]);
    if (e < 0) {
      const BatchTile tl = gp(bp.tiles)[-e - 1];
      const ARB_GLOBAL MmParams *mp = gp(bp.mm) + tl.part;
      if (tl.wave) {   // entry by entry, the terms split over the lanes
        const int64_t i = tl.i, jend = tl.j0 + 64 < mp->K ? tl.j0 + 64 : mp->K;
        for (int64_t j = tl.j0; j < jend; ++j) {
          const int64_t abase = mp->a_off + i * mp->a_rs, bbase = mp->b_off + j * mp->b_cs;
          DotOut<NS> out;
          MmSrc<Opnd<NA>, const ARB_GLOBAL MmParams *> src{mp, abase, bbase};
          run_dot<NS, Opnd<NA>, WaveReducer>(src, mp->p, !mp->approx, out);
          bool fell_back = false;
          if (out.st.bad) {
            MmSrc<SOpnd, const ARB_GLOBAL MmParams *> s2{mp, abase, bbase};
            run_dot<NS, SOpnd, WaveReducer>(s2, mp->p, !mp->approx, out);
            fell_back = true;
          }
          if (lane == 0)
            store_out<NS>(mp->C, mp->c_off + i * mp->c_rs + j * mp->c_cs, out, mp->p, mp->approx,
                          status_of(out, fell_back));
        }
        continue;
      }
      const int64_t i = tl.i, j = tl.j0 + lane;
      if (j < mp->K) {
        const int64_t abase = mp->a_off + i * mp->a_rs, bbase = mp->b_off + j * mp->b_cs;
        DotOut<NS> out;
        MmSrc<Opnd<NA>, const ARB_GLOBAL MmParams *> src{mp, abase, bbase};
        run_dot<NS, Opnd<NA>, SoloReducer>(src, mp->p, !mp->approx, out);
        bool fell_back = false;
        if (out.st.bad) {
          MmSrc<SOpnd, const ARB_GLOBAL MmParams *> s2{mp, abase, bbase};
          run_dot<NS, SOpnd, SoloReducer>(s2, mp->p, !mp->approx, out);
          fell_back = true;
        }
        store_out<NS>(mp->C, mp->c_off + i * mp->c_rs + j * mp->c_cs, out, mp->p, mp->approx,
                      status_of(out, fell_back));
      }
      continue;
    }
    const ARB_GLOBAL DotParams *prm = gp(bp.tasks) + e;
    DotOut<NS> out;
    DotSrc<Opnd<NA>, const ARB_GLOBAL DotParams *> src{prm};
    run_dot<NS, Opnd<NA>, WaveReducer>(src, prm->p, !prm->approx, out, prm->reduce != 0);
    bool fell_back = false;
    if (out.st.bad) {
      DotSrc<SOpnd, const ARB_GLOBAL DotParams *> s2{prm};
      run_dot<NS, SOpnd, WaveReducer>(s2, prm->p, !prm->approx, out, prm->reduce != 0);
      fell_back = true;
    }
    if (lane == 0) store_out<NS>(prm->R, prm->res_idx, out, prm->p, prm->approx, status_of(out, fell_back));
  }
}

// Persistent batch, long dots: each workgroup of four waves takes one dot
// task at a time from the shape's counter and runs it as
// limb_dot_block_kernel (same bits as one wave).
template <int NS, int NA>
__global__ __launch_bounds__(256) void limb_dot_batch_block_kernel(BatchShapeParams bp) {
  __shared__ int task;
  int64_t count = bp.count;
  if (bp.dcount) {
    const int64_t d = *gp(bp.dcount);
    count = d < count ? d : count;
  }
  if (count == 0) return;
  for (int64_t iter = 0; iter <= count; ++iter) {
    if (threadIdx.x == 0) task = atomicAdd(bp.counter, 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(task);
    __syncthreads();   // every thread has read it before the next take
    if (t >= count) break;   // uniform across the workgroup
    const int32_t e = __builtin_amdgcn_readfirstlane(gp(bp.order)[t]);
    const ARB_GLOBAL DotParams *prm = gp(bp.tasks) + e;
    DotOut<NS> out;
    DotSrc<Opnd<NA>, const ARB_GLOBAL DotParams *> src{prm};
    run_dot<NS, Opnd<NA>, BlockReducer<4>>(src, prm->p, !prm->approx, out, prm->reduce != 0);
    bool fell_back = false;
    if (out.st.bad) {
      DotSrc<SOpnd, const ARB_GLOBAL DotParams *> s2{prm};
      run_dot<NS, SOpnd, BlockReducer<4>>(s2, prm->p, !prm->approx, out, prm->reduce != 0);
      fell_back = true;
    }
    if (threadIdx.x == 0) store_out<NS>(prm->R, prm->res_idx, out, prm->p, prm->approx, status_of(out, fell_back));
  }
}

}  // namespace arbgpu_impl
