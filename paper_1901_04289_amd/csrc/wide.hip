// Dot products at precisions beyond the register windows of the limb
// kernels (Algorithm 1 of Johansson 2019 at any p): the accumulation window
// (Section 3.3, steps 9-11: top e_max + extend, p + extend + guard bits)
// is kept in LDS as signed 64-bit columns of 32 bits each, one workgroup
// per output.  For every term all threads stage the two operands' limbs
// that reach the window (the first shifted to the window's bit alignment)
// and each thread forms whole columns of the product: the low halves of
// the 32 x 32 -> 64 limb products of its column and the high halves of
// those one column down, so no two threads write the same column.  Product
// bits below the window bottom are dropped and counted as error units, as
// the paper's truncated products count theirs (Section 3.4).  The window
// value and its error then either certify the truncation to p bits or the
// sum is formed again exactly in a window reaching down to the lowest bit
// of every product (the fast dot with an exact fallback, Section 2).
#include "finish.hpp"
#include "limb_kernels.hpp"
#include "window.hpp"

using namespace arb;

namespace arbgpu_impl {

namespace {

constexpr int kWideThreads = 256;
constexpr int kWideCols = 4096;   // window columns held in LDS (131072 bits)
constexpr int kWideGuard = 64;    // bits below the output's p and the extend bits
constexpr int kWideOpLimbs = 2048;   // operand limbs staged per term
constexpr int kWideStage = kWideOpLimbs + 8;

// 49 KiB: the columns, then (after normalisation) the window's limbs in
// their low 32 bits; the staged operands of one term, or the upper bound
// of the certification.
struct WideLds {
  int64_t col[kWideCols];
  uint32_t a[kWideStage], b[kWideStage];   // staged operand limbs, least significant first
  // reductions
  int red_i[kWideThreads / 64][4];
  double red_d[kWideThreads / 64];
  int certified;
  int64_t hb;
};

__device__ __forceinline__ int64_t floor_div32(int64_t v) { return v >= 0 ? (v >> 5) : -((31 - v) >> 5); }

__device__ __forceinline__ uint32_t limb(const WideLds &L, int c) { return (uint32_t)L.col[c]; }
__device__ __forceinline__ void set_limb(WideLds &L, int c, uint32_t v) { L.col[c] = (int64_t)v; }

// Accumulates every term into the window [lo, lo + 32 nW) of L.col (all
// threads).  Returns, in thread 0, the error bound in units of 2^lo: one
// per product dropped whole or cut by the window bottom, plus the cut
// columns' bound, plus one per operand whose low limbs were left out.
template <class Src>
__device__ uint64_t wide_accumulate(const Src &src, int64_t nt, bool has_init, int64_t lo, int nW, WideLds &L,
                                    bool want_rad, int F, double &racc) {
  const int tid = threadIdx.x;
  for (int c = tid; c < nW; c += kWideThreads) L.col[c] = 0;
  __syncthreads();
  uint64_t err = 0;
  const int64_t total = nt + (has_init ? 1 : 0);
  for (int64_t t = 0; t < total; ++t) {
    // keep every column below 2^62: a term adds less than 2^45 to one
    // (carries out of the top column vanish modulo 2^(32 nW))
    if (t && (t & 0xFFFF) == 0) {
      if (tid == 0) {
        int64_t cy = 0;
        for (int c = 0; c < nW; ++c) {
          const int64_t v = L.col[c] + cy;
          L.col[c] = v & 0xFFFFFFFFll;
          cy = v >> 32;
        }
      }
      __syncthreads();
    }
    SOpnd a, b;
    uint32_t neg;
    if (t < nt) {
      src.term(t, a, b, neg, true);
    } else {
      src.init(a, b, true);
      neg = a.sign;
    }
    if (want_rad && tid == (int)(t % kWideThreads)) racc = ru_add(racc, rad_term(a, b, F));
    if (!a.n || !b.n) continue;
    const int64_t et = (int64_t)a.e + b.e;
    if (et <= lo) {   // the whole product lies below the window
      err += 1;
      continue;
    }
    // limbs of each operand that reach the window: the rest is below
    // 2^(et - 32 n_eff) <= 2^(lo - 96)
    const int need = (int)((et - lo + 95) / 32) + 1;
    const int na = a.n < need ? a.n : need, nb = b.n < need ? b.n : need;
    err += (na < a.n ? 1 : 0) + (nb < b.n ? 1 : 0);
    const int64_t base = et - 32 * (int64_t)(na + nb);
    const int64_t q = floor_div32(base - lo);
    const int r = (int)(base - lo - 32 * q);
    // a' = (top na limbs of a) << r, na + 1 limbs; b: top nb limbs
    for (int i = tid; i <= na; i += kWideThreads) {
      // limb i of the truncated a (least significant first) is limb
      // a.n - na + i of a
      const uint32_t lo_l = i > 0 ? a.limb_ls(a.n - na + i - 1) : 0u;
      const uint32_t hi_l = i < na ? a.limb_ls(a.n - na + i) : 0u;
      L.a[i] = r ? ((hi_l << r) | (lo_l >> (32 - r))) : hi_l;
    }
    for (int j = tid; j < nb; j += kWideThreads) L.b[j] = b.limb_ls(b.n - nb + j);
    __syncthreads();
    const int na1 = na + 1;
    // product limb k = i + j goes to column q + k (low half) and q + k + 1
    // (high half); columns below 0 are cut
    const int64_t c_lo = q > 0 ? q : 0, c_hi = q + na1 + nb + 1;
    for (int64_t c = c_lo + tid; c < c_hi && c < nW; c += kWideThreads) {
      const int64_t k = c - q;
      uint64_t sum = 0;
      {   // low halves: i + j = k
        const int64_t i0 = k - (nb - 1) > 0 ? k - (nb - 1) : 0, i1 = k < na1 - 1 ? k : na1 - 1;
        for (int64_t i = i0; i <= i1; ++i) sum += (uint32_t)(L.a[i] * L.b[k - i]);
      }
      {   // high halves: i + j = k - 1
        const int64_t k1 = k - 1;
        const int64_t i0 = k1 - (nb - 1) > 0 ? k1 - (nb - 1) : 0, i1 = k1 < na1 - 1 ? k1 : na1 - 1;
        for (int64_t i = i0; i <= i1; ++i) sum += __umulhi(L.a[i], L.b[k1 - i]);
      }
      L.col[c] += neg ? -(int64_t)sum : (int64_t)sum;
    }
    if (q < 0) {
      // cut columns: below 2 min(na + 1, nb) + 1 units of 2^lo
      err += 2 * (uint64_t)(na1 < nb ? na1 : nb) + 1;
    }
    __syncthreads();
  }
  return err;
}

// Two's-complement limbs of the window, modulo 2^(32 nW), into the low
// halves of the columns.
__device__ void wide_normalize(int nW, WideLds &L) {
  if (threadIdx.x == 0) {
    int64_t cy = 0;
    for (int c = 0; c < nW; ++c) {
      const int64_t v = L.col[c] + cy;
      set_limb(L, c, (uint32_t)v);
      cy = v >> 32;
    }
  }
  __syncthreads();
}

template <class PP>
__device__ void wide_dot(PP prm, WideLds &L) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  DotSrc<SOpnd, PP> src{prm};
  const int64_t nt = src.nterms();
  const bool has_init = src.has_init();
  const bool want_rad = !prm->approx;
  const bool reduce = prm->reduce != 0;
  // setup pass (Section 3.3): e_max, nonzero products, radius frame, and the
  // lowest bit of any product (for the exact window)
  Setup S;
  S.clear();
  int64_t lo_min = INT64_MAX;
  const int64_t total = nt + (has_init ? 1 : 0);
  for (int64_t t = tid; t < total; t += kWideThreads) {
    SOpnd a, b;
    uint32_t neg;
    if (t < nt) src.term(t, a, b, neg, false);
    else src.init(a, b, false);
    setup_term(S, a, b, want_rad || reduce);
    if (a.n && b.n) {
      const int64_t base = (int64_t)a.e + b.e - 32 * (int64_t)(a.n + b.n);
      lo_min = base < lo_min ? base : lo_min;
    }
  }
  WaveReducer::setup(S);
  for (int m = 1; m < 64; m <<= 1) {
    const int64_t o = __shfl_xor(lo_min, m, 64);
    lo_min = o < lo_min ? o : lo_min;
  }
  if (lane == 0) {
    L.red_i[wave][0] = S.emax;
    L.red_i[wave][1] = (int)S.nnz;
    L.red_i[wave][2] = S.F;
    L.red_i[wave][3] = (S.any_rad ? 1 : 0) | (S.erange ? 2 : 0);
    L.red_d[wave] = (double)0;
    L.col[wave] = lo_min;
  }
  __syncthreads();
  for (int w = 0; w < kWideThreads / 64; ++w) {
    S.emax = L.red_i[w][0] > S.emax ? L.red_i[w][0] : S.emax;
    S.F = L.red_i[w][2] > S.F ? L.red_i[w][2] : S.F;
    S.any_rad = S.any_rad || (L.red_i[w][3] & 1);
    S.erange = S.erange || (L.red_i[w][3] & 2);
    lo_min = L.col[w] < lo_min ? L.col[w] : lo_min;
  }
  uint32_t nnz = 0;
  for (int w = 0; w < kWideThreads / 64; ++w) nnz += (uint32_t)L.red_i[w][1];
  __syncthreads();
  int p = prm->p;
  if (reduce) {   // the radius-driven precision cut (Section 3.3, step 7(a))
    int64_t q = nnz ? p : 2;
    if (nnz && S.any_rad && (int64_t)S.emax - S.F + 30 < q) q = (int64_t)S.emax - S.F + 30;
    p = q < 2 ? 2 : (int)q;
  }
  const arbgpu_out &R = prm->R;
  const int64_t oidx = prm->res_idx;
  if (S.erange) {
    if (tid == 0) {
      if (!prm->approx) {
        R.rad_m[oidx] = INFINITY;
        R.rad_e[oidx] = 0;
      }
      if (R.status) R.status[oidx] = ARBGPU_ST_ERANGE;
    }
    return;
  }
  const bool rad = want_rad && S.any_rad;
  double racc = 0.0;
  uint8_t status = ARBGPU_ST_OK;
  bool exact_zero = nnz == 0;
  int64_t lo = 0;
  int nW = 1;
  if (!exact_zero) {
    const int extend = bitlen32(nnz) + 1;
    const int64_t top = (int64_t)S.emax + extend;
    nW = (int)((p + extend + kWideGuard + 31) / 32) + 1;
    lo = top - 32 * (int64_t)nW;
    const uint64_t err = wide_accumulate(src, nt, has_init, lo, nW, L, rad, S.F, racc);
    wide_normalize(nW, L);
    if (tid == 0) {
      int64_t hb = 0;
      L.certified = window_certify(nW, err, p, L.col, L.b, &hb) ? 1 : 0;
      L.hb = hb;
    }
    __syncthreads();
    if (!L.certified) {
      // exact window from just above the sum (|sum| < 2^hb units: product
      // bits above the window top are multiples of 2^(32 nW) and cancel in
      // the window's modular arithmetic) down to the lowest bit of every
      // product, so nothing is dropped
      int64_t top2 = lo + L.hb + 2;
      top2 = top2 < top ? top2 : top;
      const int64_t lo2 = 32 * floor_div32(lo_min);
      const int64_t nW2 = (top2 - lo2 + 31) / 32 + 1;
      if (nW2 > kWideCols) {   // exponent span beyond the LDS window
        if (tid == 0) {
          if (!prm->approx) {
            R.rad_m[oidx] = INFINITY;
            R.rad_e[oidx] = 0;
          }
          if (R.status) R.status[oidx] = ARBGPU_ST_ERANGE;
        }
        return;
      }
      lo = top2 - 32 * nW2;
      nW = (int)nW2;
      double unused = 0.0;
      (void)wide_accumulate(src, nt, has_init, lo, nW, L, false, S.F, unused);
      wide_normalize(nW, L);
      status = ARBGPU_ST_REFINED;
    }
  } else if (rad) {   // every midpoint product is zero: radius pass alone
    for (int64_t t = tid; t < total; t += kWideThreads) {
      SOpnd a, b;
      uint32_t neg;
      if (t < nt) src.term(t, a, b, neg, true);
      else src.init(a, b, true);
      racc = ru_add(racc, rad_term(a, b, S.F));
    }
  }
  // radius: the threads' upward partial sums, added upward
  if (rad) {
    for (int m = 1; m < 64; m <<= 1) racc = ru_add(racc, __shfl_xor(racc, m, 64));
    if (lane == 0) L.red_d[wave] = racc;
    __syncthreads();
    racc = 0.0;
    for (int w = 0; w < kWideThreads / 64; ++w) racc = ru_add(racc, L.red_d[w]);
  }
  if (tid == 0) {
    double rin_m = 0.0;
    int rin_e = 0;
    if (rad && racc != 0.0) {
      int ex;
      rin_m = __builtin_frexp(racc, &ex);
      rin_e = S.F + ex;
    }
    if (exact_zero) set_limb(L, 0, 0u);
    finish_entry([&](int q) { return limb(L, q); }, nW, lo, R, oidx, p, prm->approx, rin_m, rin_e);
    if (R.status) R.status[oidx] = status;
  }
}

__global__ __launch_bounds__(kWideThreads) void wide_dot_kernel(DotParams prm) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  wide_dot(&prm, *reinterpret_cast<WideLds *>(smem));
}

__global__ __launch_bounds__(kWideThreads) void wide_dot_batch_kernel(const DotParams *tasks, const int32_t *order) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const ARB_GLOBAL DotParams *prm = gp(tasks) + gp(order)[blockIdx.x];
  wide_dot(prm, *reinterpret_cast<WideLds *>(smem));
}

}  // namespace

// Half the window: an exact fallback over operands of p bits spans about 2p
// bits below the top of the sum.
int wide_max_precision() { return 32 * (kWideCols / 2) - 2 * kWideGuard; }

int wide_max_limbs() { return kWideOpLimbs; }

hipError_t launch_wide_dot(const DotParams &prm, hipStream_t s) {
  hipLaunchKernelGGL(wide_dot_kernel, dim3(1), dim3(kWideThreads), sizeof(WideLds), s, prm);
  return hipGetLastError();
}

const void *wide_dot_batch_kernel_ptr(size_t *lds_bytes) {
  *lds_bytes = sizeof(WideLds);
  return reinterpret_cast<const void *>(&wide_dot_batch_kernel);
}

hipError_t launch_wide_dot_batch(const DotParams *tasks, const int32_t *order, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(wide_dot_batch_kernel, dim3((unsigned)count), dim3(kWideThreads), sizeof(WideLds), s, tasks,
                     order);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
