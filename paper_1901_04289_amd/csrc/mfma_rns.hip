// Residue form of the exact block product on INT8 MFMA: for every prime
// p_j and product q, the residue modulo p_j of each entry of the integer
// matrix product A_q B_q (the multimodular integer product of Section 4's
// introduction, Johansson 2019), reduced on chip.
//
// A residue r = lo + 256 hi (balanced, |r| < 2^14) is held as two int8
// digit planes, so r_A r_B = 65536 hi hi' + 256 (lo hi' + hi lo') + lo lo'.
// One work item runs the four digit-plane pairs of one prime in that
// order and folds them by Horner's rule inside its accumulators: after the
// hi hi' pair and after the two cross pairs, every accumulator x is
// replaced by 256 (x mod p_j), with x mod p_j taken loosely in [-p_j,
// 2 p_j); the last pair leaves x = r_A r_B (mod p_j) below 2^30 in
// magnitude, stored as one int16 residue in [-p_j, p_j).  Against three
// int32 partial planes per prime this writes a sixth of the bytes and
// keeps the reduction off the reconstruction's plane reads.
#include "sliced.hpp"

namespace arbgpu_impl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

__device__ __forceinline__ int swz(int row, int chunk) { return row * kKStep + ((chunk ^ ((row >> 1) & 7)) << 4); }

// x - q p_j with q = floor(x mu_j / 2^32), mu_j = floor(2^32 / p_j): for
// |x| < 2^31 the estimate q is within one of floor(x / p_j) on either
// side, so the result lies in [-p_j, 2 p_j).
__device__ __forceinline__ int32_t loose_mod(int32_t x, int32_t p, int32_t mu) {
  const int32_t q = __mulhi(x, mu);
  return x - __mul24(q, p);
}

}  // namespace

// Workgroup: 256 threads, output tile TM x TM (256 or 128); wave w owns
// the quarter (w / 2, w % 2) of WT = TM / 2 rows and columns as NB x NB
// blocks of v_mfma_i32_32x32x32_i8 (lane l, register r: column l % 32,
// row 8 (r / 4) + 4 (l / 32) + r % 4).  The inner loop runs over (digit
// pair, 128-byte K step) with A and B tiles staged through LDS, double
// buffered, 16-byte chunks XOR-swizzled by (row >> 1) & 7, the next step's
// global loads spread over the current step's MFMAs.  The 128 tile keeps
// small products from paying for a mostly empty 256 tile.
template <int TM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, TM == 256 ? 1 : 2))) void mfma_rns_kernel(
    MfmaRnsParams P) {
  constexpr int WT = TM / 2, NB = WT / 32, U = TM / 32;
  __shared__ __attribute__((aligned(16))) uint8_t lds[2][2][TM * kKStep];  // [buf][A/B]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int ntiles = P.ntm * P.ntn;
  // Workgroups go to the 8 XCDs round-robin by id.  Work item (group,
  // tile) for XCD x = id % 8, slot = id / 8: groups x, x + 8, ..., the
  // tiles of one group in order, so that the workgroups resident on one
  // XCD share A row blocks and B column blocks in its L2.  Group g is
  // prime g % mpad of product g / mpad (mpad: m rounded up to 8).
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int g = xcd + 8 * (slot / ntiles);
  const int t = slot % ntiles;
  const int q = g / P.mpad, j = g - q * P.mpad;
  if (j >= P.m) return;   // padding prime
  const int32_t pj = P.prime[j], muj = (int32_t)P.mu[j], m256p = -256 * pj;
  const int tm = t / P.ntn, tn = t - tm * P.ntn;
  const int ksteps = (int)(P.Kp / kKStep);
  const int nsteps = 4 * ksteps;
  const int64_t planeA = P.Mp * P.Kp, planeB = P.Np * P.Kp;

  v16i acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int jj = 0; jj < NB; ++jj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][jj][r] = 0;

  // global -> register staging: thread covers chunk (tid & 7) of rows
  // (tid >> 3) + 32 u, u < U, for A and for B (a scalar base per step plus
  // a 32-bit lane offset; TM rows of K_pad bytes stay below 2^31)
  const int srow = tid >> 3, schunk = tid & 7;
  const char *tileA = reinterpret_cast<const char *>(P.A[q]) + (int64_t)2 * j * planeA + (int64_t)tm * TM * P.Kp;
  const char *tileB = reinterpret_cast<const char *>(P.B[q]) + (int64_t)2 * j * planeB + (int64_t)tn * TM * P.Kp;
  const uint32_t goff = (uint32_t)srow * (uint32_t)P.Kp + (uint32_t)schunk * 16u;
  const uint32_t rowstep = 32u * (uint32_t)P.Kp;
  v4i stA[U], stB[U];
  // pair pr: 0 (hi, hi'), 1 (lo, hi'), 2 (hi, lo'), 3 (lo, lo'); plane 0
  // of a prime is its low digit, plane 1 its high digit
  auto gload = [&](v4i (&sa)[U], v4i (&sb)[U], int pr, int ks) {
    const int a = (pr == 0 || pr == 2) ? 1 : 0;
    const int b = pr < 2 ? 1 : 0;
    const char *pa = tileA + a * planeA + ks * kKStep;
    const char *pb = tileB + b * planeB + ks * kKStep;
    // the lane offset is opaque here, so the compiler keeps a scalar base
    // per step and the 32-bit offset instead of 64-bit lane addresses
    // hoisted out of the loop (which spilled)
    uint32_t go = goff;
    asm volatile("" : "+v"(go));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      sa[u] = *reinterpret_cast<const v4i *>(pa + (go + u * rowstep));
      sb[u] = *reinterpret_cast<const v4i *>(pb + (go + u * rowstep));
    }
  };
  auto lstore = [&](const v4i (&sa)[U], const v4i (&sb)[U], int buf) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int row = srow + 32 * u;
      *reinterpret_cast<v4i *>(&lds[buf][0][swz(row, schunk)]) = sa[u];
      *reinterpret_cast<v4i *>(&lds[buf][1][swz(row, schunk)]) = sb[u];
    }
  };
  int offA[4], offB[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int chunk = kk * 2 + (lane >> 5);
    offA[kk] = swz(wm * WT + (lane & 31), chunk);
    offB[kk] = swz(wn * WT + (lane & 31), chunk);
  }

  gload(stA, stB, 0, 0);
  lstore(stA, stB, 0);
  __syncthreads();
  // one pipeline step: MFMAs on buffer step & 1 while the next step's
  // tiles load
  auto run_step = [&](int step) __attribute__((always_inline)) {
    const int buf = step & 1;
    const int nstep = step + 1 < nsteps ? step + 1 : step;
    // branch-free: on the last step the prefetch re-reads the current step
    // (a valid address) and the store fills the idle buffer
    const int npr = nstep / ksteps;
    gload(stA, stB, npr, nstep - npr * ksteps);
    const uint8_t *la = lds[buf][0];
    const uint8_t *lb = lds[buf][1];
    v4i fa[2][NB], fb[2][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      fa[0][i] = *reinterpret_cast<const v4i *>(la + offA[0] + i * 32 * kKStep);
      fb[0][i] = *reinterpret_cast<const v4i *>(lb + offB[0] + i * 32 * kKStep);
    }
#pragma unroll
    for (int kk = 0; kk < kKStep / 32; ++kk) {
      const int cur = kk & 1, nxt = cur ^ 1;
      if (kk + 1 < kKStep / 32) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          fa[nxt][i] = *reinterpret_cast<const v4i *>(la + offA[kk + 1] + i * 32 * kKStep);
          fb[nxt][i] = *reinterpret_cast<const v4i *>(lb + offB[kk + 1] + i * 32 * kKStep);
        }
      }
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int jj = 0; jj < NB; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[cur][i], fb[cur][jj], acc[i][jj], 0, 0, 0);
    }
    lstore(stA, stB, buf ^ 1);
    // instruction order (masks: 0x008 MFMA, 0x020 VMEM read, 0x100 DS
    // read, 0x200 DS write): a quarter of the next step's global loads and
    // the first slice's fragments first, then each slice's MFMAs in pairs
    // with the next slice's fragment reads and the other loads between
    // them, the LDS stores over the last slice
    constexpr int MF = NB * NB, GL = 2 * U, SL = 3 * MF / 2, FR = 2 * NB / (MF / 2);
    __builtin_amdgcn_sched_group_barrier(0x020, GL / 4, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 2 * NB, 0);
#pragma unroll
    for (int kk = 0; kk < kKStep / 32 - 1; ++kk) {
#pragma unroll
      for (int u = 0; u < MF / 2; ++u) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, FR, 0);
        const int sl = kk * (MF / 2) + u;   // SL slots carry the other 3 GL / 4 loads
        const int nl = (sl + 1) * (3 * GL / 4) / SL - sl * (3 * GL / 4) / SL;
#pragma unroll
        for (int x = 0; x < nl; ++x) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < MF; ++u) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x200, GL / MF > 0 ? GL / MF : 1, 0);
    }
    __syncthreads();
  };
  // Horner's rule after the hi hi' pair and after the cross pairs: the
  // accumulators become 256 (x mod p_j), below 2^24 in magnitude; the
  // next pairs add at most 2 K_pad 2^13 < 2^30 - 2^24 (K_pad < 2^16)
  auto horner = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          // on the accumulation register itself, through two vector
          // temporaries: left to the compiler, all the accumulators were
          // moved to vector registers together and spilled
          // 256 x - q (256 p_j) in one 24-bit multiply-add: |q| < 2^17 and
          // 256 p_j < 2^23 fit its signed 24-bit factors, and the result,
          // 256 (x - q p_j), is below 2^24 in magnitude, so its value mod
          // 2^32 is exact
          int32_t acv = acc[i][jj][r], t0, t1;
          asm volatile(
              "v_accvgpr_read_b32 %1, %0\n\t"
              "v_mul_hi_i32 %2, %1, %3\n\t"
              "v_lshlrev_b32 %1, 8, %1\n\t"
              "v_mad_i32_i24 %1, %2, %4, %1\n\t"
              "v_accvgpr_write_b32 %0, %1"
              : "+a"(acv), "=&v"(t0), "=&v"(t1)
              : "s"(muj), "s"(m256p));
          acc[i][jj][r] = acv;
        }
        // one block of 16 registers at a time
        __builtin_amdgcn_sched_barrier(0);
      }
  };
  for (int step = 0; step < nsteps; ++step) {
    run_step(step);
    if (step + 1 == ksteps || step + 1 == 3 * ksteps) horner();
  }

  // epilogue: x mod p_j in [-p_j, p_j) as int16 into plane (q, j).  The
  // accumulators go through LDS (free after the last step's barrier; each
  // wave uses its own part), one block row of 32 x WT at a time, so that
  // every lane then reduces 8 consecutive entries of a row and writes them
  // as one 16-byte store.  Row stride WT + 8 words: the two lane halves of
  // an accumulator write (rows 4 apart) fall in different bank halves.
  constexpr int RS = WT + 8, LPR = WT / 8, RP = 64 / LPR;
  const int64_t r0 = (int64_t)tm * TM + wm * WT, c0 = (int64_t)tn * TM + wn * WT;
  int16_t *Y = P.Y + ((int64_t)q * P.m + j) * P.ds;
  int32_t *wl = reinterpret_cast<int32_t *>(&lds[0][0][0]) + wave * (32 * RS);
  const int rows_in = (int)min<int64_t>(P.M - r0, WT), cols_in = (int)min<int64_t>(P.N - c0, WT);
  const bool vec = (P.N & 7) == 0;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int jj = 0; jj < NB; ++jj)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        wl[((r >> 2) * 8 + 4 * (lane >> 5) + (r & 3)) * RS + jj * 32 + (lane & 31)] = acc[i][jj][r];
    __syncthreads();
#pragma unroll 2
    for (int c = 0; c < 32 / RP; ++c) {
      const int rr = lane / LPR + RP * c, cc = (lane % LPR) * 8;   // row in the block, first column
      const v4i x0 = *reinterpret_cast<const v4i *>(wl + rr * RS + cc);
      const v4i x1 = *reinterpret_cast<const v4i *>(wl + rr * RS + cc + 4);
      uint32_t w[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t lo = (u < 2) ? x0[2 * u] : x1[2 * u - 4], hi = (u < 2) ? x0[2 * u + 1] : x1[2 * u - 3];
        int32_t a = loose_mod(lo, pj, muj), b = loose_mod(hi, pj, muj);
        a = a >= pj ? a - pj : a;
        b = b >= pj ? b - pj : b;
        w[u] = ((uint32_t)a & 0xFFFFu) | ((uint32_t)b << 16);
      }
      const int row = i * 32 + rr;
      if (row < rows_in) {
        int16_t *dst = Y + (r0 + row) * P.N + c0 + cc;
        if (vec && cc + 8 <= cols_in) {
          *reinterpret_cast<uint4 *>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (cc + u < cols_in) dst[u] = (int16_t)(w[u >> 1] >> (16 * (u & 1)));
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_mfma_rns(const MfmaRnsParams &P, hipStream_t s) {
  if ((P.tile != 256 && P.tile != 128) || P.Mp % P.tile != 0 || P.Np % P.tile != 0 || P.ntm * P.tile != P.Mp ||
      P.ntn * P.tile != P.Np || P.mpad % 8 != 0 || P.m > P.mpad || P.nprod < 1 || P.nprod > 4 ||
      P.N >= ((int64_t)1 << 22) || P.Kp >= ((int64_t)1 << 16) || P.Kp < kKStep || P.Kp % kKStep != 0)
    return hipErrorInvalidValue;
  const int64_t n = (int64_t)P.nprod * P.mpad * P.ntm * P.ntn;
  if (n == 0) return hipSuccess;
  if (P.tile == 256) hipLaunchKernelGGL(mfma_rns_kernel<256>, dim3((unsigned)n), dim3(256), 0, s, P);
  else hipLaunchKernelGGL(mfma_rns_kernel<128>, dim3((unsigned)n), dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
