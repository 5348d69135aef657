// Exact INT8-MFMA product of digit planes, summed over diagonal groups
// (the integer block product of Algorithm 2 of Johansson 2019, Section
// 4.1): for every group of (A plane, B plane) pairs, the int32 partial
// plane sum_pairs A_a B_b of one 256 x 256 output tile.  Used by both the
// base-256 slices and the residue form.
#include "sliced.hpp"

namespace arbgpu_impl {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// INT8 MFMA diagonal-group product
// ---------------------------------------------------------------------------
//
// Workgroup: 256 threads, output tile 256 x 256; wave w owns the 128 x 128
// quarter (w / 2, w % 2) as 4 x 4 blocks of v_mfma_i32_32x32x32_i8.  The
// inner loop runs over (slice pair, 128-byte K step); A and B tiles are
// staged through LDS (double buffered, 2 x 64 KiB) with the 16-byte chunk
// index XOR-swizzled by (row >> 1) & 7 so that 16 consecutive rows hit 16
// distinct bank groups.  Operand fragment of lane l: row (l % 32), inner
// bytes [16 (l / 32), +16) of a 32-byte K slice; result of lane l, register
// r: column l % 32, row 8 (r / 4) + 4 (l / 32) + r % 4.

__device__ __forceinline__ int swz(int row, int chunk) { return row * kKStep + ((chunk ^ ((row >> 1) & 7)) << 4); }

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void mfma_diag_kernel(MfmaParams P) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[2][2][kTile * kKStep];  // [buf][A/B]
  const int tid = threadIdx.x;
  // the wave index is the same across a wave: say so, so that addresses
  // built from it stay in scalar registers
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int ntiles = P.ntm * P.ntn;
  // Workgroups are handed to the 8 XCDs round-robin by id.  Work item
  // (group, tile) for XCD x = id % 8, slot = id / 8: groups x, x + 8, ...
  // (the host orders the groups so that every XCD gets a similar share),
  // tiles of one group in order, so the workgroups resident on one XCD
  // share A row blocks and B column blocks in that XCD's L2.
  const int bid = blockIdx.x;
  const int xcd = bid & 7, slot = bid >> 3;
  const int g = xcd + 8 * (slot / ntiles);
  const int t = slot % ntiles;
  const DiagGroup G = P.groups[g];
  if (G.slot < 0) return;   // padding group
  const int tm = t / P.ntn, tn = t - tm * P.ntn;
  const int ksteps = (int)(P.Kp / kKStep);
  const int nsteps = (G.a1 - G.a0) * ksteps;
  const int64_t planeA = P.Mp * P.Kp, planeB = P.Np * P.Kp;

  v16i acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

  // global -> register staging: thread covers chunk (tid & 7) of rows
  // (tid >> 3) + 32 u, u = 0..7, for A and for B; the loads for step s + 1
  // are issued at the start of step s and stored to LDS at its end.
  // (addresses: a scalar base per step plus a 32-bit lane offset; 256 rows
  // of K_pad bytes stay below 2^31 bytes)
  const int srow = tid >> 3, schunk = tid & 7;
  const char *tileA = reinterpret_cast<const char *>(P.A) + (int64_t)tm * kTile * P.Kp;
  const char *tileB = reinterpret_cast<const char *>(P.B) + (int64_t)tn * kTile * P.Kp;
  const uint32_t goff = (uint32_t)srow * (uint32_t)P.Kp + (uint32_t)schunk * 16u;
  const uint32_t rowstep = 32u * (uint32_t)P.Kp;
  v4i stA[8], stB[8];
  auto gload = [&](v4i (&sa)[8], v4i (&sb)[8], int pr, int ks) {
    const int a = G.a0 + pr;
    const int b = G.c - a;
    const char *pa = tileA + a * planeA + ks * kKStep;
    const char *pb = tileB + b * planeB + ks * kKStep;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sa[u] = *reinterpret_cast<const v4i *>(pa + (goff + u * rowstep));
      sb[u] = *reinterpret_cast<const v4i *>(pb + (goff + u * rowstep));
    }
  };
  auto lstore = [&](const v4i (&sa)[8], const v4i (&sb)[8], int buf) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = srow + 32 * u;
      *reinterpret_cast<v4i *>(&lds[buf][0][swz(row, schunk)]) = sa[u];
      *reinterpret_cast<v4i *>(&lds[buf][1][swz(row, schunk)]) = sb[u];
    }
  };
  // fragment offsets of this lane inside a 256 x 128 tile, per 32-byte K
  // slice; row block i adds i * 32 rows, which leaves the swizzle unchanged
  int offA[4], offB[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int chunk = kk * 2 + (lane >> 5);
    offA[kk] = swz(wm * 128 + (lane & 31), chunk);
    offB[kk] = swz(wn * 128 + (lane & 31), chunk);
  }

  if (nsteps > 0) {
    gload(stA, stB, 0, 0);
    lstore(stA, stB, 0);
  }
  __syncthreads();
  int pr = 0, ks = 0;
  for (int step = 0; step < nsteps; ++step) {
    const int buf = step & 1;
    int npr = pr, nks = ks + 1;
    if (nks == ksteps) { nks = 0; ++npr; }
    // The body is branch-free so that the scheduler can interleave memory
    // traffic with the MFMAs.  On the last step the prefetch re-reads the
    // current step (a valid address) and the store fills the idle buffer.
    const bool more = step + 1 < nsteps;
    gload(stA, stB, more ? npr : pr, more ? nks : ks);
    const uint8_t *la = lds[buf][0];
    const uint8_t *lb = lds[buf][1];
    v4i fa[2][4], fb[2][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      fa[0][i] = *reinterpret_cast<const v4i *>(la + offA[0] + i * 32 * kKStep);
      fb[0][i] = *reinterpret_cast<const v4i *>(lb + offB[0] + i * 32 * kKStep);
    }
#pragma unroll
    for (int kk = 0; kk < kKStep / 32; ++kk) {
      const int cur = kk & 1, nxt = cur ^ 1;
      if (kk + 1 < kKStep / 32) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          fa[nxt][i] = *reinterpret_cast<const v4i *>(la + offA[kk + 1] + i * 32 * kKStep);
          fb[nxt][i] = *reinterpret_cast<const v4i *>(lb + offB[kk + 1] + i * 32 * kKStep);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[cur][i], fb[cur][j], acc[i][j], 0, 0, 0);
    }
    lstore(stA, stB, buf ^ 1);
    // Instruction order for the scheduler (masks: 0x008 MFMA, 0x020 VMEM
    // read, 0x100 DS read, 0x200 DS write): 4 of the next step's 16 global
    // loads and the first slice's fragments first, then each slice's 16
    // MFMAs with the next slice's 8 fragment reads and the other 12 global
    // loads spread between them, and the LDS stores of the next step spread
    // over the last slice.  (All 16 loads first left the memory pipe idle
    // for most of the step: spreading them measured 2.91 -> 2.75 ms for the
    // residue form at 2048^3 and 36.2 -> 33.7 ms for base-256 slices.)
    __builtin_amdgcn_sched_group_barrier(0x020, 4, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
#pragma unroll
    for (int kk = 0; kk < kKStep / 32 - 1; ++kk) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        const int slot = kk * 8 + q;   // 24 slots carry the other 12 loads
        if ((slot + 1) * 12 / 24 > slot * 12 / 24) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
    }
    __syncthreads();
    pr = npr;
    ks = nks;
  }

  // epilogue: int32 partial plane of this diagonal group.  Addresses are a
  // wave base (the quarter's corner, scalar) plus a 32-bit byte offset: a
  // lane part and a row part that is the same for every lane (the host
  // keeps N < 2^22, so 128 rows of the plane span fewer than 2^31 bytes).
  const int64_t r0 = (int64_t)tm * kTile + wm * 128, c0 = (int64_t)tn * kTile + wn * 128;
  char *D = reinterpret_cast<char *>(P.D + (int64_t)G.slot * P.ds + r0 * P.N + c0);
  const uint32_t rowb = 4u * (uint32_t)P.N;
  const uint32_t loff = (uint32_t)(lane >> 5) * 4u * rowb + 4u * (uint32_t)(lane & 31);
  auto put = [&](uint32_t dr, int j, int32_t v) {
    *reinterpret_cast<int32_t *>(D + (loff + (dr * rowb + 128u * (uint32_t)j))) = v;
  };
  if (r0 + 128 <= P.M && c0 + 128 <= P.N) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) put(i * 32 + (r >> 2) * 8 + (r & 3), j, acc[i][j][r]);
  } else {
    // edge quarter: rows below rlim and columns below clim are inside
    const int rlim = (int)min<int64_t>(P.M - r0, 128) - (lane >> 5) * 4;
    const int clim = (int)min<int64_t>(P.N - c0, 128) - (lane & 31);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int dr = i * 32 + (r >> 2) * 8 + (r & 3);
          if (dr < rlim && j * 32 < clim) put((uint32_t)dr, j, acc[i][j][r]);
        }
  }
}

hipError_t launch_mfma(const MfmaParams &P, hipStream_t s) {
  // the group table is padded to a multiple of 8 (see the kernel's mapping)
  const int64_t n = (int64_t)P.ngroups * P.ntm * P.ntn;
  if (P.ngroups % 8 != 0 || P.N >= ((int64_t)1 << 22) || P.Kp >= ((int64_t)1 << 23)) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(mfma_diag_kernel, dim3((unsigned)n), dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace arbgpu_impl
