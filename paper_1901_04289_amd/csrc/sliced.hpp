// Scaled-integer block product on INT8 MFMA (Algorithm 2, Johansson 2019,
// Section 4): interfaces shared by the sliced kernels and the front end.
#pragma once

#include "internal.hpp"

namespace arbgpu_impl {

constexpr int kTile = 256;       // output tile edge of the MFMA kernel
constexpr int kKStep = 128;      // inner bytes per pipeline step
constexpr int kMaxSlices = 512;  // digit planes per operand (heights up to 4094 bits)

// Per-row / per-column statistics over the inner index range of a block.
struct LineStats {
  int32_t *top;    // max exponent over nonzero entries (INT32_MIN: none)
  int32_t *v2;     // min lowest-set-bit position (INT32_MAX: none)
};

struct StatsParams {
  arbgpu_arr part[2];        // operand parts (re, im)
  int nparts;
  int64_t lines, len;        // number of rows (A) / columns (B), inner length
  int64_t off, line_stride, elem_stride;
  int64_t k0;                // first inner index of the block
  LineStats out;
  int32_t *gmax;             // [0] max height, [1] max precision, [2] erange flag,
                             // [3] max |position| of a top or lowest set bit
};

// One operand of the block product, sliced into balanced base-256 digits.
struct SliceParams {
  arbgpu_arr part[2];
  int64_t lines, len;        // lines = rows of A (or columns of B); len = inner length per part
  int64_t off, line_stride, elem_stride;
  int64_t k0;
  int mode;                  // 0: real; 1: [re; -im] (inner 2 len); 2: [im; re]; 3: [re, im]
  int64_t lines_pad, k_pad;  // plane shape [L][lines_pad][k_pad]
  int L;                     // number of digit planes
  const int32_t *v2;         // scaling per line: value * 2^-v2 is an integer
  int8_t *planes;
};

// A diagonal group: slice pairs (a, c - a) for a in [a0, a1), summed into
// one int32 partial plane `slot`.
struct DiagGroup {
  int32_t c, a0, a1, slot;
};

struct MfmaParams {
  const int8_t *A;       // [LA][Mp][Kp]
  const int8_t *B;       // [LB][Np][Kp]
  int32_t *D;            // [nslots][ds]: entry (i, j) of plane s at s ds + i N + j
  const DiagGroup *groups;
  int64_t M, N, Mp, Np, Kp;
  int64_t ds;            // plane stride in entries (>= M N)
  int ntm, ntn;          // tiles along M and N
  int ngroups;
};

struct RecombParams {
  const int32_t *D;        // [nslots][ds]
  int64_t ds;              // plane stride in entries
  const int32_t *slot_of;  // [Lc + 1]: slots of diagonal c are slot_of[c] .. slot_of[c+1]-1
  int Lc;                  // number of diagonals (LA + LB - 1)
  int64_t M, N;
  uint32_t *T;             // [nT][M*N] two's complement limbs, least significant first
  int nT;
  const int32_t *rowv2, *colv2;
  arbgpu_out C;
  int64_t c_off, c_rs, c_cs;
  int p;
  int approx;
  const double *rin_m;     // propagated radius per entry (nullable)
  const int32_t *rin_e;
  // truncated diagonal set: ebits >= 0 when the diagonals below some c0
  // were left out, their sum below 2^ebits in magnitude; an entry whose
  // truncation this does not certify goes to fb_list (count fb_count) for
  // the exact per-entry product
  int ebits;
  int64_t *fb_list;
  int32_t *fb_count;
};

struct RadPrepParams {
  arbgpu_arr part[2];
  int nparts;
  int64_t lines, len, off, line_stride, elem_stride;
  int mode;                  // as in SliceParams (inner index layout)
  int side;                  // 0: A side -> (|m|, r); 1: B side -> (|m| + r, r)
  int32_t *scale0, *scale1;  // per-line exponent frames of v0 and v1
  double *v0, *v1;           // [lines][len_total] scaled upper bounds
  int32_t *tiny;             // set when a value fell too far below its frame
};

struct RadGemmParams {
  const double *a_m, *a_r;   // [M][Kt]: |A| and R_A, row-scaled
  const double *b_mr, *b_r;  // [Kt][N]: |B| + R_B and R_B, column-scaled
  const int32_t *a_s0, *a_s1, *b_s0, *b_s1;   // frames of a_m, a_r, b_mr, b_r
  const int32_t *tiny;       // nonzero: the exact kernel writes the result
  int64_t M, N, Kt;
  double *out_m;             // [M*N]
  int32_t *out_e;
  // inner dimension split over the third grid dimension: splits ranges of
  // kchunk (a multiple of 16) indices, whose two partial sums per entry go
  // to part[split][sum][M*N] and are added by rad_gemm_finish; splits = 1
  // writes the result directly (part unused)
  int splits;
  int64_t kchunk;
  double *part;
};
// Inner-dimension splits of the radius product of an M x N result over Kt
// (enough workgroups to fill the device, each split at least 64 long).
int rad_gemm_splits(int64_t M, int64_t N, int64_t Kt);

// Per-entry radius with per-entry frames (fallback of the radius product).
struct RadExactParams {
  arbgpu_arr A[2], B[2];
  int a_mode, b_mode;        // inner layouts as in SliceParams
  int64_t len, Kt, M, N;
  int64_t a_off, a_rs, a_cs, b_off, b_rs, b_cs;
  const int32_t *tiny;       // zero: nothing to do
  double *out_m;
  int32_t *out_e;
};

// Multimodular form of the block product: residues of the scaled integers
// modulo m odd primes below 2^15, each split into two balanced int8 digits
// (planes 2j: low digit, 2j + 1: high digit of prime j).
// Per-prime constants of the reconstruction's first phase in one 32-byte
// record, so that a prime's constants arrive by one scalar load.
struct RnsCrtPrime {
  uint32_t p, mu;           // the prime and floor(2^32 / p)
  int32_t cb;               // (P / p)^-1 mod p, balanced (|cb| < p / 2)
  uint32_t kp2;             // 2 p ceil(2^30 / p)
  double rp;                // 1 / p
  uint32_t half, pad;       // (p - 1) / 2
};
static_assert(sizeof(RnsCrtPrime) == 32, "one 32-byte record per prime");

struct RnsTables {
  const int32_t *prime;     // [m]
  const uint32_t *mu;       // [m] floor(2^32 / p)
  const uint32_t *kp;       // [m] p ceil(2^30 / p): makes values above -2^30 nonnegative
  // [nrt][32][kd] int8 digits (lo, hi) of the balanced 256^a mod p_j,
  // inner index a < 4 nw (zero beyond); row r of tile rt holds prime
  // 16 rt + r / 2, lo for even r and hi for odd r (column r of a 32 x 32
  // MFMA result, lane pairs then hold a prime's two sums), nrt = ceil(m / 16)
  const int8_t *wd;
  const uint32_t *c;        // [m] (P / p_j)^-1 mod p_j, P = prod p_j
  const double *rp;         // [m] 1 / p_j
  const RnsCrtPrime *crt;   // [m]
  // [ncc][32][kc] balanced base-256 digits of the reconstruction weights:
  // inner index 2j -> P / p_j, 2j + 1 -> 256 P / p_j, 2m -> P, 2m + 1 ->
  // 256 P, zero beyond; digit column 32 cc + sigma(r) in row r, sigma(r) =
  // 16 ((r / 4) % 2) + 4 (r / 8) + r % 4 (lane half h of a 32 x 32 MFMA
  // result then holds digits 16 h .. 16 h + 15 of its column in order)
  const int8_t *qd;
  int m;
  int nw;                   // words of 4 base-256 digits per element
  int kd;                   // inner length of wd: 4 nw rounded up to 32
  int kc;                   // inner length of qd: 2m + 2 rounded up to 32
  int ncc;                  // 32-digit column chunks: ceil(W / 8)
};

struct RnsSliceParams {
  arbgpu_arr part[2];
  int64_t lines, len;        // as SliceParams
  int64_t off, line_stride, elem_stride;
  int64_t k0;
  int mode;
  int64_t lines_pad, k_pad;
  int L;                     // base-256 digits of the scaled integers
  const int32_t *v2;
  RnsTables tab;
  int8_t *planes;            // [2m][lines_pad][k_pad]
  // nullable: residue planes of another operand of the same layout; when
  // set, sum receives the residues of the sum of the two operands
  const int8_t *addend;
  int8_t *sum;
};

struct RnsCrtParams {
  // residues r_j of the block products (int16 in [-p_j, p_j)): product q,
  // prime j, entry ij at Y[(q m + j) ds + ij]; the reconstructed value is
  // sum_c sgn[c] * (product src[c]) for c < nsrc (complex parts: AC - BD,
  // and AD + BC or (A + B)(C + D) - AC - BD)
  const int16_t *Y;
  int64_t ds;                // plane stride in entries
  int nsrc;
  int src[3], sgn[3];
  RnsTables tab;
  int64_t M, N;
  int W;                     // two's-complement limbs of T
  const int32_t *rowv2, *colv2;
  arbgpu_out C;
  int64_t c_off, c_rs, c_cs;
  int p;
  int approx;
  const double *rin_m;
  const int32_t *rin_e;
  uint32_t *t_out;           // nullable: the W limbs of T, limb q of entry ij at t_out[q t_ld + ij]
  int64_t t_ld;
};

// Destination of the exact block integer T (two's-complement limbs, least
// significant first, limb k of entry ij at T[q][k ld + ij], sign-extended
// to cap limbs) for output part q.
struct TSink {
  uint32_t *T[2];
  int64_t ld;
  int32_t cap;
};
// Copies n limbs per entry from src (limb k of entry ij at src[k mn + ij])
// and sign-extends them to cap limbs.
// Lowest set-bit positions per line to the caller (0 for a line with no
// nonzero entry).
hipError_t launch_v2_out(const int32_t *v2, int64_t n, int32_t *out, hipStream_t s);
hipError_t launch_t_copy(const uint32_t *src, int n, int64_t mn, uint32_t *dst, int64_t ld, int cap, hipStream_t s);

// Residues of the block products on INT8 MFMA, reduced per prime on chip
// (work item: product, prime, 256 x 256 tile).
struct MfmaRnsParams {
  const int8_t *A[4], *B[4]; // per product: digit planes [2m][Mp][Kp], [2m][Np][Kp]
  int16_t *Y;                // [nprod][m][ds]
  const int32_t *prime;      // [m]
  const uint32_t *mu;        // [m] floor(2^32 / p_j)
  int nprod, m, mpad;        // mpad: m rounded up to a multiple of 8
  int64_t M, N, Mp, Np, Kp, ds;
  int tile;                  // output tile edge: 256 or 128 (Mp, Np are multiples)
  int ntm, ntn;
};
hipError_t launch_mfma_rns(const MfmaRnsParams &P, hipStream_t s);

hipError_t launch_rns_slice(const RnsSliceParams &P, hipStream_t s);
hipError_t launch_rns_crt(const RnsCrtParams &P, hipStream_t s);
// dynamic LDS of the reconstruction kernel for ew entries per workgroup
size_t rns_crt_lds(int ew, int kc, int W);
// the same with or without the per-chunk carry words of the runs
size_t rns_crt_lds(int ew, int kc, int W, bool runs);
// its budget: 64 KiB of digit rows and limbs plus the chunk carries, at
// most 32 entries x 64 chunks x 4 bytes (a gfx950 workgroup may hold up to
// 160 KiB)
constexpr size_t kRnsCrtLds = 65536 + 8192;

// Greedy block extraction (one workgroup).
struct PlanParams {
  arbgpu_arr A[2], B[2];
  int nparts;
  int64_t M, N, inner;
  int64_t a_off, a_rs, a_cs, b_off, b_rs, b_cs;
  int hmax;                 // largest admissible integer height (floor of h)
  int basecase;             // shorter blocks become dot-product chunks
  int2 *hlA, *hlB;          // (top exponent, lowest set bit) per element: A [inner][M], B [inner][N]
  int64_t *bounds;          // [2 * max_blocks]
  int32_t *kinds;           // [max_blocks]: 0 block, 1 basecase
  int64_t max_blocks;
  int32_t *nblocks;
};

// Final per-entry sum over block results and basecase terms, rounded once.
struct MergeParams {
  arbgpu_arr T;             // exact block results, element (s, ij) at s * M * N + ij
  int nS;
  arbgpu_arr A[2], B[2];
  int64_t a_off, a_rs, a_cs, b_off, b_rs, b_cs;
  const int64_t *bk;        // inner indices of the basecase chunks
  int64_t nbk;
  CompTab ct;
  int64_t M, N;
  arbgpu_out C;
  int64_t c_off, c_rs, c_cs;
  int p;
  int approx;
  const double *rin_m;      // propagated radius per entry (nullable)
  const int32_t *rin_e;
};

// One inner-index range of the partition: kind 0 is a scaled-integer block,
// kind 1 a basecase chunk evaluated term by term; ha, hb are the largest
// row and column heights over the range.
struct BlockSpan {
  int64_t k0, k1;
  int32_t kind;
  int32_t ha, hb;
};

// Greedy partition of the inner range under the integer height bound hmax,
// with every block's line statistics (synchronizes s to read the result
// back): block b's statistics, laid out as line_stats leaves them (rtop[M],
// rv2[M], ctop[N], cv2[N], gA[4], gB[4]), start at *stats + b * stride.
int plan_blocks(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, bool cplx, int hmax, hipStream_t s,
                std::vector<BlockSpan> &out, int32_t **stats = nullptr, int64_t *stride = nullptr);

// Per-block line statistics from the planner's element table.
struct BlockStatsParams {
  const int2 *hlA, *hlB;
  int64_t M, N;
  const int64_t *bounds;    // [2 nb] (k0, k1) per block
  const int32_t *nblocks;
  int64_t max_blocks;
  int32_t *out;             // [max_blocks][stride]
  int64_t stride;
};
hipError_t launch_block_stats(const BlockStatsParams &P, hipStream_t s);

// Line-major copy (limbs, exponents, counts) of an operand block.
struct GatherParams {
  arbgpu_arr src;
  int64_t off, line_stride, elem_stride, k0;
  int64_t lines, len;
  uint32_t *limbs;          // [cap][lines * len]
  int32_t *exp, *nls;       // [lines * len]
};
hipError_t launch_gather(const GatherParams &P, hipStream_t s);

hipError_t launch_plan(const PlanParams &P, hipStream_t s);
hipError_t launch_merge(const MergeParams &P, int ns, hipStream_t s);

hipError_t launch_stats_rows(const StatsParams &P, hipStream_t s);
hipError_t launch_stats_cols(const StatsParams &P, hipStream_t s);
hipError_t launch_slice(const SliceParams &P, hipStream_t s);
hipError_t launch_mfma(const MfmaParams &P, hipStream_t s);

// Stride of the int32 partial planes: the entry count rounded up to 64,
// which keeps every plane 256-byte aligned.
inline int64_t plane_stride(int64_t mn) { return (mn + 63) / 64 * 64; }
hipError_t launch_recombine(const RecombParams &P, hipStream_t s);
hipError_t launch_rad_prep(const RadPrepParams &P, hipStream_t s);
hipError_t launch_rad_gemm(const RadGemmParams &P, hipStream_t s);
hipError_t launch_rad_exact(const RadExactParams &P, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);

}  // namespace arbgpu_impl
