/*
 * arbgpu — arbitrary-precision ball dot products and matrix products on
 * AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Johansson 2019, Section 2 and Section 3): given balls
 * x_i = [m_i +- r_i], y_i = [m'_i +- r'_i], an optional initial ball and a
 * sub flag, compute a ball [m +- r] containing
 *     initial + (-1)^sub * sum_{i<N} x_i y_i
 * at output precision p >= 2, operands at mixed precisions.  This library
 * fixes the midpoint to be the *exact* sum truncated toward zero to p bits
 * (a refinement of the paper's error of order 2^-p sum|x_i y_i|; the paper
 * falls back to a slower exact summation when its fast sum cannot decide,
 * Section 2), and the radius to an upper bound of
 *     [inexact] 2^(e_m - p) + r_initial + sum_i (|m_i| r'_i + |m'_i| r_i + r_i r'_i)
 * that is tight to within a relative 2^-20.  Matrix products (Section 4)
 * give every entry exactly the dot product of its row and column.
 *
 * Memory: every pointer in the structs below is DEVICE memory owned by the
 * caller (for instance torch tensors).  The library never frees or keeps
 * them; inputs must stay valid until the work completes on the stream.
 * Calls are asynchronous on the given HIP stream; return codes report
 * host-side validation and launch errors only.  Per-element outcomes are
 * written to the output's status bytes.
 *
 * Number format (eq. (1) with 32-bit limbs), element idx of an array:
 *   nls[idx]  bits 0..30: limb count n (0 means the value is zero),
 *             bit 31: sign;
 *   exp[idx]  exponent e with 2^(e-1) <= |m| < 2^e, |e| < 2^28;
 *   limbs[k*ld + idx], k = 0..n-1, most significant limb first; the top
 *             limb has its top bit set; value = (-1)^sign *
 *             sum_k limbs[k*ld+idx] * 2^(e - 32(k+1)).  k < cap.
 *   rad_m[idx], rad_e[idx]: radius rad_m * 2^rad_e with rad_m in [0.5, 1)
 *             or 0 (finite); both pointers NULL for exact arrays.
 */
#ifndef ARBGPU_H
#define ARBGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define ARBGPU_OK        0   /* done (or enqueued, for stream calls)           */
#define ARBGPU_NOTREADY  1   /* arbgpu_poll: the ticket has not completed      */
#define ARBGPU_EINVAL   -1   /* bad argument: p < 2, shape, stride, cap, NULL  */
#define ARBGPU_ERANGE   -2   /* an exponent |e| >= 2^28 reached the host check */
#define ARBGPU_ENOMEM   -3   /* workspace allocation failed                    */
#define ARBGPU_EAGAIN   -4   /* arbgpu_submit: over the HBM budget, try later  */
#define ARBGPU_EDEVICE  -5   /* HIP error; text in arbgpu_last_error           */

/* Flags. */
#define ARBGPU_APPROX       0x01u /* midpoints only; radius outputs untouched   */
#define ARBGPU_COMPLEX      0x02u /* rectangular complex balls: re and im parts */
#define ARBGPU_REDUCE_PREC  0x04u /* radius-driven precision cut (Section 3.3,
                                     step 7(a)): p' = max(2, min(p,
                                     e_max - e_rad + 30)); changes the midpoint */
#define ARBGPU_ALGO_LIMB    0x10u /* matmul and dot: force the limb-window
                                     kernels (dots: no digit product)      */
#define ARBGPU_ALGO_SLICED  0x20u /* matmul: force the scaled-integer INT8 path
                                     with base-256 digit slices               */
#define ARBGPU_ALGO_RNS     0x40u /* matmul: force the scaled-integer INT8 path
                                     with residues modulo primes < 2^15
                                     (multimodular, Section 4)             */
#define ARBGPU_COMPLEX_4M   0x80u /* complex matmul on the residue path: four
                                     real block products AC, BD, AD, BC
                                     instead of the three of eq. (2)
                                     (Section 3.6, Section 4.3), AC, BD and
                                     (A+B)(C+D); both are exact, so no
                                     output bit changes                    */

/* Per-element status bytes. */
#define ARBGPU_ST_OK       0   /* result written                                 */
#define ARBGPU_ST_REFINED  1   /* result written; the fast window could not
                                  decide the truncation and the exact refinement
                                  passes were used                               */
#define ARBGPU_ST_ERANGE   2   /* an input exponent had |e| >= 2^28 or a radius
                                  was not finite, or (dots beyond the register
                                  windows) the exact fallback's exponent span
                                  exceeded the LDS window; the output value is
                                  undefined and its radius infinite              */

typedef struct arbgpu_ctx arbgpu_ctx;
typedef void *arbgpu_stream;   /* a hipStream_t; NULL is the null stream */

typedef struct {
  const uint32_t *limbs;   /* [cap][ld] limb planes                          */
  int64_t ld;              /* distance between limb planes, in elements      */
  int32_t cap;             /* number of limb planes (max n)                  */
  const int32_t *exp;
  const int32_t *nls;
  const double *rad_m;     /* NULL: exact                                    */
  const int32_t *rad_e;    /* NULL iff rad_m is NULL                         */
} arbgpu_arr;

typedef struct {
  uint32_t *limbs;         /* [cap][ld]; needs cap >= ceil(p/32)             */
  int64_t ld;
  int32_t cap;
  int32_t *exp;
  int32_t *nls;
  double *rad_m;           /* may be NULL only with ARBGPU_APPROX            */
  int32_t *rad_e;
  uint8_t *status;         /* may be NULL                                    */
} arbgpu_out;

/* A matrix view: element (i, j) is element off + i*rs + j*cs of the array
 * (strides may be negative).  `im` is read only with ARBGPU_COMPLEX. */
typedef struct {
  arbgpu_arr re, im;
  int64_t rows, cols, off, rs, cs;
} arbgpu_mat;

typedef struct {
  arbgpu_out re, im;
  int64_t rows, cols, off, rs, cs;
} arbgpu_omat;

/* Create a context on HIP device `device`.  `hbm_budget_bytes` bounds the
 * workspace the context may hold and the footprint arbgpu_submit admits
 * (0 = 3/4 of the device's free memory).  `tune_cache` (nullable) names a
 * JSON file of autotuned launch parameters.  device = -1 makes a host-only
 * context that validates arguments and plans but launches nothing (every
 * compute call then returns ARBGPU_EDEVICE).  Returns ARBGPU_OK, EINVAL,
 * EDEVICE. */
int arbgpu_init(arbgpu_ctx **ctx, int device, size_t hbm_budget_bytes,
                const char *tune_cache);

/* Free the context and its workspace (after synchronizing its device). */
void arbgpu_destroy(arbgpu_ctx *ctx);

/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *arbgpu_last_error(const arbgpu_ctx *ctx);

/* Dot product (Section 3, the arb_dot / acb_dot problem statement):
 *   res[res_idx] = initial[init_idx] + (-1)^sub sum_{i<N} x[xoff+i*xstep] * y[yoff+i*ystep]
 * `initial` may be NULL.  Strides may be negative or zero.  With
 * ARBGPU_COMPLEX, `res`, `initial`, `x`, `y` each point to TWO structs
 * {real part, imaginary part} and the real and imaginary results are each
 * the exact sum of their 2N real terms, rounded once (Section 3.6).
 * A dot without an initial value, of 1 to 65536 terms, whose p plus the
 * term count's bit length plus 24 guard bits (plus 40 for a complex dot)
 * fits 1120 bits runs first as one exact INT8 MFMA product of its
 * operands' 7-bit digits (the scaled-integer product of Section 4 for a
 * 1 x N by N x 1 product); the part whose truncation that window cannot
 * certify, or a dot whose exponents spread beyond it, then runs on the
 * limb kernels (same output bits; ARBGPU_ALGO_LIMB skips the digit
 * product).  Precisions whose window (p + bitlength(t + 1) + 41 bits with
 * t = N + 1 terms, 2N + 1 for complex) fits the widest compiled register
 * window (38 limbs, 1216 bits) run one wave per output; larger ones run
 * one workgroup per output with the window in LDS, up to p = 65408 with
 * operands of at most 2048 limbs.  There an exact fallback whose span from
 * the top of the sum down to the lowest bit of any product exceeds 131072
 * bits is not run: the output gets status ARBGPU_ST_ERANGE and an infinite
 * radius.
 * EINVAL: p < 2, N < 0, NULL operand, cap of res < ceil(p/32), radius
 * output NULL without APPROX, p above 65408, or operands wider than 2048
 * limbs where the register windows do not hold p. */
int arbgpu_dot(arbgpu_ctx *ctx, const arbgpu_out *res, int64_t res_idx,
               const arbgpu_arr *initial, int64_t init_idx, int sub,
               const arbgpu_arr *x, int64_t xoff, int64_t xstep,
               const arbgpu_arr *y, int64_t yoff, int64_t ystep,
               int64_t N, int64_t p, uint32_t flags, arbgpu_stream stream);

/* Matrix product C = A B (Section 4): A is rows x inner, B is inner x cols,
 * C is rows x cols; every entry equals arbgpu_dot of its row and column.
 * ALGO flags choose the limb-window kernel (Algorithm 1 per entry) or the
 * scaled-integer block product on INT8 MFMA (Algorithm 2) with base-256
 * slices or with residues modulo small primes; none changes a single
 * output bit.  EINVAL on shape mismatch, p < 2, output cap too
 * small, NULL pointers, or when the chosen (or, without an ALGO flag,
 * every) path cannot hold the operands: the limb kernel's window as for
 * arbgpu_dot; base-256 slices up to integer heights of 4094 bits per
 * block; residues up to heights of about 4060 bits (127 words of four
 * base-256 digits, so that the residue sums stay below 2^30) while the
 * exact block values fit the reconstruction's LDS rows (about 8000 bits). */
int arbgpu_mat_mul(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A,
                   const arbgpu_mat *B, int64_t p, uint32_t flags,
                   arbgpu_stream stream);

/* The exact integer block product of Algorithm 2 (Section 4.1) with the
 * whole inner range taken as one block, midpoints only (radii are not
 * read): with v_i the lowest set-bit position over the nonzero entries of
 * row i of A and w_j that of column j of B (both parts together with
 * ARBGPU_COMPLEX; 0 for a line without nonzero entries), the scaled
 * integers a_ik 2^-v_i and b_kj 2^-w_j, and
 *     T_ij = sum_k (a_ik 2^-v_i)(b_kj 2^-w_j),  so  (A B)_ij = T_ij 2^(v_i + w_j)
 * (the paper's E_s = diag(2^e_i) is e_i = -v_i).  Complex: T_re from
 * Re(A)Re(B) - Im(A)Im(B) and T_im from Re(A)Im(B) + Im(A)Re(B).  Writes
 * T as capT two's-complement 32-bit limbs, least significant first, limb
 * k of entry (i, j) at T_re[k*ldT + i*cols + j] (and T_im with
 * ARBGPU_COMPLEX; T_im is not read otherwise), and v, w to row_v2[rows],
 * col_v2[cols]; all DEVICE memory owned by the caller.  Flags: COMPLEX,
 * ALGO_SLICED or ALGO_RNS (neither: the automatic choice), COMPLEX_4M.
 * A debugging and verification entry point of the INT8 path; it
 * synchronizes `stream` once to read the line statistics.  EINVAL: NULL
 * pointers, shape mismatch, ldT < rows*cols, an integer height above the
 * chosen form's limit, or capT below the limbs T needs (the needed count
 * is in arbgpu_last_error); ERANGE: an exponent outside (-2^28, 2^28). */
int arbgpu_mat_mul_exact_t(arbgpu_ctx *ctx, uint32_t *T_re, uint32_t *T_im, int64_t ldT,
                           int32_t capT, int32_t *row_v2, int32_t *col_v2,
                           const arbgpu_mat *A, const arbgpu_mat *B, uint32_t flags,
                           arbgpu_stream stream);

/* For callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * product of arbgpu_mat_mul, with the same arguments, results and errors,
 * whose workspace is cut from one static 256 MiB device array instead of
 * the context's buffers; it calls no device allocation or free.  Products
 * whose footprint (arbgpu_mat_mul_footprint) exceeds 256 MiB are rejected
 * with EINVAL before any work; a product that splits into several blocks
 * fails with ENOMEM when its exact block values do not fit what is left.
 * Each device holds its own copy of the array until the process ends, and
 * every call on a device shares it: calls that overlap on one device
 * (other streams, threads or contexts) race.  It keeps the last call's
 * contents; each call sets up what it reads.  Not for device -1. */
int arbgpu_mat_mul_noalloc(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A,
                           const arbgpu_mat *B, int64_t p, uint32_t flags,
                           arbgpu_stream stream);

/* Workspace.  Each context keeps device workspace buffers that grow to
 * the largest call made so far (never beyond its HBM budget) and are
 * reused by later calls; growing one waits for the work the context has
 * enqueued (on every stream it used), not for the whole device.
 * arbgpu_reserve grows them ahead of time to what a matrix product of the
 * given shape, precision and flags can take (an upper bound over the limb
 * kernel and both INT8 forms when its inner range is one block; a product
 * that splits into several blocks also holds its exact block values), so
 * that calls on shapes within it allocate no device memory.  Reads only
 * the shapes, caps and radius pointers of A and B.  EINVAL on bad
 * arguments, ENOMEM over the budget, EDEVICE on a host-only context. */
int arbgpu_reserve(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B,
                   int64_t p, uint32_t flags);
/* Workspace bookkeeping of the context and its request loop's slots:
 * *allocs = device allocations made so far (workspace growth and batch
 * creation; a warmed call sequence that allocates nothing leaves it
 * unchanged), *bytes = workspace bytes held now.  Either pointer may be
 * NULL.  EINVAL on a NULL context. */
int arbgpu_workspace_info(arbgpu_ctx *ctx, int64_t *allocs, int64_t *bytes);
/* The footprint arbgpu_submit admits a matrix product with: the sum over
 * the workspace buffers of what arbgpu_reserve would grow them to, written
 * to *bytes.  Host-only contexts may call it.  EINVAL on bad arguments. */
int arbgpu_mat_mul_footprint(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B,
                             int64_t p, uint32_t flags, size_t *bytes);

/* Autotuner of the matrix product's path.  Runs the product C = A B (the
 * arguments of arbgpu_mat_mul, no ALGO flag) on every applicable path --
 * the limb kernel (unless its work is far beyond the INT8 path's), base-256
 * slices, and residues on 256 x 256 and on 128 x 128 MFMA tiles -- once
 * untimed and twice between HIP events on `stream`, and records the
 * fastest for the product's class in the context's tune table (saved to
 * the tune-cache file when the context has one): real or complex, balls or
 * midpoints, and the ceiling base-2 logarithms of max(rows, cols), of the
 * inner length and of p.  Later arbgpu_mat_mul calls without an ALGO flag
 * take the recorded path for their class (results are the same on every
 * path).  Writes the choice (1 limb, 2 slices, 3 residues/256, 4
 * residues/128) to *choice when not NULL.  Overwrites C; synchronizes
 * `stream`.  EINVAL on bad arguments or an ALGO flag. */
int arbgpu_tune_mat_mul(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A,
                        const arbgpu_mat *B, int64_t p, uint32_t flags,
                        arbgpu_stream stream, int32_t *choice);

/* Block partition of Algorithm 2 (Section 4.1) for the product A B at
 * precision p: the inner index range is cut greedily, from index 0 upward,
 * into ranges over which every row of A and every column of B keeps integer
 * height (highest exponent minus lowest set bit over its nonzero entries,
 * both parts together with ARBGPU_COMPLEX) at most
 * floor(1.25 min(p, max(p_A, p_B)) + 192), p_M being the largest number of
 * significant bits of an entry of M.  A range shorter than 30 indices is
 * extended to min(30, remaining) and marked as a basecase chunk (evaluated
 * with dot products).  Writes min(*nblocks, max_blocks) pairs
 * (bounds[2i], bounds[2i+1]) = (k0, k1) and kinds[i] (0 block, 1 basecase)
 * to HOST arrays and the total count to *nblocks; synchronizes `stream`.
 * Only ARBGPU_COMPLEX is accepted in flags.  EINVAL on NULL pointers, shape
 * mismatch, p < 2, an exponent outside (-2^28, 2^28). */
int arbgpu_plan_blocks(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B,
                       int64_t p, uint32_t flags, int64_t *bounds, int32_t *kinds,
                       int64_t max_blocks, int64_t *nblocks, arbgpu_stream stream);

/* One dot product of a batch: the arguments of arbgpu_dot by value.
 * Complex jobs (ARBGPU_COMPLEX in flags) use both entries of res, init, x
 * and y as {real part, imaginary part}; real jobs use entry 0 only.
 * init[0].limbs == NULL means no initial value.  flags: APPROX, COMPLEX,
 * REDUCE_PREC. */
typedef struct {
  arbgpu_out res[2];
  int64_t res_idx;
  arbgpu_arr init[2];
  int64_t init_idx;
  arbgpu_arr x[2], y[2];
  int64_t xoff, xstep, yoff, ystep, N, p;
  uint32_t flags;
  int32_t sub;
} arbgpu_dot_job;

/* A resident batch of dot products (the persistent batched launch): the
 * jobs are validated, grouped by kernel (digit-product jobs by digit block
 * count, real or complex; the others by limb-kernel shape: window and
 * operand limbs, chosen from p, N and operand widths), ordered longest
 * first, copied to device memory once, and bound into one HIP graph.  Each
 * launch replays the graph on `stream`: one persistent kernel per group
 * whose workgroups or waves take jobs from a device work counter until the
 * queue is empty, then, per limb shape, the limb kernel over the parts the
 * digit products handed back (a list the device fills).  A job gives the
 * same bits as arbgpu_dot.  The operand and output arrays the jobs name
 * must stay valid while the batch is launched.  Waves per compute unit per
 * group come from the context's tune table (arbgpu_batch_tune), else a
 * default.
 * create: EINVAL on a bad job (its index in the message), ENOMEM, EDEVICE.
 * launch: EDEVICE on HIP errors.  destroy waits for the device. */
typedef struct arbgpu_batch arbgpu_batch;
int arbgpu_batch_create(arbgpu_ctx *ctx, const arbgpu_dot_job *jobs, int64_t njobs,
                        arbgpu_batch **batch);
int arbgpu_batch_launch(arbgpu_batch *batch, arbgpu_stream stream);
/* Autotuner: times every shape of the batch alone at 1, 2, 4, 8 and 16
 * waves per compute unit, keeps the fastest in the context's tune table
 * (written back to the context's tune_cache file when one was given), and
 * rebuilds the graph.  Synchronizes `stream`. */
int arbgpu_batch_tune(arbgpu_batch *batch, arbgpu_stream stream);
/* Writes up to n values {jobs, kernel tasks (one per output part), runs,
 * then per run (NS, NA, tasks, waves per CU, microseconds of the run alone
 * when tuned, else 0)} to out (host memory).  A digit-product run reports
 * NS = -(digit blocks) and NA = 1 (real) or 2 (complex); a fallback run
 * its limb shape and its list's capacity. */
int arbgpu_batch_info(arbgpu_batch *batch, int64_t *out, int n);
void arbgpu_batch_destroy(arbgpu_batch *batch);

/* Request loop (serving).  A job is a dot product or a matrix product over
 * device-resident operands, described by value; submit copies the
 * descriptors (never the operands), validates every job (nothing is queued
 * when one is bad; EINVAL names its index), and admits the set only if its
 * workspace footprint fits next to the work already in flight within the
 * loop's HBM budget: EAGAIN (try again after polling) when it does not fit
 * now, ENOMEM when it never can (a job larger than one slot's share of the
 * budget).  Worker slots, each with its own stream and workspace (kept
 * between requests), run the queue in order; requests on different slots
 * overlap on the device, and dot jobs found together at the head of the
 * queue run as one persistent batch launch.  Results are the same as from
 * arbgpu_dot / arbgpu_mat_mul.  Operands and outputs must stay valid until
 * the job's ticket polls as done.  The loop starts at the first submit with
 * 4 slots and half the context's budget unless configured before. */
#define ARBGPU_JOB_DOT     1
#define ARBGPU_JOB_MATMUL  2
typedef struct {
  int32_t kind;            /* ARBGPU_JOB_DOT or ARBGPU_JOB_MATMUL             */
  arbgpu_dot_job dot;      /* kind == ARBGPU_JOB_DOT                          */
  arbgpu_omat C;           /* kind == ARBGPU_JOB_MATMUL: C = A B at precision */
  arbgpu_mat A, B;         /*   p with flags, as arbgpu_mat_mul               */
  int64_t p;
  uint32_t flags;
} arbgpu_job;

/* A resident batch of dot products and matrix products (arbgpu_job
 * descriptors, the arguments of arbgpu_dot and arbgpu_mat_mul by value) in
 * the same persistent launch: a matrix product becomes tiles of 64 entries
 * of one row, each entry one lane's dot product on the limb kernel, queued
 * with the dot products of the same kernel shape (longest first), so that
 * many small products of uneven size and precision run in one graph
 * launch.  Matrix products in a batch take the limb kernel: the INT8 ALGO
 * flags and COMPLEX_4M are refused (EINVAL), as is a precision beyond the
 * kernel's window.  Launch, tune, info and destroy as for a dot batch
 * (info counts tasks plus tiles). */
int arbgpu_batch_create_mixed(arbgpu_ctx *ctx, const arbgpu_job *jobs, int64_t njobs,
                              arbgpu_batch **batch);

/* (Re)starts the loop with `slots` workers (1..16) and an HBM budget in
 * bytes for the workspace of admitted jobs (0: half the context budget).
 * EINVAL while requests are in flight. */
int arbgpu_serve_config(arbgpu_ctx *ctx, int slots, size_t budget_bytes);
/* Reserves, in every slot of the loop (starting it with the defaults when
 * needed), the workspace the largest of these jobs takes (arbgpu_reserve
 * per matrix product; a dot job reserves a full batch of dot tasks), so
 * that requests no larger allocate nothing.  Each slot holds at most the
 * loop's budget divided by the slot count.  EINVAL on a bad job, ENOMEM
 * when a slot's share is too small. */
int arbgpu_serve_reserve(arbgpu_ctx *ctx, const arbgpu_job *jobs, int64_t njobs);
/* Queues njobs jobs and writes their tickets (host array). */
int arbgpu_submit(arbgpu_ctx *ctx, const arbgpu_job *jobs, int64_t njobs, uint64_t *tickets);
/* Waits up to timeout_us (0: no wait) for a ticket: OK when its job is
 * done, NOTREADY when not yet, the job's error code when it failed (text
 * in arbgpu_last_error), EINVAL for an unknown ticket. */
int arbgpu_poll(arbgpu_ctx *ctx, uint64_t ticket, int64_t timeout_us);
/* Submit, start and completion times of a ticket in nanoseconds of a
 * monotonic host clock (start and completion 0 until they happen). */
int arbgpu_ticket_times(arbgpu_ctx *ctx, uint64_t ticket, int64_t times_ns[3]);

/* Per-kernel timing with HIP events recorded on the caller's stream around
 * each launch (for measurement; off by default).  arbgpu_timing(ctx, 1)
 * clears old records and starts recording, 0 stops.  arbgpu_timing_read
 * waits for the recorded launches of `kernel` ("mfma", "slice", "stats",
 * "recombine", "rad_gemm", "plan", "merge", "limb_mm", "limb_dot",
 * "dot_batch") and returns their total
 * milliseconds and count.  EINVAL on NULL arguments. */
int arbgpu_timing(arbgpu_ctx *ctx, int enable);
int arbgpu_timing_read(arbgpu_ctx *ctx, const char *kernel, double *ms_total,
                       int64_t *launches);

/* Shape of the last scaled-integer product run on this context: writes up
 * to n of {digit planes of A, digit planes of B, int32 partial planes,
 * diagonal groups, inner length, rows, cols, parts, primes (0 for base-256
 * slices), digit-plane pairs multiplied} to out (host memory).  All zero
 * before the first such product.  EINVAL on NULL. */
int arbgpu_plan_info(arbgpu_ctx *ctx, int64_t *out, int n);

/* Machine limits measured on the context's device, the denominators the
 * kernels' roofline fractions are read against (the published figures are
 * for a 2.4 GHz clock the chip need not hold under load).  Runs six
 * microbenchmark kernels on `stream`, each once untimed and then five times
 * between HIP events, and waits for them; takes about a second.  Writes up
 * to n of these to out (host memory):
 *   [0] dense INT8 matrix-core throughput, TOP/s (32x32x32 int8 MFMA,
 *       operands in registers, 8 independent accumulators per wave)
 *   [1] dense FP64 matrix-core throughput, TFLOP/s (16x16x4 f64 MFMA)
 *   [2] HBM copy bandwidth, GB/s counting bytes read plus bytes written
 *   [3] HBM read bandwidth, GB/s
 *   [4] vector 32x32+64 -> 64-bit integer multiply-adds (v_mad_u64_u32),
 *       G lane-operations/s
 *   [5] vector high-half 32x32 multiplies (v_mul_hi_u32), G lane-ops/s
 *   [6] mean shader clock during the INT8 probe, MHz (cycle counter over
 *       the constant-rate wall clock)
 *   [7] compute units
 * and zeros past 7.  `buf` is caller-owned device scratch of `bytes` bytes,
 * 256-byte aligned, at least 264 MiB (8 MiB of sinks and clock records plus
 * two streamed halves of a multiple of 128 MiB; give 2 GiB or more so the
 * halves exceed the on-package cache); its contents are overwritten and
 * need no initialisation.  EINVAL on NULL, misalignment or a short buffer,
 * EDEVICE on a host-only context or a HIP error.  Not for graph capture. */
int arbgpu_probe_peaks(arbgpu_ctx *ctx, void *buf, size_t bytes, arbgpu_stream stream,
                       double *out, int n);

#ifdef __cplusplus
}
#endif

#endif /* ARBGPU_H */
