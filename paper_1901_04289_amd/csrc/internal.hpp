// Internal interfaces between the C-ABI front end (api.hip) and the kernel
// translation units.  Not installed; the public interface is arbgpu.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/arbgpu.h"

namespace arbgpu_impl {
struct Server;                  // request loop (serve.hip)
void server_delete(Server *s);
}  // namespace arbgpu_impl

// Context: one device, one error string, a grow-only device workspace.
struct arbgpu_ctx {
  int device;            // -1: host-only
  size_t budget;
  std::string err;
  std::mutex mu;
  struct Buf {
    void *ptr = nullptr;
    size_t size = 0;
    bool owned = true;   // false: a view into memory the context does not free
  };
  std::vector<Buf> ws;   // indexed by workspace slot
  // device allocations the context has made (workspace growth, batches)
  int64_t allocs = 0;
  // no workspace growth: a call that needs more fails with ENOMEM
  bool ws_fixed = false;
  // carve mode: every workspace buffer of a call is cut, in request order,
  // from [bump_base, bump_base + bump_size) (memory the context does not
  // own); bump_top is the next free offset
  char *bump_base = nullptr;
  size_t bump_size = 0, bump_top = 0;
  // the context arbgpu_mat_mul_noalloc runs its calls on (carve mode over
  // the device's static scratch); created with a device context
  arbgpu_ctx *noalloc_view = nullptr;
  // streams this context has enqueued work on since the workspace last
  // grew; growth waits for them (and only them) before freeing a buffer
  std::vector<hipStream_t> streams_seen;
  // per-kernel event timing (arbgpu_timing)
  bool timing = false;
  struct TimedLaunch {
    const char *name;
    hipEvent_t start, stop;
  };
  std::vector<TimedLaunch> timed;
  // shape of the last scaled-integer product: digit planes of A and B,
  // partial planes, diagonal groups, inner length, rows, cols
  // {planes of A, planes of B, partial planes, diagonal groups, inner
  // length, rows, cols, parts, primes (0: base-256 slices), digit pairs}
  int64_t last_plan[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  // autotuned launch parameters ("dot_batch:NSxNA" -> waves per CU), and
  // the file they are loaded from and saved to (may be empty)
  std::map<std::string, int> tune;
  std::string tune_path;
  arbgpu_impl::Server *server = nullptr;   // started by the first submit
  int64_t rns_key = -1;                    // residue tables in the workspace (primes, digit words)
  // the line statistics' maxima read back through pinned memory, and the
  // event that marks their arrival (created on first use)
  int32_t *stats_host = nullptr;
  hipEvent_t ev_stats = nullptr;
  ~arbgpu_ctx();
};

namespace arbgpu_impl {

// Workspace slots (each holds one growing device buffer).
enum WsSlot {
  WS_STATS = 0, WS_PLANES_A, WS_PLANES_B, WS_PLANES_B2, WS_D, WS_T, WS_TABLES,
  WS_RAD_A, WS_RAD_B, WS_RAD_OUT, WS_PLAN, WS_BLOCKS, WS_BATCH, WS_RNS, WS_GATHER, WS_RAD_PART, WS_DOTFLAG, WS_COUNT
};

// Device buffer of at least `bytes` in workspace slot `slot` (nullptr and
// the context error set on failure).  Grows by reallocation, after the
// work this context enqueued has finished; the previous contents are not
// kept.  A fixed workspace never grows.
void *ws_get(arbgpu_ctx *ctx, int slot, size_t bytes);
// Grows every slot to at least sizes[slot] bytes (outside any call's
// work: for reservation ahead of the calls).
int ws_reserve(arbgpu_ctx *ctx, const size_t sizes[WS_COUNT]);
// Records that the current call enqueues work on s.
void ctx_use_stream(arbgpu_ctx *ctx, hipStream_t s);

int set_error(arbgpu_ctx *ctx, int code, const char *fmt, ...);

// Tune table file: a flat JSON object of string keys and integer values.
void tune_load(arbgpu_ctx *ctx);
void tune_save(arbgpu_ctx *ctx);

// Records HIP events around one kernel launch on `s` when the context's
// timing is enabled.
struct KernelTimer {
  arbgpu_ctx *ctx;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  const char *name;
  KernelTimer(arbgpu_ctx *c, const char *n, hipStream_t st) : ctx(c), s(st), name(n) {
    if (ctx && ctx->timing && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
      (void)hipEventRecord(a, s);
  }
  ~KernelTimer() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      ctx->timed.push_back({name, a, b});
    }
  }
};

// The static scratch of the allocation-free entry point (noalloc.hip):
// its size, the once-per-device lookup of its address (with the device
// current) and that address (nullptr before the lookup).
size_t noalloc_scratch_bytes();
int noalloc_setup(int device);
char *noalloc_scratch(int device);

// Matrix product after validation: the INT8 path or the limb kernel.
// Path choices of a matrix product (the autotuner's values): 0 the built-in
// rule, then the limb kernel, base-256 slices, residues on 256 or 128 tiles.
constexpr int kChoiceRule = 0, kChoiceLimb = 1, kChoiceSlices = 2, kChoiceRns256 = 3, kChoiceRns128 = 4;

// `choice` forces a path (kChoice*); kChoiceRule takes the tuned choice of
// the product's class when there is one, else the built-in rule.
int mat_mul_run(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p,
                uint32_t flags, hipStream_t s, int choice = kChoiceRule);

// Scaled-integer INT8-MFMA matrix product; returns ARBGPU_OK, an error, or
// kNotApplicable when the operands need the limb kernel (more than one
// block under the height bound, inner length below the basecase, exponent
// range errors to be flagged per element).
constexpr int kNotApplicable = 100;
int sliced_mat_mul(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B,
                   int64_t p, uint32_t flags, hipStream_t s, bool forced, int choice);
// Tune-table key of a matrix product: complex or real, balls or midpoints,
// and the ceiling base-2 logarithms of the output edge, inner length and p.
std::string mat_mul_class(const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags);

// Exact integer block product over the whole inner range (arbgpu_mat_mul_exact_t).
int exact_block_product(arbgpu_ctx *ctx, uint32_t *T_re, uint32_t *T_im, int64_t ldT, int32_t capT, int32_t *row_v2,
                        int32_t *col_v2, const arbgpu_mat *A, const arbgpu_mat *B, uint32_t flags, hipStream_t s);

// Block partition of Algorithm 2 for the product A B at precision p:
// writes up to max_blocks (k0, k1) pairs and kinds to host arrays.
int plan_partition(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags,
                   hipStream_t s, int64_t *bounds, int32_t *kinds, int64_t max_blocks, int64_t *nblocks);

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
  int reduce;               // radius-driven precision cut (Section 3.3, step 7(a))
  CompTab ct;
  int na;                   // operand limbs of the job's limb-kernel shape (its radius bound)
  int digit;                // digit-product blocks (digit_dot.hip) of the job, 0: the limb kernels
  int fb;                   // in a batch: the fallback list of the task's limb shape
};

// Window / operand-limb template choice for the limb kernels.
struct LimbShape {
  int ns;   // window limbs
  int na;   // operand limbs held in registers
};

bool limb_shape_for(int p, int64_t nterms, int cap, LimbShape *out);
// Dot products beyond every compiled window: the LDS-window kernel
// (wide.hip), one workgroup per output, up to wide_max_precision() bits.
// A LimbShape of {0, 0} stands for it.
int wide_max_precision();
int wide_max_limbs();   // operand limbs the LDS staging holds
hipError_t launch_wide_dot(const DotParams &prm, hipStream_t s);
hipError_t launch_wide_dot_batch(const DotParams *tasks, const int32_t *order, int64_t count, hipStream_t s);
// the batch kernel (arguments: tasks, order; one workgroup per listed task)
// and its dynamic LDS
const void *wide_dot_batch_kernel_ptr(size_t *lds_bytes);
template <int NS, int NA>
hipError_t launch_mm_shape(const MmParams &prm, hipStream_t s);
template <int NS, int NA>
hipError_t launch_dot_shape(const DotParams &prm, hipStream_t s, const int32_t *gate);
template <int NS, int NA>
hipError_t launch_mm_list_shape(const MmParams &prm, const int64_t *list, const int32_t *count, int64_t max_count,
                                hipStream_t s);
// Products with fewer entries than this run one wave per entry (the terms
// split over its lanes), larger ones one lane per entry.
constexpr int64_t kMmWaveEntries = 1 << 17;
// A single dot of this many real terms or more runs on a workgroup of four
// waves instead of one (same bits).
constexpr int64_t kDotBlockTerms = 1024;
hipError_t launch_limb_mm(const MmParams &prm, LimbShape sh, hipStream_t s);
// The entries listed in list[0 .. *count) (device memory, *count <=
// max_count), by index i K + j, on the limb kernel.
hipError_t launch_limb_mm_list(const MmParams &prm, LimbShape sh, const int64_t *list, const int32_t *count,
                               int64_t max_count, hipStream_t s);

// A tile of a matrix product in a batch: entries (i, j0 .. j0 + 63) of
// output part `part` (an MmParams of the batch).
struct BatchTile {
  int32_t part;
  int32_t wave;   // 1: the whole wave takes the tile's entries one by one
  int64_t i, j0;
};

// Persistent batched kernel of one shape.
struct BatchShapeParams {
  const DotParams *tasks;   // every dot task of the batch (device memory)
  const MmParams *mm;       // every matrix-product part of the batch
  const BatchTile *tiles;   // every matrix-product tile of the batch
  const int32_t *order;     // this shape's work, longest first: dot task e >= 0, tile -e - 1
  int64_t count;
  int32_t *counter;         // work counter, zero before the launch
  const int32_t *dcount;    // if set, only the first *dcount entries of `order` (a device-filled list)
};
template <int NS, int NA>
const void *dot_batch_kernel_shape(bool block);
// kernel taking (BatchShapeParams): a wave per task, or (block) a
// workgroup of four waves per dot task
const void *dot_batch_kernel(LimbShape sh, bool block = false);

// One-shot batch of dot jobs on stream s (validated here; the task list is
// staged in the context workspace; synchronizes s).
int dot_batch_run(arbgpu_ctx *ctx, const arbgpu_dot_job *jobs, int64_t njobs, hipStream_t s);

// Validates the arguments of a matrix product (EINVAL with the context
// error set on a bad argument).
int mat_mul_check(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p,
                  uint32_t flags);

// Upper bound of the workspace bytes per slot a matrix product takes when
// its inner range is one scaled-integer block (either INT8 form, unless an
// ALGO flag fixes it) or a limb-kernel product; a product that splits into
// several blocks holds its exact block values besides (WS_BLOCKS, not
// included).  mat_mul_footprint is their sum (admission by HBM footprint).
void mat_mul_ws_sizes(const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags, size_t out[]);
size_t mat_mul_footprint(const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags);
// Workspace of a one-shot dot batch of up to n tasks.
size_t dot_batch_ws(int64_t n);

// Validates one dot job and builds its kernel tasks (one per output part)
// and kernel shape; sets the context error and returns EINVAL on a bad job.
int dot_tasks(arbgpu_ctx *ctx, const arbgpu_dot_job &job, const char *who, DotParams prm[2], int *ntasks,
              LimbShape *shape);
// `gate` (device memory, may be null): the launch does nothing unless *gate
// is nonzero (a dot the digit product handed over).
hipError_t launch_limb_dot(const DotParams &prm, LimbShape sh, hipStream_t s, const int32_t *gate = nullptr);

// Dot products as one small INT8 matrix product of operand digits each
// (digit_dot.hip).  digit_blocks: the digit blocks (32 digits of 7 bits)
// per operand a job takes on that path, 0 when it stays on the limb
// kernels (initial value, length, precision, a forced path).
constexpr int kDigitMaxBlocks = 5;
int digit_blocks(const DotParams &prm, LimbShape sh);
// One job (its tasks: the real part, or the real and imaginary parts of a
// complex dot); flags[q] (device memory) receives 1 when part q must be
// redone by the limb kernel, else 0.
hipError_t launch_digit_dot(const DotParams *prm, int lb, int32_t *flags, hipStream_t s);
struct DigitBatchParams {
  const DotParams *tasks;   // every dot task of the batch
  const int32_t *order;     // this run's jobs (index of the job's first task), longest first
  int64_t count;
  int32_t *counter;         // work counter, zero before the launch
  int32_t *fb_list;         // fallback lists, list f at fb_base[f]
  const int32_t *fb_base;
  int32_t *fb_count;        // entries of each list, zero before the launch
};
// kernel taking (DigitBatchParams), one workgroup per job, and its dynamic LDS
const void *digit_dot_batch_kernel(int lb, bool cplx, size_t *lds_bytes);

}  // namespace arbgpu_impl
