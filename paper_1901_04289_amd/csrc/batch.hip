// Resident batch of dot products: validation and grouping by kernel shape,
// a device-resident task queue, one HIP graph of persistent per-shape
// kernels, and the autotuner of their launch width.
//
// Every job becomes one task per output part (Section 3.6: the real and
// imaginary parts of a complex dot are separate real dots of 2N terms).
// Tasks of one (window limbs, operand limbs) shape are ordered longest
// first, so the persistent waves that take them from the shape's work
// counter finish close together.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace arbgpu_impl;

namespace {

__global__ void batch_reset_kernel(int32_t *c, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) c[i] = 0;
}

constexpr int kDefaultWaves = 8;          // waves per compute unit
constexpr int kTuneWaves[] = {1, 2, 4, 8, 16};

std::string tune_key(LimbShape sh, bool block) {
  return "dot_batch:" + std::to_string(sh.ns) + "x" + std::to_string(sh.na) + (block ? ":w4" : "");
}

std::string tune_key_digit(int lb, bool cplx) {
  return "dot_digit:" + std::to_string(lb) + (cplx ? "c" : "r");
}

// A run: a persistent kernel over a slice of the order array.  Limb runs
// (one shape; four waves per task for long dots), digit-product runs (jobs
// of one block count, real or complex) and fallback runs (the limb kernel
// over the device-filled list of one shape's parts that a digit run handed
// back; begin and count are the list's base and capacity).
struct ShapeRun {
  LimbShape sh;
  bool block;             // long dots: four waves per task
  int64_t begin, count;   // slice of the order array
  int waves;              // per compute unit
  float tuned_ms;         // time of this run alone at `waves` (0: not tuned)
  int digit = 0;          // > 0: digit-product run with this many blocks
  bool cplx = false;      // digit run of complex jobs
  int fb = -1;            // >= 0: fallback run over list fb
};

// The work of a batch: dot tasks, matrix-product parts and their tiles,
// the runs over `order` (limb work by shape, longest first, then the digit
// jobs by block count, longest first) and the fallback lists (one per limb
// shape of a digit job's tasks).
struct BatchPlan {
  std::vector<DotParams> tasks;
  std::vector<MmParams> mm;
  std::vector<BatchTile> tiles;
  std::vector<int32_t> order;   // dot task e >= 0, tile -e - 1; digit runs: the job's first task
  std::vector<ShapeRun> runs;
  std::vector<int32_t> fb_base, fb_cap;   // per fallback list
  int64_t fb_total = 0;
};

// Validates one matrix-product job of a batch and adds its parts and
// tiles (the limb kernel, one 64-entry row segment per tile).
int plan_matmul(arbgpu_ctx *ctx, const arbgpu_job &j, const char *who, BatchPlan &bp, std::vector<LimbShape> &shape_of,
                std::vector<double> &cost) {
  if (j.flags & (ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS | ARBGPU_COMPLEX_4M))
    return set_error(ctx, ARBGPU_EINVAL, "%s: a batch runs matrix products on the limb kernel (no INT8 ALGO flag)", who);
  int rc = mat_mul_check(ctx, &j.C, &j.A, &j.B, j.p, j.flags);
  if (rc) return rc;
  const bool cplx = j.flags & ARBGPU_COMPLEX;
  const int nparts = cplx ? 2 : 1;
  int cap = std::max(j.A.re.cap, j.B.re.cap);
  if (cplx) cap = std::max(cap, std::max(j.A.im.cap, j.B.im.cap));
  LimbShape sh;
  if (!limb_shape_for((int)j.p, j.A.cols * nparts, cap, &sh))
    return set_error(ctx, ARBGPU_EINVAL, "%s: precision %lld above the limb kernel's window", who, (long long)j.p);
  const int64_t M = j.A.rows, N = j.A.cols, K = j.B.cols;
  if ((int64_t)bp.tiles.size() + M * ((K + 63) / 64) * nparts > ((int64_t)1 << 30))
    return set_error(ctx, ARBGPU_EINVAL, "%s: too many matrix tiles", who);
  const double w = (double)std::min(cap, sh.na);
  const arbgpu_out *cparts[2] = {&j.C.re, &j.C.im};
  for (int q = 0; q < nparts; ++q) {
    MmParams prm;
    memset(&prm, 0, sizeof prm);
    prm.A[0] = j.A.re;
    prm.A[1] = cplx ? j.A.im : j.A.re;
    prm.B[0] = j.B.re;
    prm.B[1] = cplx ? j.B.im : j.B.re;
    prm.C = *cparts[q];
    prm.M = M; prm.N = N; prm.K = K;
    prm.a_off = j.A.off; prm.a_rs = j.A.rs; prm.a_cs = j.A.cs;
    prm.b_off = j.B.off; prm.b_rs = j.B.rs; prm.b_cs = j.B.cs;
    prm.c_off = j.C.off; prm.c_rs = j.C.rs; prm.c_cs = j.C.cs;
    prm.p = (int)j.p;
    prm.approx = (j.flags & ARBGPU_APPROX) != 0;
    prm.ct = !cplx ? comp_real() : (q == 0 ? comp_re() : comp_im());
    const int32_t part = (int32_t)bp.mm.size();
    bp.mm.push_back(prm);
    // the tiles take each entry the way the product alone would (a wave
    // per entry below kMmWaveEntries entries, else a lane), so a product
    // gives the same bits in a batch and alone
    const int32_t wave = M * K < kMmWaveEntries ? 1 : 0;
    for (int64_t i = 0; i < M; ++i)
      for (int64_t j0 = 0; j0 < K; j0 += 64) {
        bp.tiles.push_back(BatchTile{part, wave, i, j0});
        shape_of.push_back(sh);
        // 64 entries, each a whole dot of its own lane
        cost.push_back(64.0 * (double)(N * prm.ct.ncomp + 1) * w * w);
      }
  }
  return ARBGPU_OK;
}

// Validates the jobs (dot jobs from `dots`, or dot and matrix-product jobs
// from `jobs`) and builds the batch's work; sets the context error on a
// bad job.
int plan_batch(arbgpu_ctx *ctx, const arbgpu_dot_job *dots, const arbgpu_job *jobs, int64_t njobs, const char *who,
               BatchPlan &bp) {
  // work item w < tasks: dot task w; else tile w - tasks (filled in below)
  std::vector<LimbShape> shape_dot, shape_tile;
  std::vector<double> cost_dot, cost_tile;
  std::vector<int32_t> digit_jobs;           // first task of each digit-product job
  std::vector<LimbShape> fb_shapes;          // limb shape of each fallback list
  bp = BatchPlan();
  for (int64_t i = 0; i < njobs; ++i) {
    int rc;
    if (jobs && jobs[i].kind == ARBGPU_JOB_MATMUL) {
      rc = plan_matmul(ctx, jobs[i], who, bp, shape_tile, cost_tile);
    } else if (jobs && jobs[i].kind != ARBGPU_JOB_DOT) {
      rc = set_error(ctx, ARBGPU_EINVAL, "%s: unknown job kind %d", who, jobs[i].kind);
    } else {
      const arbgpu_dot_job &dj = jobs ? jobs[i].dot : dots[i];
      DotParams prm[2];
      int nt = 0;
      LimbShape sh;
      rc = dot_tasks(ctx, dj, who, prm, &nt, &sh);
      if (!rc) {
        int cap = 1;
        for (int q = 0; q < nt; ++q) cap = std::max(cap, std::max(dj.x[q].cap, dj.y[q].cap));
        const double w = (double)std::min(cap, sh.na);
        if (prm[0].digit) {
          int f = 0;
          while (f < (int)fb_shapes.size() && !(fb_shapes[f].ns == sh.ns && fb_shapes[f].na == sh.na)) ++f;
          if (f == (int)fb_shapes.size()) {
            fb_shapes.push_back(sh);
            bp.fb_cap.push_back(0);
          }
          bp.fb_cap[f] += nt;
          for (int q = 0; q < nt; ++q) prm[q].fb = f;
          digit_jobs.push_back((int32_t)bp.tasks.size());
        }
        for (int q = 0; q < nt; ++q) {
          bp.tasks.push_back(prm[q]);
          shape_dot.push_back(sh);
          cost_dot.push_back((double)(prm[q].N * prm[q].ct.ncomp + 1) * w * w);
        }
      }
    }
    if (rc) {
      ctx->err = "job " + std::to_string(i) + ": " + ctx->err;
      return rc;
    }
  }
  const size_t nd = bp.tasks.size(), nt = bp.tiles.size();
  if (nd + nt > (size_t)0x7FFFFFFF) return set_error(ctx, ARBGPU_EINVAL, "%s: too much work in one batch", who);
  auto shape = [&](size_t w) -> const LimbShape & { return w < nd ? shape_dot[w] : shape_tile[w - nd]; };
  auto cost = [&](size_t w) { return w < nd ? cost_dot[w] : cost_tile[w - nd]; };
  // dots of kDotBlockTerms real terms or more run on four waves each
  auto is_long = [&](size_t w) {
    return w < nd && shape_dot[w].ns > 0 && bp.tasks[w].N * bp.tasks[w].ct.ncomp >= kDotBlockTerms;
  };
  // limb work: dot tasks outside the digit runs, and the tiles
  std::vector<int32_t> work;
  work.reserve(nd + nt);
  for (size_t w = 0; w < nd + nt; ++w)
    if (w >= nd || !bp.tasks[w].digit) work.push_back((int32_t)w);
  std::stable_sort(work.begin(), work.end(), [&](int32_t x, int32_t y) {
    const LimbShape &a = shape(x), &c = shape(y);
    if (a.ns != c.ns) return a.ns > c.ns;
    if (a.na != c.na) return a.na > c.na;
    if (is_long(x) != is_long(y)) return is_long(x);
    return cost(x) > cost(y);
  });
  bp.order.resize(work.size());
  for (size_t t = 0; t < work.size(); ++t) {
    const size_t w = (size_t)work[t];
    bp.order[t] = w < nd ? (int32_t)w : -(int32_t)(w - nd) - 1;
    const LimbShape &sh = shape(w);
    const bool blk = is_long(w);
    if (bp.runs.empty() || bp.runs.back().sh.ns != sh.ns || bp.runs.back().sh.na != sh.na ||
        bp.runs.back().block != blk) {
      auto it = ctx->tune.find(tune_key(sh, blk));
      bp.runs.push_back({sh, blk, (int64_t)t, 0, it != ctx->tune.end() ? it->second : kDefaultWaves, 0.f});
    }
    bp.runs.back().count++;
  }
  // digit jobs: by block count and kind, longest first
  auto dcost = [&](int32_t e) { return (double)bp.tasks[e].N * bp.tasks[e].ct.ncomp * bp.tasks[e].digit; };
  std::stable_sort(digit_jobs.begin(), digit_jobs.end(), [&](int32_t x, int32_t y) {
    const DotParams &a = bp.tasks[x], &c = bp.tasks[y];
    if (a.digit != c.digit) return a.digit > c.digit;
    if (a.ct.ncomp != c.ct.ncomp) return a.ct.ncomp > c.ct.ncomp;
    return dcost(x) > dcost(y);
  });
  for (int32_t e : digit_jobs) {
    const DotParams &d = bp.tasks[e];
    const bool cplx = d.ct.ncomp == 2;
    if (bp.runs.empty() || bp.runs.back().digit != d.digit || bp.runs.back().cplx != cplx) {
      auto it = ctx->tune.find(tune_key_digit(d.digit, cplx));
      ShapeRun r{LimbShape{0, 0}, true, (int64_t)bp.order.size(), 0,
                 it != ctx->tune.end() ? it->second : kDefaultWaves, 0.f};
      r.digit = d.digit;
      r.cplx = cplx;
      bp.runs.push_back(r);
    }
    bp.order.push_back(e);
    bp.runs.back().count++;
  }
  // fallback runs, one per list
  for (size_t f = 0; f < fb_shapes.size(); ++f) {
    bp.fb_base.push_back((int32_t)bp.fb_total);
    ShapeRun r{fb_shapes[f], false, bp.fb_total, bp.fb_cap[f], kDefaultWaves, 0.f};
    r.fb = (int)f;
    bp.runs.push_back(r);
    bp.fb_total += bp.fb_cap[f];
  }
  return ARBGPU_OK;
}

// Workgroups of a persistent run: four tasks per workgroup (a wave each),
// or one (block runs), at most `waves` waves per compute unit.
unsigned blocks_for(int64_t count, int waves, int num_cu, bool block) {
  const int64_t by_work = block ? count : (count + 3) / 4;
  const int64_t by_width = std::max<int64_t>(1, (int64_t)num_cu * waves / 4);
  return (unsigned)std::max<int64_t>(1, std::min(by_work, by_width));
}

int device_cus(int device) {
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0) return ncu;
  return 256;
}

}  // namespace

namespace arbgpu_impl {

// Runs a plan can have: two per limb shape, the LDS-window run, two per
// digit block count and one fallback run per limb shape.
constexpr int kMaxRuns = 128;

size_t dot_batch_ws(int64_t n) {
  // tasks, order (at most one entry per task), fallback lists, their bases,
  // the run counters and the list counts
  return sizeof(DotParams) * (size_t)n + sizeof(int32_t) * (2 * (size_t)n + 3 * (size_t)kMaxRuns) + 64;
}

// Device side of a plan.
struct DevPlan {
  DotParams *tasks;
  MmParams *mm;
  BatchTile *tiles;
  int32_t *order;
  int32_t *counters;   // a work counter per run, then an entry count per fallback list
  int32_t *fb_list;
  int32_t *fb_base;
  int nruns;
};

// Kernel, grid, dynamic LDS and arguments of run k (the argument pointers
// point into this object).
struct RunLaunch {
  BatchShapeParams bp;
  DigitBatchParams dp;
  const DotParams *wt;
  const int32_t *wo;
  void *args[2];
  const void *func = nullptr;
  dim3 grid;
  size_t lds = 0;
  RunLaunch(const ShapeRun &r, size_t k, const DevPlan &d, int num_cu, int waves) {
    if (r.digit) {
      dp = DigitBatchParams{d.tasks, d.order + r.begin, r.count, d.counters + k, d.fb_list, d.fb_base,
                            d.counters + d.nruns};
      func = digit_dot_batch_kernel(r.digit, r.cplx, &lds);
      grid = dim3(blocks_for(r.count, waves, num_cu, true));
      args[0] = &dp;
    } else if (r.fb >= 0) {
      bp = BatchShapeParams{d.tasks, d.mm, d.tiles, d.fb_list + r.begin, r.count, d.counters + k,
                            d.counters + d.nruns + r.fb};
      func = dot_batch_kernel(r.sh, false);
      grid = dim3(blocks_for(r.count, waves, num_cu, false));
      args[0] = &bp;
    } else if (r.sh.ns == 0) {   // beyond the register windows: one workgroup per dot
      wt = d.tasks;
      wo = d.order + r.begin;
      func = wide_dot_batch_kernel_ptr(&lds);
      grid = dim3((unsigned)r.count);
      args[0] = &wt;
      args[1] = &wo;
    } else {
      bp = BatchShapeParams{d.tasks, d.mm, d.tiles, d.order + r.begin, r.count, d.counters + k, nullptr};
      func = dot_batch_kernel(r.sh, r.block);
      grid = dim3(blocks_for(r.count, waves, num_cu, r.block));
      args[0] = &bp;
    }
  }
  hipError_t launch(hipStream_t s) const {
    return hipLaunchKernel(func, grid, dim3(256), const_cast<void **>(args), lds, s);
  }
};

int dot_batch_run(arbgpu_ctx *ctx, const arbgpu_dot_job *jobs, int64_t njobs, hipStream_t s) {
  BatchPlan plan;
  int rc = plan_batch(ctx, jobs, nullptr, njobs, "dot batch", plan);
  const std::vector<DotParams> &tasks = plan.tasks;
  const std::vector<int32_t> &order = plan.order;
  const std::vector<ShapeRun> &runs = plan.runs;
  if (rc || tasks.empty()) return rc;
  if ((int)runs.size() > kMaxRuns) return set_error(ctx, ARBGPU_EINVAL, "dot batch: too many kernel runs");
  const size_t tb = sizeof(DotParams) * tasks.size(), ob = sizeof(int32_t) * order.size();
  char *w = (char *)ws_get(ctx, WS_BATCH, dot_batch_ws((int64_t)tasks.size()));
  if (!w) return ARBGPU_ENOMEM;
  DevPlan d;
  d.tasks = (DotParams *)w;
  d.mm = nullptr;
  d.tiles = nullptr;
  d.order = (int32_t *)(w + tb);
  d.fb_list = d.order + order.size();
  d.fb_base = d.fb_list + plan.fb_total;
  d.counters = d.fb_base + plan.fb_base.size();
  d.nruns = (int)runs.size();
  hipError_t e = hipMemcpyAsync(d.tasks, tasks.data(), tb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d.order, order.data(), ob, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !plan.fb_base.empty())
    e = hipMemcpyAsync(d.fb_base, plan.fb_base.data(), sizeof(int32_t) * plan.fb_base.size(), hipMemcpyHostToDevice,
                       s);
  if (e == hipSuccess) {
    int n = (int)(runs.size() + plan.fb_base.size());
    void *rargs[] = {&d.counters, &n};
    e = hipLaunchKernel(reinterpret_cast<const void *>(&batch_reset_kernel), dim3((unsigned)((n + 255) / 256)),
                        dim3(256), rargs, 0, s);
  }
  const int ncu = device_cus(ctx->device);
  // in stream order: the fallback runs come after every digit run
  for (size_t k = 0; k < runs.size() && e == hipSuccess; ++k) {
    RunLaunch rl(runs[k], k, d, ncu, runs[k].waves);
    e = rl.launch(s);
  }
  // the host task list must outlive its asynchronous upload
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "dot batch: %s", hipGetErrorString(e));
  return ARBGPU_OK;
}

}  // namespace arbgpu_impl

struct arbgpu_batch {
  arbgpu_ctx *ctx = nullptr;
  int64_t njobs = 0;
  std::vector<ShapeRun> runs;
  int64_t ntasks = 0, ntiles = 0;
  int nfb = 0;   // fallback lists
  DotParams *d_tasks = nullptr;
  MmParams *d_mm = nullptr;
  BatchTile *d_tiles = nullptr;
  int32_t *d_order = nullptr;
  int32_t *d_counters = nullptr;   // a work counter per run, then an entry count per fallback list
  int32_t *d_fb = nullptr;         // fallback lists, then their bases
  int num_cu = 256;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~arbgpu_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void *q : {(void *)d_tasks, (void *)d_mm, (void *)d_tiles, (void *)d_order, (void *)d_counters, (void *)d_fb})
      if (q) (void)hipFree(q);
  }

  int64_t fb_total() const {
    int64_t t = 0;
    for (auto &r : runs)
      if (r.fb >= 0) t += r.count;
    return t;
  }

  DevPlan dev() const {
    return DevPlan{d_tasks, d_mm, d_tiles, d_order, d_counters, d_fb, d_fb + fb_total(), (int)runs.size()};
  }

  // counters of every run and list cleared: a kernel node (no memset nodes)
  hipKernelNodeParams reset_params(void **rargs) const {
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof kp);
    kp.func = reinterpret_cast<void *>(&batch_reset_kernel);
    kp.gridDim = dim3((unsigned)((*(int *)rargs[1] + 255) / 256));
    kp.blockDim = dim3(256);
    kp.kernelParams = rargs;
    return kp;
  }

  int build_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    hipError_t e = hipGraphCreate(&graph, 0);
    if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "hipGraphCreate: %s", hipGetErrorString(e));
    int n = (int)std::max<size_t>(1, runs.size() + nfb);
    void *rargs[] = {&d_counters, &n};
    hipKernelNodeParams kp = reset_params(rargs);
    hipGraphNode_t reset;
    e = hipGraphAddKernelNode(&reset, graph, nullptr, 0, &kp);
    if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "graph node: %s", hipGetErrorString(e));
    const DevPlan d = dev();
    // limb, LDS-window and digit runs after the reset; fallback runs after
    // every digit run
    std::vector<hipGraphNode_t> digit_nodes;
    for (int pass = 0; pass < 2; ++pass)
      for (size_t k = 0; k < runs.size(); ++k) {
        if ((runs[k].fb >= 0) != (pass == 1)) continue;
        RunLaunch rl(runs[k], k, d, num_cu, runs[k].waves);
        hipKernelNodeParams np;
        memset(&np, 0, sizeof np);
        np.func = const_cast<void *>(rl.func);
        np.gridDim = rl.grid;
        np.blockDim = dim3(256);
        np.sharedMemBytes = (unsigned)rl.lds;
        np.kernelParams = rl.args;
        hipGraphNode_t node;
        if (pass == 0)
          e = hipGraphAddKernelNode(&node, graph, &reset, 1, &np);
        else
          e = hipGraphAddKernelNode(&node, graph, digit_nodes.data(), digit_nodes.size(), &np);
        if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "graph node: %s", hipGetErrorString(e));
        if (runs[k].digit) digit_nodes.push_back(node);
      }
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return ARBGPU_OK;
  }
};

namespace {

int batch_create(arbgpu_ctx *ctx, const arbgpu_dot_job *dots, const arbgpu_job *jobs, int64_t njobs,
                 arbgpu_batch **batch, const char *who) {
  if (!ctx || !batch) return ARBGPU_EINVAL;
  *batch = nullptr;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (njobs < 0 || (njobs > 0 && !dots && !jobs)) return set_error(ctx, ARBGPU_EINVAL, "%s: bad job list", who);
  if (njobs > (int64_t)1 << 29) return set_error(ctx, ARBGPU_EINVAL, "%s: too many jobs", who);
  BatchPlan plan;
  const int prc = plan_batch(ctx, dots, jobs, njobs, who, plan);
  if (prc) return prc;
  if (ctx->device < 0) return set_error(ctx, ARBGPU_EDEVICE, "host-only context cannot launch work");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  arbgpu_batch *b = new (std::nothrow) arbgpu_batch;
  if (!b) return ARBGPU_ENOMEM;
  b->ctx = ctx;
  b->njobs = njobs;
  b->ntasks = (int64_t)plan.tasks.size();
  b->ntiles = (int64_t)plan.tiles.size();
  b->num_cu = device_cus(ctx->device);
  b->runs = plan.runs;
  auto up = [&](void **dst, const void *src, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipMalloc(dst, std::max<size_t>(bytes, 16));
    if (e == hipSuccess) ++ctx->allocs;
    if (e == hipSuccess && bytes && src) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  up((void **)&b->d_tasks, plan.tasks.data(), sizeof(DotParams) * plan.tasks.size());
  up((void **)&b->d_mm, plan.mm.data(), sizeof(MmParams) * plan.mm.size());
  up((void **)&b->d_tiles, plan.tiles.data(), sizeof(BatchTile) * plan.tiles.size());
  up((void **)&b->d_order, plan.order.data(), sizeof(int32_t) * plan.order.size());
  b->nfb = (int)plan.fb_base.size();
  up((void **)&b->d_counters, nullptr, sizeof(int32_t) * std::max<size_t>(1, b->runs.size() + b->nfb));
  {   // fallback lists (filled on the device), then their bases
    std::vector<int32_t> fb((size_t)plan.fb_total, 0);
    fb.insert(fb.end(), plan.fb_base.begin(), plan.fb_base.end());
    up((void **)&b->d_fb, fb.data(), sizeof(int32_t) * fb.size());
  }
  if (e != hipSuccess) {
    delete b;
    return set_error(ctx, ARBGPU_ENOMEM, "%s: %s", who, hipGetErrorString(e));
  }
  const int rc = b->build_graph();
  if (rc) {
    delete b;
    return rc;
  }
  *batch = b;
  return ARBGPU_OK;
}

}  // namespace

extern "C" {

int arbgpu_batch_create(arbgpu_ctx *ctx, const arbgpu_dot_job *jobs, int64_t njobs, arbgpu_batch **batch) {
  return batch_create(ctx, jobs, nullptr, njobs, batch, "arbgpu_batch_create");
}

int arbgpu_batch_create_mixed(arbgpu_ctx *ctx, const arbgpu_job *jobs, int64_t njobs, arbgpu_batch **batch) {
  return batch_create(ctx, nullptr, jobs, njobs, batch, "arbgpu_batch_create_mixed");
}

int arbgpu_batch_launch(arbgpu_batch *b, arbgpu_stream stream) {
  if (!b) return ARBGPU_EINVAL;
  arbgpu_ctx *ctx = b->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) {
    KernelTimer kt(ctx, "dot_batch", s);
    e = hipGraphLaunch(b->exec, s);
  }
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "arbgpu_batch_launch: %s", hipGetErrorString(e));
  return ARBGPU_OK;
}

int arbgpu_batch_tune(arbgpu_batch *b, arbgpu_stream stream) {
  if (!b) return ARBGPU_EINVAL;
  arbgpu_ctx *ctx = b->ctx;
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipSetDevice(ctx->device);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  const DevPlan d = b->dev();
  for (size_t k = 0; k < b->runs.size() && e == hipSuccess; ++k) {
    ShapeRun &r = b->runs[k];
    // one workgroup per dot, or a device-filled list: no width to tune
    if ((r.sh.ns == 0 && !r.digit) || r.fb >= 0) continue;
    float best = 3.0e38f;
    int best_w = r.waves;
    for (int w : kTuneWaves) {
      float ms_min = 0.f;
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        RunLaunch rl(r, k, d, b->num_cu, w);
        // every counter and list count (a digit run fills the lists)
        int n = (int)(b->runs.size() + b->nfb);
        int32_t *ctr = b->d_counters;
        void *rargs[] = {&ctr, &n};
        e = hipLaunchKernel(reinterpret_cast<const void *>(&batch_reset_kernel), dim3((unsigned)((n + 255) / 256)),
                            dim3(256), rargs, 0, s);
        if (e == hipSuccess) e = hipEventRecord(t0, s);
        if (e == hipSuccess) e = rl.launch(s);
        if (e == hipSuccess) e = hipEventRecord(t1, s);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (rep == 0 || ms < ms_min) ms_min = ms;
      }
      if (e != hipSuccess) break;
      if (ms_min < best) {
        best = ms_min;
        best_w = w;
      }
    }
    r.waves = best_w;
    r.tuned_ms = best;
    ctx->tune[r.digit ? tune_key_digit(r.digit, r.cplx) : tune_key(r.sh, r.block)] = best_w;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "arbgpu_batch_tune: %s", hipGetErrorString(e));
  tune_save(ctx);
  return b->build_graph();
}

int arbgpu_batch_info(arbgpu_batch *b, int64_t *out, int n) {
  if (!b || !out || n < 0) return ARBGPU_EINVAL;
  std::vector<int64_t> v = {b->njobs, b->ntasks + b->ntiles, (int64_t)b->runs.size()};
  for (auto &r : b->runs) {
    // digit runs: (-blocks, 1 real | 2 complex)
    v.push_back(r.digit ? -r.digit : r.sh.ns);
    v.push_back(r.digit ? (r.cplx ? 2 : 1) : r.sh.na);
    v.push_back(r.count);
    v.push_back(r.waves);
    v.push_back((int64_t)(r.tuned_ms * 1000.f));
  }
  for (int i = 0; i < n; ++i) out[i] = i < (int)v.size() ? v[i] : 0;
  return ARBGPU_OK;
}

void arbgpu_batch_destroy(arbgpu_batch *b) {
  if (!b) return;
  if (b->ctx && b->ctx->device >= 0 && hipSetDevice(b->ctx->device) == hipSuccess) (void)hipDeviceSynchronize();
  delete b;
}

}  // extern "C"
