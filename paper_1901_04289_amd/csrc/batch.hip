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

struct ShapeRun {
  LimbShape sh;
  bool block;             // long dots: four waves per task
  int64_t begin, count;   // slice of the order array
  int waves;              // per compute unit
  float tuned_ms;         // time of this run alone at `waves` (0: not tuned)
};

// The work of a batch: dot tasks, matrix-product parts and their tiles,
// and the per-shape runs over `order` (by shape, longest first).
struct BatchPlan {
  std::vector<DotParams> tasks;
  std::vector<MmParams> mm;
  std::vector<BatchTile> tiles;
  std::vector<int32_t> order;   // dot task e >= 0, tile -e - 1
  std::vector<ShapeRun> runs;
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
  std::vector<int32_t> work(nd + nt);
  for (size_t w = 0; w < work.size(); ++w) work[w] = (int32_t)w;
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

size_t dot_batch_ws(int64_t n, int nshapes) {
  return sizeof(DotParams) * (size_t)n + sizeof(int32_t) * ((size_t)n + (size_t)nshapes) + 64;
}

int dot_batch_run(arbgpu_ctx *ctx, const arbgpu_dot_job *jobs, int64_t njobs, hipStream_t s) {
  BatchPlan plan;
  int rc = plan_batch(ctx, jobs, nullptr, njobs, "dot batch", plan);
  const std::vector<DotParams> &tasks = plan.tasks;
  const std::vector<int32_t> &order = plan.order;
  const std::vector<ShapeRun> &runs = plan.runs;
  if (rc || tasks.empty()) return rc;
  const size_t tb = sizeof(DotParams) * tasks.size(), ob = sizeof(int32_t) * order.size();
  char *w = (char *)ws_get(ctx, WS_BATCH, dot_batch_ws((int64_t)tasks.size(), (int)runs.size()));
  if (!w) return ARBGPU_ENOMEM;
  DotParams *d_tasks = (DotParams *)w;
  int32_t *d_order = (int32_t *)(w + tb);
  int32_t *d_ctr = d_order + order.size();
  hipError_t e = hipMemcpyAsync(d_tasks, tasks.data(), tb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_order, order.data(), ob, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    int n = (int)runs.size();
    void *rargs[] = {&d_ctr, &n};
    e = hipLaunchKernel(reinterpret_cast<const void *>(&batch_reset_kernel), dim3((unsigned)((n + 255) / 256)),
                        dim3(256), rargs, 0, s);
  }
  const int ncu = device_cus(ctx->device);
  for (size_t k = 0; k < runs.size() && e == hipSuccess; ++k) {
    if (runs[k].sh.ns == 0) {   // beyond the register windows: one workgroup per dot
      e = launch_wide_dot_batch(d_tasks, d_order + runs[k].begin, runs[k].count, s);
      continue;
    }
    BatchShapeParams bp{d_tasks, nullptr, nullptr, d_order + runs[k].begin, runs[k].count, d_ctr + k};
    void *args[] = {&bp};
    e = hipLaunchKernel(dot_batch_kernel(runs[k].sh, runs[k].block),
                        dim3(blocks_for(runs[k].count, runs[k].waves, ncu, runs[k].block)), dim3(256), args, 0, s);
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
  DotParams *d_tasks = nullptr;
  MmParams *d_mm = nullptr;
  BatchTile *d_tiles = nullptr;
  int32_t *d_order = nullptr;
  int32_t *d_counters = nullptr;
  int num_cu = 256;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~arbgpu_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void *q : {(void *)d_tasks, (void *)d_mm, (void *)d_tiles, (void *)d_order, (void *)d_counters})
      if (q) (void)hipFree(q);
  }

  unsigned blocks_for(const ShapeRun &r, int waves) const { return ::blocks_for(r.count, waves, num_cu, r.block); }

  BatchShapeParams params(size_t k) const {
    return BatchShapeParams{d_tasks, d_mm, d_tiles, d_order + runs[k].begin, runs[k].count, d_counters + k};
  }

  int build_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    hipError_t e = hipGraphCreate(&graph, 0);
    if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "hipGraphCreate: %s", hipGetErrorString(e));
    // counters are cleared by a kernel node: memset nodes are not used
    int n = (int)std::max<size_t>(1, runs.size());
    void *rargs[] = {&d_counters, &n};
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof kp);
    kp.func = reinterpret_cast<void *>(&batch_reset_kernel);
    kp.gridDim = dim3((unsigned)((n + 255) / 256));
    kp.blockDim = dim3(256);
    kp.kernelParams = rargs;
    hipGraphNode_t reset;
    e = hipGraphAddKernelNode(&reset, graph, nullptr, 0, &kp);
    if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "graph node: %s", hipGetErrorString(e));
    for (size_t k = 0; k < runs.size(); ++k) {
      BatchShapeParams bp = params(k);
      const int32_t *wide_order = d_order + runs[k].begin;
      void *args[] = {&bp};
      void *wargs[] = {&d_tasks, &wide_order};
      hipKernelNodeParams np;
      memset(&np, 0, sizeof np);
      if (runs[k].sh.ns == 0) {   // beyond the register windows: one workgroup per dot
        size_t lds = 0;
        np.func = const_cast<void *>(wide_dot_batch_kernel_ptr(&lds));
        np.gridDim = dim3((unsigned)runs[k].count);
        np.sharedMemBytes = (unsigned)lds;
        np.kernelParams = wargs;
      } else {
        np.func = const_cast<void *>(dot_batch_kernel(runs[k].sh, runs[k].block));
        np.gridDim = dim3(blocks_for(runs[k], runs[k].waves));
        np.kernelParams = args;
      }
      np.blockDim = dim3(256);
      hipGraphNode_t node;
      e = hipGraphAddKernelNode(&node, graph, &reset, 1, &np);
      if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "graph node: %s", hipGetErrorString(e));
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
  up((void **)&b->d_counters, nullptr, sizeof(int32_t) * std::max<size_t>(1, b->runs.size()));
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
  for (size_t k = 0; k < b->runs.size() && e == hipSuccess; ++k) {
    if (b->runs[k].sh.ns == 0) continue;   // one workgroup per dot: no width to tune
    float best = 3.0e38f;
    int best_w = b->runs[k].waves;
    for (int w : kTuneWaves) {
      float ms_min = 0.f;
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        BatchShapeParams bp = b->params(k);
        void *args[] = {&bp};
        int one = 1;
        int32_t *ctr = bp.counter;
        void *rargs[] = {&ctr, &one};
        e = hipLaunchKernel(reinterpret_cast<const void *>(&batch_reset_kernel), dim3(1), dim3(256), rargs, 0, s);
        if (e == hipSuccess) e = hipEventRecord(t0, s);
        if (e == hipSuccess)
          e = hipLaunchKernel(dot_batch_kernel(b->runs[k].sh, b->runs[k].block), dim3(b->blocks_for(b->runs[k], w)),
                              dim3(256), args, 0, s);
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
    b->runs[k].waves = best_w;
    b->runs[k].tuned_ms = best;
    ctx->tune[tune_key(b->runs[k].sh, b->runs[k].block)] = best_w;
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
    v.push_back(r.sh.ns);
    v.push_back(r.sh.na);
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
