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

std::string tune_key(LimbShape sh) {
  return "dot_batch:" + std::to_string(sh.ns) + "x" + std::to_string(sh.na);
}

struct ShapeRun {
  LimbShape sh;
  int64_t begin, count;   // slice of the order array
  int waves;              // per compute unit
  float tuned_ms;         // time of this shape alone at `waves` (0: not tuned)
};

// Validates the jobs and builds the tasks, their order (by shape, longest
// first) and the per-shape runs; sets the context error on a bad job.
int plan_batch(arbgpu_ctx *ctx, const arbgpu_dot_job *jobs, int64_t njobs, const char *who,
               std::vector<DotParams> &tasks, std::vector<int32_t> &order, std::vector<ShapeRun> &runs) {
  std::vector<LimbShape> shape_of;
  std::vector<double> cost;
  tasks.clear();
  runs.clear();
  tasks.reserve((size_t)njobs * 2);
  for (int64_t i = 0; i < njobs; ++i) {
    DotParams prm[2];
    int nt = 0;
    LimbShape sh;
    const int rc = dot_tasks(ctx, jobs[i], who, prm, &nt, &sh);
    if (rc) {
      ctx->err = "job " + std::to_string(i) + ": " + ctx->err;
      return rc;
    }
    int cap = 1;
    for (int q = 0; q < nt; ++q) cap = std::max(cap, std::max(jobs[i].x[q].cap, jobs[i].y[q].cap));
    const double w = (double)std::min(cap, sh.na);
    for (int q = 0; q < nt; ++q) {
      tasks.push_back(prm[q]);
      shape_of.push_back(sh);
      cost.push_back((double)(prm[q].N * prm[q].ct.ncomp + 1) * w * w);
    }
  }
  order.resize(tasks.size());
  for (size_t t = 0; t < tasks.size(); ++t) order[t] = (int32_t)t;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const LimbShape &a = shape_of[x], &c = shape_of[y];
    if (a.ns != c.ns) return a.ns > c.ns;
    if (a.na != c.na) return a.na > c.na;
    return cost[x] > cost[y];
  });
  for (size_t t = 0; t < order.size(); ++t) {
    const LimbShape &sh = shape_of[order[t]];
    if (runs.empty() || runs.back().sh.ns != sh.ns || runs.back().sh.na != sh.na) {
      auto it = ctx->tune.find(tune_key(sh));
      runs.push_back({sh, (int64_t)t, 0, it != ctx->tune.end() ? it->second : kDefaultWaves, 0.f});
    }
    runs.back().count++;
  }
  return ARBGPU_OK;
}

unsigned blocks_for(int64_t count, int waves, int num_cu) {
  const int64_t by_work = (count + 3) / 4;
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
  std::vector<DotParams> tasks;
  std::vector<int32_t> order;
  std::vector<ShapeRun> runs;
  int rc = plan_batch(ctx, jobs, njobs, "dot batch", tasks, order, runs);
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
    BatchShapeParams bp{d_tasks, d_order + runs[k].begin, runs[k].count, d_ctr + k};
    void *args[] = {&bp};
    e = hipLaunchKernel(dot_batch_kernel(runs[k].sh), dim3(blocks_for(runs[k].count, runs[k].waves, ncu)),
                        dim3(256), args, 0, s);
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
  int64_t ntasks = 0;
  DotParams *d_tasks = nullptr;
  int32_t *d_order = nullptr;
  int32_t *d_counters = nullptr;
  int num_cu = 256;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~arbgpu_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_tasks) (void)hipFree(d_tasks);
    if (d_order) (void)hipFree(d_order);
    if (d_counters) (void)hipFree(d_counters);
  }

  unsigned blocks_for(const ShapeRun &r, int waves) const { return ::blocks_for(r.count, waves, num_cu); }

  BatchShapeParams params(size_t k) const {
    return BatchShapeParams{d_tasks, d_order + runs[k].begin, runs[k].count, d_counters + k};
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
      void *args[] = {&bp};
      hipKernelNodeParams np;
      memset(&np, 0, sizeof np);
      np.func = const_cast<void *>(dot_batch_kernel(runs[k].sh));
      np.gridDim = dim3(blocks_for(runs[k], runs[k].waves));
      np.blockDim = dim3(256);
      np.kernelParams = args;
      hipGraphNode_t node;
      e = hipGraphAddKernelNode(&node, graph, &reset, 1, &np);
      if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "graph node: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return ARBGPU_OK;
  }
};

extern "C" {

int arbgpu_batch_create(arbgpu_ctx *ctx, const arbgpu_dot_job *jobs, int64_t njobs, arbgpu_batch **batch) {
  if (!ctx || !batch) return ARBGPU_EINVAL;
  *batch = nullptr;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (njobs < 0 || (njobs > 0 && !jobs)) return set_error(ctx, ARBGPU_EINVAL, "arbgpu_batch_create: bad job list");
  if (njobs > (int64_t)1 << 29) return set_error(ctx, ARBGPU_EINVAL, "arbgpu_batch_create: too many jobs");
  std::vector<DotParams> tasks;
  std::vector<int32_t> order;
  std::vector<ShapeRun> runs;
  const int prc = plan_batch(ctx, jobs, njobs, "arbgpu_batch_create", tasks, order, runs);
  if (prc) return prc;
  if (ctx->device < 0) return set_error(ctx, ARBGPU_EDEVICE, "host-only context cannot launch work");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  arbgpu_batch *b = new (std::nothrow) arbgpu_batch;
  if (!b) return ARBGPU_ENOMEM;
  b->ctx = ctx;
  b->njobs = njobs;
  b->ntasks = (int64_t)tasks.size();
  b->num_cu = device_cus(ctx->device);
  b->runs = runs;
  const size_t tb = sizeof(DotParams) * std::max<size_t>(1, tasks.size());
  const size_t ob = sizeof(int32_t) * std::max<size_t>(1, order.size());
  const size_t cb = sizeof(int32_t) * std::max<size_t>(1, b->runs.size());
  if ((e = hipMalloc(&b->d_tasks, tb)) != hipSuccess || (e = hipMalloc(&b->d_order, ob)) != hipSuccess ||
      (e = hipMalloc(&b->d_counters, cb)) != hipSuccess) {
    delete b;
    return set_error(ctx, ARBGPU_ENOMEM, "arbgpu_batch_create: %s", hipGetErrorString(e));
  }
  ctx->allocs += 3;
  if (!tasks.empty() &&
      ((e = hipMemcpy(b->d_tasks, tasks.data(), sizeof(DotParams) * tasks.size(), hipMemcpyHostToDevice)) !=
           hipSuccess ||
       (e = hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice)) !=
           hipSuccess)) {
    delete b;
    return set_error(ctx, ARBGPU_EDEVICE, "arbgpu_batch_create upload: %s", hipGetErrorString(e));
  }
  const int rc = b->build_graph();
  if (rc) {
    delete b;
    return rc;
  }
  *batch = b;
  return ARBGPU_OK;
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
          e = hipLaunchKernel(dot_batch_kernel(b->runs[k].sh), dim3(b->blocks_for(b->runs[k], w)), dim3(256), args,
                              0, s);
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
    ctx->tune[tune_key(b->runs[k].sh)] = best_w;
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "arbgpu_batch_tune: %s", hipGetErrorString(e));
  tune_save(ctx);
  return b->build_graph();
}

int arbgpu_batch_info(arbgpu_batch *b, int64_t *out, int n) {
  if (!b || !out || n < 0) return ARBGPU_EINVAL;
  std::vector<int64_t> v = {b->njobs, b->ntasks, (int64_t)b->runs.size()};
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
