// C-ABI front end of libarbgpu: argument validation, context, dispatch.
//
// Every entry point validates its arguments on the host before it touches
// the device, so argument errors are reported synchronously and are
// testable without a GPU (arbgpu_init with device -1).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace arbgpu_impl;

arbgpu_ctx::~arbgpu_ctx() {
  if (server) arbgpu_impl::server_delete(server);
  delete noalloc_view;
  for (auto &t : timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto &b : ws)
    if (b.ptr && b.owned) (void)hipFree(b.ptr);
  if (ev_stats) (void)hipEventDestroy(ev_stats);
  if (stats_host) (void)hipHostFree(stats_host);
}

namespace arbgpu_impl {

int set_error(arbgpu_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

namespace {

// Waits for the work this context enqueued (on every stream it used) so
// that a workspace buffer can be freed; other contexts' work is not waited
// for.
void ctx_drain(arbgpu_ctx *ctx) {
  for (hipStream_t st : ctx->streams_seen) (void)hipStreamSynchronize(st);
  ctx->streams_seen.clear();
}

bool ws_grow(arbgpu_ctx *ctx, int slot, size_t bytes) {
  arbgpu_ctx::Buf &b = ctx->ws[slot];
  size_t total = bytes;
  for (int i = 0; i < (int)ctx->ws.size(); ++i)
    if (i != slot && ctx->ws[i].owned) total += ctx->ws[i].size;
  if (ctx->budget && total > ctx->budget) {
    set_error(ctx, ARBGPU_ENOMEM, "workspace of %zu bytes exceeds the HBM budget %zu", total, ctx->budget);
    return false;
  }
  if (b.ptr) {
    ctx_drain(ctx);
    if (b.owned) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.size = 0;
    if (slot == WS_RNS) ctx->rns_key = -1;
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    set_error(ctx, ARBGPU_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    return false;
  }
  ++ctx->allocs;
  b.ptr = p;
  b.size = bytes;
  b.owned = true;
  return true;
}

}  // namespace

void *ws_get(arbgpu_ctx *ctx, int slot, size_t bytes) {
  if ((int)ctx->ws.size() < WS_COUNT) ctx->ws.resize(WS_COUNT);
  arbgpu_ctx::Buf &b = ctx->ws[slot];
  if (bytes == 0) bytes = 256;
  if (b.size >= bytes) return b.ptr;
  if (ctx->bump_base) {
    const size_t off = (ctx->bump_top + 255) & ~(size_t)255;
    if (off > ctx->bump_size || bytes > ctx->bump_size - off) {
      set_error(ctx, ARBGPU_ENOMEM, "the call needs more than the %zu bytes of its fixed scratch", ctx->bump_size);
      return nullptr;
    }
    b.ptr = ctx->bump_base + off;
    b.size = bytes;
    b.owned = false;
    ctx->bump_top = off + bytes;
    if (slot == WS_RNS) ctx->rns_key = -1;   // a new place: the tables are uploaded again
    return b.ptr;
  }
  if (ctx->ws_fixed) {
    set_error(ctx, ARBGPU_ENOMEM, "workspace slot %d holds %zu bytes, the call needs %zu (fixed workspace)", slot,
              b.size, bytes);
    return nullptr;
  }
  return ws_grow(ctx, slot, bytes) ? b.ptr : nullptr;
}

int ws_reserve(arbgpu_ctx *ctx, const size_t sizes[WS_COUNT]) {
  if ((int)ctx->ws.size() < WS_COUNT) ctx->ws.resize(WS_COUNT);
  for (int k = 0; k < WS_COUNT; ++k)
    if (sizes[k] > ctx->ws[k].size) {
      if (ctx->ws_fixed)
        return set_error(ctx, ARBGPU_ENOMEM, "workspace slot %d is fixed at %zu bytes", k, ctx->ws[k].size);
      if (!ws_grow(ctx, k, sizes[k])) return ARBGPU_ENOMEM;
    }
  return ARBGPU_OK;
}

void ctx_use_stream(arbgpu_ctx *ctx, hipStream_t s) {
  for (hipStream_t t : ctx->streams_seen)
    if (t == s) return;
  ctx->streams_seen.push_back(s);
}

void tune_load(arbgpu_ctx *ctx) {
  FILE *f = fopen(ctx->tune_path.c_str(), "r");
  if (!f) return;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  fclose(f);
  // "key": value pairs; anything else is skipped
  size_t i = 0;
  while ((i = txt.find('"', i)) != std::string::npos) {
    const size_t j = txt.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = txt.substr(i + 1, j - i - 1);
    size_t k = j + 1;
    while (k < txt.size() && (txt[k] == ' ' || txt[k] == ':' || txt[k] == '\t')) ++k;
    char *end = nullptr;
    const long v = strtol(txt.c_str() + k, &end, 10);
    if (end != txt.c_str() + k) ctx->tune[key] = (int)v;
    i = j + 1;
  }
}

void tune_save(arbgpu_ctx *ctx) {
  if (ctx->tune_path.empty()) return;
  FILE *f = fopen(ctx->tune_path.c_str(), "w");
  if (!f) return;
  fprintf(f, "{");
  bool first = true;
  for (auto &kv : ctx->tune) {
    fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
    first = false;
  }
  fprintf(f, "\n}\n");
  fclose(f);
}

}  // namespace arbgpu_impl

namespace {

int fail(arbgpu_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

int hip_fail(arbgpu_ctx *ctx, hipError_t e, const char *where) {
  return fail(ctx, ARBGPU_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

// Element index range [lo, hi] touched by off + i*s1 + j*s2, 0 <= i < n1,
// 0 <= j < n2.
void index_range(int64_t off, int64_t n1, int64_t s1, int64_t n2, int64_t s2, int64_t *lo, int64_t *hi) {
  int64_t a = off, b = off;
  if (n1 > 0) {
    int64_t d = (n1 - 1) * s1;
    if (d < 0) a += d; else b += d;
  }
  if (n2 > 0) {
    int64_t d = (n2 - 1) * s2;
    if (d < 0) a += d; else b += d;
  }
  *lo = a;
  *hi = b;
}

bool arr_ok(const arbgpu_arr &a) {
  if (!a.limbs || !a.exp || !a.nls) return false;
  if (a.cap < 1 || a.ld < 1) return false;
  if ((a.rad_m == nullptr) != (a.rad_e == nullptr)) return false;
  return true;
}

bool out_ok(const arbgpu_out &o, int64_t p, bool approx) {
  if (!o.limbs || !o.exp || !o.nls) return false;
  if (o.ld < 1) return false;
  if ((int64_t)o.cap * 32 < p) return false;
  if (!approx && (!o.rad_m || !o.rad_e)) return false;
  return true;
}

// Indices [lo, hi] must be non-negative and the limb planes must not
// overlap the index range (ld covers the largest index).
bool range_ok(int64_t lo, int64_t hi, int64_t ld) { return lo >= 0 && hi < ld; }

hipStream_t to_stream(arbgpu_stream s) { return reinterpret_cast<hipStream_t>(s); }

int bind_device(arbgpu_ctx *ctx, arbgpu_stream s) {
  if (ctx->device < 0) return fail(ctx, ARBGPU_EDEVICE, "host-only context cannot launch work");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  ctx_use_stream(ctx, to_stream(s));
  return ARBGPU_OK;
}

}  // namespace

namespace arbgpu_impl {

int dot_tasks(arbgpu_ctx *ctx, const arbgpu_dot_job &job, const char *who, DotParams prm[2], int *ntasks,
              LimbShape *shape) {
  const uint32_t flags = job.flags;
  const bool approx = flags & ARBGPU_APPROX;
  const bool cplx = flags & ARBGPU_COMPLEX;
  const int nparts = cplx ? 2 : 1;
  const bool has_init = job.init[0].limbs != nullptr;
  const int64_t p = job.p, N = job.N;
  if (flags & ~(ARBGPU_APPROX | ARBGPU_COMPLEX | ARBGPU_REDUCE_PREC | ARBGPU_ALGO_LIMB))
    return fail(ctx, ARBGPU_EINVAL, "%s: unknown flags 0x%x", who, flags);
  if (p < 2 || p > (1 << 20)) return fail(ctx, ARBGPU_EINVAL, "%s: p=%lld out of range", who, (long long)p);
  if (N < 0) return fail(ctx, ARBGPU_EINVAL, "%s: N < 0", who);
  int cap = 1;
  for (int q = 0; q < nparts; ++q) {
    if (!out_ok(job.res[q], p, approx)) return fail(ctx, ARBGPU_EINVAL, "%s: bad result array (cap, pointers)", who);
    if (job.res_idx < 0 || job.res_idx >= job.res[q].ld)
      return fail(ctx, ARBGPU_EINVAL, "%s: res_idx out of range", who);
    if (!arr_ok(job.x[q]) || !arr_ok(job.y[q])) return fail(ctx, ARBGPU_EINVAL, "%s: bad operand array", who);
    int64_t lo, hi;
    index_range(job.xoff, N, job.xstep, 0, 0, &lo, &hi);
    if (N > 0 && !range_ok(lo, hi, job.x[q].ld)) return fail(ctx, ARBGPU_EINVAL, "%s: x index out of range", who);
    index_range(job.yoff, N, job.ystep, 0, 0, &lo, &hi);
    if (N > 0 && !range_ok(lo, hi, job.y[q].ld)) return fail(ctx, ARBGPU_EINVAL, "%s: y index out of range", who);
    if (has_init) {
      if (!arr_ok(job.init[q])) return fail(ctx, ARBGPU_EINVAL, "%s: bad initial array", who);
      if (job.init_idx < 0 || job.init_idx >= job.init[q].ld)
        return fail(ctx, ARBGPU_EINVAL, "%s: init_idx out of range", who);
      cap = job.init[q].cap > cap ? job.init[q].cap : cap;
    }
    cap = job.x[q].cap > cap ? job.x[q].cap : cap;
    cap = job.y[q].cap > cap ? job.y[q].cap : cap;
  }
  if (!limb_shape_for((int)p, N * nparts + 1, cap, shape)) {
    // beyond every register window: the LDS-window kernel
    if (p > wide_max_precision())
      return fail(ctx, ARBGPU_EINVAL, "%s: precision %lld above %d bits", who, (long long)p, wide_max_precision());
    if (cap > wide_max_limbs())
      return fail(ctx, ARBGPU_EINVAL, "%s: operands of %d limbs above %d", who, cap, wide_max_limbs());
    *shape = LimbShape{0, 0};
  }
  for (int q = 0; q < nparts; ++q) {
    DotParams &d = prm[q];
    memset(&d, 0, sizeof d);
    for (int k = 0; k < 2; ++k) {
      const int src = cplx ? k : 0;
      d.X[k] = job.x[src];
      d.Y[k] = job.y[src];
      if (has_init) d.I[k] = job.init[src];
    }
    d.has_init = has_init;
    d.init_idx = job.init_idx;
    d.init_part = q;
    d.R = job.res[q];
    d.res_idx = job.res_idx;
    d.xoff = job.xoff; d.xstep = job.xstep; d.yoff = job.yoff; d.ystep = job.ystep; d.N = N;
    d.p = (int)p;
    d.approx = approx;
    d.sub = job.sub ? 1u : 0u;
    d.reduce = (flags & ARBGPU_REDUCE_PREC) != 0;
    d.ct = !cplx ? comp_real() : (q == 0 ? comp_re() : comp_im());
    d.na = shape->na;
    d.fb = -1;
  }
  const int lb = (flags & ARBGPU_ALGO_LIMB) ? 0 : digit_blocks(prm[0], *shape);
  for (int q = 0; q < nparts; ++q) prm[q].digit = lb;
  *ntasks = nparts;
  return ARBGPU_OK;
}

}  // namespace arbgpu_impl

extern "C" {

int arbgpu_init(arbgpu_ctx **ctx, int device, size_t hbm_budget_bytes, const char *tune_cache) {
  if (!ctx) return ARBGPU_EINVAL;
  *ctx = nullptr;
  if (device < -1) return ARBGPU_EINVAL;
  arbgpu_ctx *c = new (std::nothrow) arbgpu_ctx;
  if (!c) return ARBGPU_ENOMEM;
  c->device = device;
  c->budget = hbm_budget_bytes;
  if (tune_cache && tune_cache[0]) {
    c->tune_path = tune_cache;
    tune_load(c);
  }
  if (device >= 0) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device >= n) {
      delete c;
      return ARBGPU_EDEVICE;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) {
      delete c;
      return ARBGPU_EDEVICE;
    }
    if (c->budget == 0) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess) c->budget = fr / 4 * 3;
    }
    // the allocation-free entry point's scratch address on this device, and
    // the context its calls run on
    c->noalloc_view = new (std::nothrow) arbgpu_ctx;
    if (!c->noalloc_view || noalloc_setup(device) != ARBGPU_OK) {
      delete c;
      return ARBGPU_EDEVICE;
    }
    c->noalloc_view->device = device;
    c->noalloc_view->budget = 0;
    c->noalloc_view->ws.resize(WS_COUNT);
  }
  *ctx = c;
  return ARBGPU_OK;
}

void arbgpu_destroy(arbgpu_ctx *ctx) {
  if (!ctx) return;
  if (ctx->device >= 0 && hipSetDevice(ctx->device) == hipSuccess) (void)hipDeviceSynchronize();
  delete ctx;
}

const char *arbgpu_last_error(const arbgpu_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

int arbgpu_timing(arbgpu_ctx *ctx, int enable) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (auto &t : ctx->timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  ctx->timed.clear();
  ctx->timing = enable != 0;
  return ARBGPU_OK;
}

int arbgpu_plan_info(arbgpu_ctx *ctx, int64_t *out, int n) {
  if (!ctx || !out || n < 0) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (int i = 0; i < n; ++i) out[i] = i < 10 ? ctx->last_plan[i] : 0;
  return ARBGPU_OK;
}

int arbgpu_timing_read(arbgpu_ctx *ctx, const char *kernel, double *ms_total, int64_t *launches) {
  if (!ctx || !kernel || !ms_total || !launches) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  double tot = 0.0;
  int64_t n = 0;
  for (auto &t : ctx->timed) {
    if (strcmp(t.name, kernel) != 0) continue;
    hipError_t e = hipEventSynchronize(t.stop);
    if (e != hipSuccess) return fail(ctx, ARBGPU_EDEVICE, "hipEventSynchronize: %s", hipGetErrorString(e));
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, t.start, t.stop);
    if (e != hipSuccess) return fail(ctx, ARBGPU_EDEVICE, "hipEventElapsedTime: %s", hipGetErrorString(e));
    tot += ms;
    ++n;
  }
  *ms_total = tot;
  *launches = n;
  return ARBGPU_OK;
}

int arbgpu_dot(arbgpu_ctx *ctx, const arbgpu_out *res, int64_t res_idx, const arbgpu_arr *initial,
               int64_t init_idx, int sub, const arbgpu_arr *x, int64_t xoff, int64_t xstep,
               const arbgpu_arr *y, int64_t yoff, int64_t ystep, int64_t N, int64_t p, uint32_t flags,
               arbgpu_stream stream) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!res || !x || !y) return fail(ctx, ARBGPU_EINVAL, "arbgpu_dot: NULL argument");
  const int nparts = (flags & ARBGPU_COMPLEX) ? 2 : 1;
  arbgpu_dot_job job;
  memset(&job, 0, sizeof job);
  for (int q = 0; q < nparts; ++q) {
    job.res[q] = res[q];
    job.x[q] = x[q];
    job.y[q] = y[q];
    if (initial) job.init[q] = initial[q];
  }
  job.res_idx = res_idx;
  job.init_idx = init_idx;
  job.xoff = xoff; job.xstep = xstep; job.yoff = yoff; job.ystep = ystep; job.N = N; job.p = p;
  job.flags = flags;
  job.sub = sub;
  if (initial && !initial[0].limbs) return fail(ctx, ARBGPU_EINVAL, "arbgpu_dot: bad initial array");
  DotParams prm[2];
  int nt = 0;
  LimbShape sh;
  int rc = dot_tasks(ctx, job, "arbgpu_dot", prm, &nt, &sh);
  if (rc) return rc;
  if ((rc = bind_device(ctx, stream))) return rc;
  const hipStream_t s = to_stream(stream);
  if (prm[0].digit) {
    // the digit product, then the limb kernel for any part it hands back
    int32_t *flags = (int32_t *)ws_get(ctx, WS_DOTFLAG, 2 * sizeof(int32_t));
    if (!flags) return ARBGPU_ENOMEM;
    {
      KernelTimer kt(ctx, "digit_dot", s);
      hipError_t e = launch_digit_dot(prm, prm[0].digit, flags, s);
      if (e != hipSuccess) return hip_fail(ctx, e, "arbgpu_dot launch");
    }
    for (int q = 0; q < nt; ++q) {
      hipError_t e = launch_limb_dot(prm[q], sh, s, flags + q);
      if (e != hipSuccess) return hip_fail(ctx, e, "arbgpu_dot launch");
    }
    return ARBGPU_OK;
  }
  for (int q = 0; q < nt; ++q) {
    KernelTimer kt(ctx, "limb_dot", s);
    hipError_t e = sh.ns ? launch_limb_dot(prm[q], sh, s) : launch_wide_dot(prm[q], s);
    if (e != hipSuccess) return hip_fail(ctx, e, "arbgpu_dot launch");
  }
  return ARBGPU_OK;
}

static int validate_mat(arbgpu_ctx *ctx, const arbgpu_mat *m, int nparts, const char *name) {
  if (!m) return fail(ctx, ARBGPU_EINVAL, "%s is NULL", name);
  if (m->rows < 0 || m->cols < 0) return fail(ctx, ARBGPU_EINVAL, "%s: negative shape", name);
  const arbgpu_arr *parts[2] = {&m->re, &m->im};
  for (int q = 0; q < nparts; ++q) {
    if (!arr_ok(*parts[q])) return fail(ctx, ARBGPU_EINVAL, "%s: bad array", name);
    int64_t lo, hi;
    index_range(m->off, m->rows, m->rs, m->cols, m->cs, &lo, &hi);
    if (m->rows > 0 && m->cols > 0 && !range_ok(lo, hi, parts[q]->ld))
      return fail(ctx, ARBGPU_EINVAL, "%s: element index out of range", name);
  }
  return ARBGPU_OK;
}

}  // extern "C"

namespace arbgpu_impl {

int mat_mul_check(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p,
                  uint32_t flags) {
  const bool approx = flags & ARBGPU_APPROX;
  const bool cplx = flags & ARBGPU_COMPLEX;
  const int nparts = cplx ? 2 : 1;
  if (flags & ~(ARBGPU_APPROX | ARBGPU_COMPLEX | ARBGPU_ALGO_LIMB | ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS |
                ARBGPU_COMPLEX_4M))
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul: unknown flags 0x%x", flags);
  const uint32_t algo = flags & (ARBGPU_ALGO_LIMB | ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS);
  if (algo & (algo - 1)) return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul: conflicting ALGO flags");
  if (p < 2 || p > (1 << 20)) return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul: p=%lld out of range", (long long)p);
  int rc;
  if ((rc = validate_mat(ctx, A, nparts, "A"))) return rc;
  if ((rc = validate_mat(ctx, B, nparts, "B"))) return rc;
  if (!C) return fail(ctx, ARBGPU_EINVAL, "C is NULL");
  if (A->cols != B->rows) return fail(ctx, ARBGPU_EINVAL, "inner dimensions differ (%lld vs %lld)",
                                      (long long)A->cols, (long long)B->rows);
  if (C->rows != A->rows || C->cols != B->cols) return fail(ctx, ARBGPU_EINVAL, "C has the wrong shape");
  const arbgpu_out *cparts[2] = {&C->re, &C->im};
  for (int q = 0; q < nparts; ++q) {
    if (!out_ok(*cparts[q], p, approx)) return fail(ctx, ARBGPU_EINVAL, "C: bad output array (cap, pointers)");
    int64_t lo, hi;
    index_range(C->off, C->rows, C->rs, C->cols, C->cs, &lo, &hi);
    if (C->rows > 0 && C->cols > 0 && !range_ok(lo, hi, cparts[q]->ld))
      return fail(ctx, ARBGPU_EINVAL, "C: element index out of range");
  }
  return ARBGPU_OK;
}

}  // namespace arbgpu_impl

extern "C" {

int arbgpu_mat_mul(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p,
                   uint32_t flags, arbgpu_stream stream) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  int rc = mat_mul_check(ctx, C, A, B, p, flags);
  if (rc) return rc;
  if (C->rows == 0 || C->cols == 0) return ARBGPU_OK;
  if ((rc = bind_device(ctx, stream))) return rc;
  return mat_mul_run(ctx, C, A, B, p, flags, to_stream(stream));
}

}  // extern "C"

namespace arbgpu_impl {

// Seconds the limb kernel needs for a product, from measured rates: a wave
// per entry below kMmWaveEntries entries (about 30 us per part to start,
// then (3.5e-11 + 3.6e-13 w^2) s per real term at full occupancy, w the
// operand limbs that reach the window), one lane per entry above
// ((7e-12 + 2e-13 w^2) s per term).
double limb_mm_seconds(int64_t M, int64_t N, int64_t K, int64_t p, int cap, bool cplx) {
  const double w = (double)std::min<int64_t>(cap, (p + 64 + 31) / 32);
  const double entries = (double)M * (double)K, nparts = cplx ? 2.0 : 1.0;
  const double terms = entries * (double)N * nparts;   // per part
  if (M * K < kMmWaveEntries) return nparts * (30e-6 + terms * (3.5e-11 + 3.6e-13 * w * w));
  return nparts * terms * (7e-12 + 2e-13 * w * w);
}

// The least the scaled-integer path takes for any product (statistics,
// slicing, product, reconstruction and their launches), real and complex.
constexpr double kInt8FloorReal = 180e-6, kInt8FloorComplex = 250e-6;

int mat_mul_run(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p,
                uint32_t flags, hipStream_t stream, int choice) {
  int rc;
  if (choice == kChoiceRule && !(flags & (ARBGPU_ALGO_LIMB | ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS)) &&
      !ctx->tune.empty()) {
    auto it = ctx->tune.find(mat_mul_class(A, B, p, flags));
    if (it != ctx->tune.end()) choice = it->second;
  }
  const bool approx = flags & ARBGPU_APPROX;
  const bool cplx = flags & ARBGPU_COMPLEX;
  const int nparts = cplx ? 2 : 1;
  const arbgpu_out *cparts[2] = {&C->re, &C->im};
  int cap = A->re.cap > B->re.cap ? A->re.cap : B->re.cap;
  if (cplx) {
    cap = A->im.cap > cap ? A->im.cap : cap;
    cap = B->im.cap > cap ? B->im.cap : cap;
  }
  LimbShape sh;
  const bool limb_ok = limb_shape_for((int)p, A->cols * nparts, cap, &sh);
  // automatic choice: products the limb kernel finishes before the
  // scaled-integer path could start go to the limb kernel
  if (limb_ok && choice == kChoiceRule && !(flags & (ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS)) &&
      limb_mm_seconds(A->rows, A->cols, B->cols, p, cap, cplx) < (cplx ? kInt8FloorComplex : kInt8FloorReal))
    choice = kChoiceLimb;
  if (!(flags & ARBGPU_ALGO_LIMB) && !(choice == kChoiceLimb && limb_ok)) {
    // the scaled-integer path, forced when asked for or when the limb
    // kernel's window cannot hold the precision
    rc = sliced_mat_mul(ctx, C, A, B, p, flags, stream,
                        (flags & (ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS)) != 0 || !limb_ok, choice);
    if (rc != kNotApplicable) return rc;
  }
  if (!limb_ok)
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul: precision %lld above the limb kernel's window", (long long)p);
  for (int q = 0; q < nparts; ++q) {
    MmParams prm;
    memset(&prm, 0, sizeof prm);
    prm.A[0] = A->re;
    prm.A[1] = cplx ? A->im : A->re;
    prm.B[0] = B->re;
    prm.B[1] = cplx ? B->im : B->re;
    prm.C = *cparts[q];
    prm.M = A->rows;
    prm.N = A->cols;
    prm.K = B->cols;
    prm.a_off = A->off; prm.a_rs = A->rs; prm.a_cs = A->cs;
    prm.b_off = B->off; prm.b_rs = B->rs; prm.b_cs = B->cs;
    prm.c_off = C->off; prm.c_rs = C->rs; prm.c_cs = C->cs;
    prm.p = (int)p;
    prm.approx = approx;
    prm.ct = !cplx ? comp_real() : (q == 0 ? comp_re() : comp_im());
    KernelTimer kt(ctx, "limb_mm", stream);
    hipError_t e = launch_limb_mm(prm, sh, stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "arbgpu_mat_mul launch");
  }
  return ARBGPU_OK;
}

}  // namespace arbgpu_impl

extern "C" {

int arbgpu_plan_blocks(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags,
                       int64_t *bounds, int32_t *kinds, int64_t max_blocks, int64_t *nblocks, arbgpu_stream stream) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (flags & ~ARBGPU_COMPLEX) return fail(ctx, ARBGPU_EINVAL, "arbgpu_plan_blocks: unknown flags 0x%x", flags);
  const int nparts = (flags & ARBGPU_COMPLEX) ? 2 : 1;
  if (p < 2 || p > (1 << 20)) return fail(ctx, ARBGPU_EINVAL, "arbgpu_plan_blocks: p=%lld out of range", (long long)p);
  if (!nblocks || max_blocks < 0 || (max_blocks > 0 && (!bounds || !kinds)))
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_plan_blocks: bad output arrays");
  int rc;
  if ((rc = validate_mat(ctx, A, nparts, "A"))) return rc;
  if ((rc = validate_mat(ctx, B, nparts, "B"))) return rc;
  if (A->cols != B->rows) return fail(ctx, ARBGPU_EINVAL, "inner dimensions differ (%lld vs %lld)",
                                      (long long)A->cols, (long long)B->rows);
  *nblocks = 0;
  if (A->cols == 0) return ARBGPU_OK;
  if ((rc = bind_device(ctx, stream))) return rc;
  return plan_partition(ctx, A, B, p, flags, to_stream(stream), bounds, kinds, max_blocks, nblocks);
}

int arbgpu_mat_mul_noalloc(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B,
                           int64_t p, uint32_t flags, arbgpu_stream stream) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  int rc = mat_mul_check(ctx, C, A, B, p, flags);
  if (rc) return rc;
  if (C->rows == 0 || C->cols == 0) return ARBGPU_OK;
  if ((rc = bind_device(ctx, stream))) return rc;
  const size_t need = mat_mul_footprint(A, B, p, flags), have = noalloc_scratch_bytes();
  if (need > have)
    return fail(ctx, ARBGPU_EINVAL,
                "arbgpu_mat_mul_noalloc: the product may take %zu bytes of workspace; the fixed scratch holds %zu",
                need, have);
  char *base = noalloc_scratch(ctx->device);
  arbgpu_ctx *v = ctx->noalloc_view;
  if (!base || !v) return fail(ctx, ARBGPU_EDEVICE, "arbgpu_mat_mul_noalloc: no scratch on device %d", ctx->device);
  // every buffer of this call is cut afresh from the scratch, whose
  // contents the previous call left: the residue tables are uploaded again
  for (auto &b : v->ws) b = arbgpu_ctx::Buf{nullptr, 0, false};
  v->bump_base = base;
  v->bump_size = have;
  v->bump_top = 0;
  v->rns_key = -1;
  v->err.clear();
  rc = mat_mul_run(v, C, A, B, p, flags, to_stream(stream));
  if (rc) ctx->err = v->err;
  memcpy(ctx->last_plan, v->last_plan, sizeof ctx->last_plan);
  return rc;
}

int arbgpu_tune_mat_mul(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p,
                        uint32_t flags, arbgpu_stream stream, int32_t *choice) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (flags & (ARBGPU_ALGO_LIMB | ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS))
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_tune_mat_mul: ALGO flags fix the path; nothing to tune");
  int rc = mat_mul_check(ctx, C, A, B, p, flags);
  if (rc) return rc;
  if (C->rows == 0 || C->cols == 0 || A->cols == 0)
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_tune_mat_mul: empty product");
  if ((rc = bind_device(ctx, stream))) return rc;
  const hipStream_t s = to_stream(stream);
  const bool cplx = flags & ARBGPU_COMPLEX;
  int cap = std::max(A->re.cap, B->re.cap);
  if (cplx) cap = std::max(cap, std::max(A->im.cap, B->im.cap));
  LimbShape ls;
  const bool limb_ok = limb_shape_for((int)p, A->cols * (cplx ? 2 : 1), cap, &ls);
  // the limb kernel's work: (window-limb products per term) x terms; far
  // beyond the INT8 path it is not timed
  const double w = (double)std::min<int64_t>(cap, (p + 31) / 32 + 2);
  const double limb_work = (double)A->rows * B->cols * A->cols * (cplx ? 4 : 1) * w * w;
  std::vector<int> cand;
  if (limb_ok && limb_work < 4e10) cand.push_back(kChoiceLimb);
  cand.push_back(kChoiceSlices);
  cand.push_back(kChoiceRns256);
  cand.push_back(kChoiceRns128);
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
    return fail(ctx, ARBGPU_EDEVICE, "arbgpu_tune_mat_mul: hipEventCreate");
  int best = kChoiceRule;
  float tbest = 0.f;
  for (int c : cand) {
    // one untimed call (it sizes the workspace), then two timed
    if (mat_mul_run(ctx, C, A, B, p, flags, s, c) != ARBGPU_OK) continue;
    float ms = 0.f;
    bool ok = hipEventRecord(ev[0], s) == hipSuccess;
    for (int r = 0; r < 2 && ok; ++r) ok = mat_mul_run(ctx, C, A, B, p, flags, s, c) == ARBGPU_OK;
    ok = ok && hipEventRecord(ev[1], s) == hipSuccess && hipEventSynchronize(ev[1]) == hipSuccess &&
         hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess;
    if (ok && (best == kChoiceRule || ms < tbest)) {
      best = c;
      tbest = ms;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (best == kChoiceRule) return fail(ctx, ARBGPU_EDEVICE, "arbgpu_tune_mat_mul: no path ran: %s", ctx->err.c_str());
  ctx->err.clear();
  ctx->tune[mat_mul_class(A, B, p, flags)] = best;
  if (!ctx->tune_path.empty()) tune_save(ctx);
  if (choice) *choice = best;
  return ARBGPU_OK;
}

int arbgpu_reserve(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (flags & ~(ARBGPU_APPROX | ARBGPU_COMPLEX | ARBGPU_ALGO_LIMB | ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS |
                ARBGPU_COMPLEX_4M))
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_reserve: unknown flags 0x%x", flags);
  if (p < 2 || p > (1 << 20)) return fail(ctx, ARBGPU_EINVAL, "arbgpu_reserve: p=%lld out of range", (long long)p);
  const int nparts = (flags & ARBGPU_COMPLEX) ? 2 : 1;
  int rc;
  if ((rc = validate_mat(ctx, A, nparts, "A"))) return rc;
  if ((rc = validate_mat(ctx, B, nparts, "B"))) return rc;
  if (A->cols != B->rows) return fail(ctx, ARBGPU_EINVAL, "inner dimensions differ (%lld vs %lld)",
                                      (long long)A->cols, (long long)B->rows);
  if (ctx->device < 0) return fail(ctx, ARBGPU_EDEVICE, "host-only context cannot hold a workspace");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  size_t sz[WS_COUNT];
  mat_mul_ws_sizes(A, B, p, flags, sz);
  return ws_reserve(ctx, sz);
}

int arbgpu_mat_mul_footprint(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags,
                             size_t *bytes) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!bytes) return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul_footprint: NULL output");
  if (flags & ~(ARBGPU_APPROX | ARBGPU_COMPLEX | ARBGPU_ALGO_LIMB | ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS |
                ARBGPU_COMPLEX_4M))
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul_footprint: unknown flags 0x%x", flags);
  if (p < 2 || p > (1 << 20))
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul_footprint: p=%lld out of range", (long long)p);
  const int nparts = (flags & ARBGPU_COMPLEX) ? 2 : 1;
  int rc;
  if ((rc = validate_mat(ctx, A, nparts, "A"))) return rc;
  if ((rc = validate_mat(ctx, B, nparts, "B"))) return rc;
  if (A->cols != B->rows) return fail(ctx, ARBGPU_EINVAL, "inner dimensions differ (%lld vs %lld)",
                                      (long long)A->cols, (long long)B->rows);
  *bytes = mat_mul_footprint(A, B, p, flags);
  return ARBGPU_OK;
}

int arbgpu_mat_mul_exact_t(arbgpu_ctx *ctx, uint32_t *T_re, uint32_t *T_im, int64_t ldT, int32_t capT,
                           int32_t *row_v2, int32_t *col_v2, const arbgpu_mat *A, const arbgpu_mat *B,
                           uint32_t flags, arbgpu_stream stream) {
  if (!ctx) return ARBGPU_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (flags & ~(ARBGPU_COMPLEX | ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS | ARBGPU_COMPLEX_4M))
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul_exact_t: unknown flags 0x%x", flags);
  if ((flags & ARBGPU_ALGO_SLICED) && (flags & ARBGPU_ALGO_RNS))
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul_exact_t: conflicting ALGO flags");
  const int nparts = (flags & ARBGPU_COMPLEX) ? 2 : 1;
  int rc;
  if ((rc = validate_mat(ctx, A, nparts, "A"))) return rc;
  if ((rc = validate_mat(ctx, B, nparts, "B"))) return rc;
  if (A->cols != B->rows) return fail(ctx, ARBGPU_EINVAL, "inner dimensions differ (%lld vs %lld)",
                                      (long long)A->cols, (long long)B->rows);
  if (!T_re || (nparts == 2 && !T_im) || !row_v2 || !col_v2 || capT < 1 || ldT < 0)
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul_exact_t: bad output arguments");
  if (A->rows == 0 || B->cols == 0 || A->cols == 0)
    return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul_exact_t: empty product");
  if (ldT < A->rows * B->cols) return fail(ctx, ARBGPU_EINVAL, "arbgpu_mat_mul_exact_t: ldT below rows * cols");
  if ((rc = bind_device(ctx, stream))) return rc;
  return exact_block_product(ctx, T_re, T_im, ldT, capT, row_v2, col_v2, A, B, flags, to_stream(stream));
}

}  // extern "C"
