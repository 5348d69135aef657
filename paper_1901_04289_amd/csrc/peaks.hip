// Microbenchmarks of the machine limits the kernels are measured against:
// dense INT8 and FP64 matrix-core throughput, HBM bandwidth (copy and
// read), the vector ALU's 32-bit integer multiply throughput (the limb
// kernels' 32x32->64 products and the residue kernels' Barrett steps), and
// the shader clock while the matrix cores are busy.  Every kernel keeps its
// working set in registers or streams a caller-provided buffer; all
// indexes stay inside the layout checked on the host.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include "arbgpu.h"
#include "internal.hpp"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;          // 4 waves per workgroup
constexpr int kComputeBlocks = 2048;   // 8 workgroups (32 waves) per CU on 256 CUs
constexpr int kCopyBlocks = 8192, kCopyUnroll = 4;   // 16-byte loads in flight per lane
constexpr int kReadBlocks = 2048, kReadUnroll = 8;
constexpr int kChains = 8;             // independent accumulators per lane

// Buffer layout: per-thread sinks, per-wave clock pairs, then the two
// streaming halves.
constexpr size_t kSinkBytes = (size_t)kComputeBlocks * kThreads * 4;   // 2 MiB
constexpr size_t kClockOff = kSinkBytes;
constexpr size_t kClockBytes = (size_t)kComputeBlocks * (kThreads / 64) * 16;
constexpr size_t kDataOff = 8u << 20;
constexpr size_t kHalfGrain = (size_t)kCopyBlocks * kThreads * kCopyUnroll * 16;   // 128 MiB
static_assert(kHalfGrain % ((size_t)kReadBlocks * kThreads * kReadUnroll * 16) == 0, "read chunks");

__global__ __launch_bounds__(kThreads) void probe_mfma_i8(uint32_t *sink, uint64_t *clk, int iters, int seed) {
  const int t = threadIdx.x;
  const v4i a = {seed ^ t, seed + t, 3 * seed + t, t};
  const v4i b = {t, seed, seed ^ 7, t + 1};
  v16i acc[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) acc[j] = v16i{} + j;
  const uint64_t c0 = clock64(), r0 = wall_clock64();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[j], 0, 0, 0);
  }
  const uint64_t c1 = clock64(), r1 = wall_clock64();
  int s = 0;
#pragma unroll
  for (int j = 0; j < kChains; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[j][e];
  const int g = blockIdx.x * kThreads + t;
  sink[g] = (uint32_t)s;
  if ((t & 63) == 0) {
    clk[2 * (g >> 6)] = c1 - c0;
    clk[2 * (g >> 6) + 1] = r1 - r0;
  }
}

__global__ __launch_bounds__(kThreads) void probe_mfma_f64(uint32_t *sink, int iters, int seed) {
  const int t = threadIdx.x;
  const double a = 1.0 + (t + seed) * 0x1p-12, b = 0.5 - t * 0x1p-14;
  v4d acc[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) acc[j] = v4d{} + (double)j;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  sink[blockIdx.x * kThreads + t] = (uint32_t)__double2loint(s);
}

// x <- lo32(x) * m + x: one v_mad_u64_u32 per step.
__global__ __launch_bounds__(kThreads) void probe_mad_u64(uint32_t *sink, int iters, uint32_t m) {
  const int t = threadIdx.x;
  uint64_t x[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) x[j] = ((uint64_t)(t + 977 * j) << 7) | (uint64_t)j;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = (uint64_t)(uint32_t)x[j] * m + x[j];
  }
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s ^= x[j];
  sink[blockIdx.x * kThreads + t] = (uint32_t)(s ^ (s >> 32));
}

// y <- high 32 bits of y * m: one v_mul_hi_u32 per step.
__global__ __launch_bounds__(kThreads) void probe_mul_hi(uint32_t *sink, int iters, uint32_t m) {
  const int t = threadIdx.x;
  uint32_t y[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) y[j] = 0xF0000000u | (uint32_t)(t * 131 + j);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) y[j] = __umulhi(y[j], m);
  }
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s ^= y[j];
  sink[blockIdx.x * kThreads + t] = s;
}

// Each workgroup streams its own contiguous chunk of `per_block` 16-byte
// vectors, a multiple of U * kThreads, so every index stays in its chunk.
// Nontemporal accesses (the data is touched once) and whole-chunk streams
// measured fastest among grid-strided, unrolled and chunked forms.
template <int U>
__global__ __launch_bounds__(kThreads) void probe_copy(const v4u *__restrict__ src, v4u *__restrict__ dst,
                                                       int64_t per_block) {
  const v4u *p = src + blockIdx.x * per_block;
  v4u *q = dst + blockIdx.x * per_block;
  for (int64_t i = threadIdx.x; i < per_block; i += U * kThreads) {
    v4u v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(p + i + u * kThreads);
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], q + i + u * kThreads);
  }
}

template <int U>
__global__ __launch_bounds__(kThreads) void probe_read(const v4u *__restrict__ src, uint32_t *sink,
                                                       int64_t per_block) {
  const v4u *p = src + blockIdx.x * per_block;
  uint32_t s = 0;
  for (int64_t i = threadIdx.x; i < per_block; i += U * kThreads) {
    v4u v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = p[i + u * kThreads];
#pragma unroll
    for (int u = 0; u < U; ++u) s ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  sink[blockIdx.x * kThreads + threadIdx.x] = s;
}

// Mean milliseconds of one launch over `reps` launches after one warm-up.
template <class F>
hipError_t time_launches(hipStream_t s, int reps, F launch, double *ms) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(a, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  *ms = (double)t / reps;
  return e;
}

}  // namespace

extern "C" int arbgpu_probe_peaks(arbgpu_ctx *ctx, void *buf, size_t bytes, arbgpu_stream stream, double *out,
                                  int n) {
  using arbgpu_impl::set_error;
  if (!ctx || !buf || !out || n < 0) return set_error(ctx, ARBGPU_EINVAL, "arbgpu_probe_peaks: NULL argument");
  if (((uintptr_t)buf & 255u) != 0)
    return set_error(ctx, ARBGPU_EINVAL, "arbgpu_probe_peaks: buffer not 256-byte aligned");
  if (bytes < kDataOff + 2 * kHalfGrain)
    return set_error(ctx, ARBGPU_EINVAL, "arbgpu_probe_peaks: buffer of %zu bytes, need at least %zu", bytes,
                     kDataOff + 2 * kHalfGrain);
  if (ctx->device < 0) return set_error(ctx, ARBGPU_EDEVICE, "host-only context cannot launch work");
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  int cus = 0, wall_khz = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, ctx->device);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "hipDeviceGetAttribute: %s", hipGetErrorString(e));

  char *base = static_cast<char *>(buf);
  uint32_t *sink = reinterpret_cast<uint32_t *>(base);
  uint64_t *clk = reinterpret_cast<uint64_t *>(base + kClockOff);
  static_assert(kClockOff + kClockBytes <= kDataOff, "clock records overlap the streamed data");
  const size_t half = (bytes - kDataOff) / 2 / kHalfGrain * kHalfGrain;
  const int64_t nvec = (int64_t)(half / 16);
  const v4u *src = reinterpret_cast<const v4u *>(base + kDataOff);
  v4u *dst = reinterpret_cast<v4u *>(base + kDataOff + half);
  const int reps = 5;
  double r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double ms = 0.0;

  // Dense INT8 matrix cores: 32x32x32 multiply-adds = 65536 operations.
  const int it_i8 = 2048;
  e = time_launches(s, reps, [&] {
    probe_mfma_i8<<<kComputeBlocks, kThreads, 0, s>>>(sink, clk, it_i8, 1);
  }, &ms);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "int8 probe: %s", hipGetErrorString(e));
  r[0] = (double)kComputeBlocks * (kThreads / 64) * it_i8 * kChains * 65536.0 / (ms * 1e-3) / 1e12;

  // Shader clock: cycle counter over the constant-rate counter, per wave of
  // the last launch.
  {
    const int nw = kComputeBlocks * (kThreads / 64);
    uint64_t *h = new uint64_t[2 * (size_t)nw];
    e = hipMemcpyAsync(h, clk, sizeof(uint64_t) * 2 * nw, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    double cyc = 0.0, rt = 0.0;
    for (int w = 0; w < nw; ++w) {
      cyc += (double)h[2 * w];
      rt += (double)h[2 * w + 1];
    }
    delete[] h;
    if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "clock readback: %s", hipGetErrorString(e));
    r[6] = rt > 0.0 ? cyc / rt * (wall_khz * 1e-3) : 0.0;
  }

  // FP64 matrix cores: 16x16x4 multiply-adds = 2048 flops.
  const int it_f64 = 1024;
  e = time_launches(s, reps, [&] {
    probe_mfma_f64<<<kComputeBlocks, kThreads, 0, s>>>(sink, it_f64, 1);
  }, &ms);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "fp64 probe: %s", hipGetErrorString(e));
  r[1] = (double)kComputeBlocks * (kThreads / 64) * it_f64 * kChains * 2048.0 / (ms * 1e-3) / 1e12;

  // HBM: copy (bytes read plus bytes written) and read-only.
  e = time_launches(s, reps, [&] {
    probe_copy<kCopyUnroll><<<kCopyBlocks, kThreads, 0, s>>>(src, dst, nvec / kCopyBlocks);
  }, &ms);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "copy probe: %s", hipGetErrorString(e));
  r[2] = 2.0 * (double)half / (ms * 1e-3) / 1e9;
  e = time_launches(s, reps, [&] {
    probe_read<kReadUnroll><<<kReadBlocks, kThreads, 0, s>>>(src, sink, nvec / kReadBlocks);
  }, &ms);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "read probe: %s", hipGetErrorString(e));
  r[3] = (double)half / (ms * 1e-3) / 1e9;

  // Vector ALU multiplies, counted per lane.
  const int it_valu = 4096;
  const double lanes = (double)kComputeBlocks * kThreads * it_valu * kChains;
  e = time_launches(s, reps, [&] {
    probe_mad_u64<<<kComputeBlocks, kThreads, 0, s>>>(sink, it_valu, 0x9E3779B9u);
  }, &ms);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "mad_u64 probe: %s", hipGetErrorString(e));
  r[4] = lanes / (ms * 1e-3) / 1e9;
  e = time_launches(s, reps, [&] {
    probe_mul_hi<<<kComputeBlocks, kThreads, 0, s>>>(sink, it_valu, 0xFFFFFFF1u);
  }, &ms);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "mul_hi probe: %s", hipGetErrorString(e));
  r[5] = lanes / (ms * 1e-3) / 1e9;
  r[7] = (double)cus;

  for (int i = 0; i < n; ++i) out[i] = i < 8 ? r[i] : 0.0;
  return ARBGPU_OK;
}
