// Host orchestration of the scaled-integer INT8-MFMA matrix product
// (Algorithm 2, Johansson 2019, Section 4): statistics, block decision,
// slicing, diagonal-group schedule, MFMA product, recombination and the
// radius products.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sliced.hpp"

namespace arbgpu_impl {

namespace {

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

}  // namespace

int sliced_mat_mul(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p,
                   uint32_t flags, hipStream_t s, bool forced) {
  const bool cplx = flags & ARBGPU_COMPLEX;
  const bool approx = flags & ARBGPU_APPROX;
  const int nparts = cplx ? 2 : 1;
  const int64_t M = A->rows, N = B->cols, K = A->cols;     // C is M x N, inner K
  const int64_t Kt = cplx ? 2 * K : K;                     // inner length of the real products
  // Basecase (Algorithm 2: blocks shorter than 30 use dot products).
  if (!forced && K < 30) return kNotApplicable;
  const int64_t Kp = round_up(std::max<int64_t>(Kt, 1), kKStep);
  // int32 partial planes: P pairs of Kp terms of |d d'| <= 2^14 each
  const int64_t pmax = ((int64_t)0x7FFFFFFF) / (Kp << 14);
  if (pmax < 1) {
    if (forced) return set_error(ctx, ARBGPU_EINVAL, "sliced product: inner length %lld too long", (long long)Kt);
    return kNotApplicable;
  }

  // ---- statistics ---------------------------------------------------------
  const int64_t Mp = round_up(std::max<int64_t>(M, 1), kTile), Np = round_up(std::max<int64_t>(N, 1), kTile);
  size_t st_bytes = sizeof(int32_t) * (size_t)(2 * M + 2 * N + 8);
  int32_t *st = (int32_t *)ws_get(ctx, WS_STATS, st_bytes);
  if (!st) return ARBGPU_ENOMEM;
  int32_t *rtop = st, *rv2 = st + M, *ctop = st + 2 * M, *cv2 = st + 2 * M + N;
  int32_t *gA = st + 2 * M + 2 * N, *gB = gA + 4;
  hipError_t e = launch_fill_i32(gA, 0, 8, s);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "fill: %s", hipGetErrorString(e));
  StatsParams sp;
  memset(&sp, 0, sizeof sp);
  sp.part[0] = A->re;
  sp.part[1] = cplx ? A->im : A->re;
  sp.nparts = nparts;
  sp.lines = M; sp.len = K; sp.off = A->off; sp.line_stride = A->rs; sp.elem_stride = A->cs; sp.k0 = 0;
  sp.out = LineStats{rtop, rv2};
  sp.gmax = gA;
  StatsParams sq = sp;
  sq.part[0] = B->re;
  sq.part[1] = cplx ? B->im : B->re;
  sq.lines = N; sq.len = K; sq.off = B->off; sq.line_stride = B->cs; sq.elem_stride = B->rs;
  sq.out = LineStats{ctop, cv2};
  sq.gmax = gB;
  {
    KernelTimer t_stats(ctx, "stats", s);
    if ((e = launch_stats_rows(sp, s)) == hipSuccess) e = launch_stats_cols(sq, s);
  }
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "stats: %s", hipGetErrorString(e));
  int32_t g[8];
  if ((e = hipMemcpyAsync(g, gA, sizeof g, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return set_error(ctx, ARBGPU_EDEVICE, "stats readback: %s", hipGetErrorString(e));
  const int HA = g[0], HB = g[4];
  const int pA = g[1], pB = g[5];
  if (g[2] || g[6]) return kNotApplicable;   // out-of-range exponents: flagged per entry by the limb kernel
  // Height bound of Algorithm 2: h = 1.25 min(p, max(p_A, p_B)) + 192.  With
  // every line below it the whole inner range is one block.
  const double h = 1.25 * (double)std::min<int64_t>(p, std::max(pA, pB)) + 192.0;
  if (!forced && (HA > h || HB > h)) return kNotApplicable;
  const int LA = std::max(1, (HA + 1 + 7) / 8), LB = std::max(1, (HB + 1 + 7) / 8);
  if (LA > kMaxSlices || LB > kMaxSlices) {
    if (forced) return set_error(ctx, ARBGPU_EINVAL, "sliced product: integer height %d too large", std::max(HA, HB));
    return kNotApplicable;
  }

  // ---- diagonal-group schedule --------------------------------------------
  const int Lc = LA + LB - 1;
  std::vector<DiagGroup> groups;
  std::vector<int32_t> slot_of(Lc + 1, 0);
  int nslots = 0;
  for (int c = 0; c < Lc; ++c) {
    const int lo = std::max(0, c - LB + 1), hi = std::min(c, LA - 1) + 1;
    slot_of[c] = nslots;
    const int np = hi - lo;
    const int nch = (int)((np + pmax - 1) / pmax);
    const int per = (np + nch - 1) / nch;   // balanced chunks
    for (int a0 = lo; a0 < hi; a0 += per) groups.push_back(DiagGroup{c, a0, std::min(hi, a0 + per), nslots++});
  }
  slot_of[Lc] = nslots;
  std::stable_sort(groups.begin(), groups.end(),
                   [](const DiagGroup &x, const DiagGroup &y) { return (x.a1 - x.a0) > (y.a1 - y.a0); });
  const int ngroups_real = (int)groups.size();
  while (groups.size() % 8) groups.push_back(DiagGroup{0, 0, 0, -1});   // padding for the XCD mapping
  const int nq = (Lc + 3) / 4, nT = nq + 2;
  {
    const int64_t plan[8] = {LA, LB, nslots, ngroups_real, Kt, M, N, nparts};
    memcpy(ctx->last_plan, plan, sizeof plan);
  }

  // ---- workspace ------------------------------------------------------------
  const size_t bytesA = (size_t)LA * Mp * Kp, bytesB = (size_t)LB * Np * Kp;
  int8_t *planesA = (int8_t *)ws_get(ctx, WS_PLANES_A, bytesA);
  int8_t *planesB = (int8_t *)ws_get(ctx, WS_PLANES_B, bytesB);
  int8_t *planesB2 = cplx ? (int8_t *)ws_get(ctx, WS_PLANES_B2, bytesB) : nullptr;
  int32_t *D = (int32_t *)ws_get(ctx, WS_D, sizeof(int32_t) * (size_t)nslots * M * N);
  uint32_t *T = (uint32_t *)ws_get(ctx, WS_T, sizeof(uint32_t) * (size_t)nT * M * N);
  const size_t tab_bytes = sizeof(DiagGroup) * groups.size() + sizeof(int32_t) * slot_of.size();
  char *tabs = (char *)ws_get(ctx, WS_TABLES, tab_bytes);
  if (!planesA || !planesB || (cplx && !planesB2) || !D || !T || !tabs) return ARBGPU_ENOMEM;
  DiagGroup *dgroups = (DiagGroup *)tabs;
  int32_t *dslot = (int32_t *)(tabs + sizeof(DiagGroup) * groups.size());
  if ((e = hipMemcpyAsync(dgroups, groups.data(), sizeof(DiagGroup) * groups.size(), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(dslot, slot_of.data(), sizeof(int32_t) * slot_of.size(), hipMemcpyHostToDevice, s)) !=
          hipSuccess)
    return set_error(ctx, ARBGPU_EDEVICE, "table upload: %s", hipGetErrorString(e));

  // ---- radius products (ball inputs only) -----------------------------------
  const bool radA = A->re.rad_m || (cplx && A->im.rad_m);
  const bool radB = B->re.rad_m || (cplx && B->im.rad_m);
  const bool want_rad = !approx && (radA || radB);
  double *rad_out_m[2] = {nullptr, nullptr};
  int32_t *rad_out_e[2] = {nullptr, nullptr};
  if (want_rad) {
    const size_t na = (size_t)M * Kt, nb = (size_t)N * Kt;
    char *ra = (char *)ws_get(ctx, WS_RAD_A, 2 * sizeof(double) * na + sizeof(int32_t) * M);
    char *rb = (char *)ws_get(ctx, WS_RAD_B, 2 * sizeof(double) * nb + sizeof(int32_t) * N);
    char *ro = (char *)ws_get(ctx, WS_RAD_OUT, (size_t)nparts * (sizeof(double) + sizeof(int32_t)) * M * N);
    if (!ra || !rb || !ro) return ARBGPU_ENOMEM;
    RadPrepParams pa;
    memset(&pa, 0, sizeof pa);
    pa.part[0] = A->re;
    pa.part[1] = cplx ? A->im : A->re;
    pa.nparts = nparts;
    pa.lines = M; pa.len = K; pa.off = A->off; pa.line_stride = A->rs; pa.elem_stride = A->cs;
    pa.mode = cplx ? 3 : 0;
    pa.side = 0;
    pa.v0 = (double *)ra;
    pa.v1 = (double *)ra + na;
    pa.scale = (int32_t *)((double *)ra + 2 * na);
    if ((e = launch_rad_prep(pa, s)) != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "rad prep: %s", hipGetErrorString(e));
    for (int q = 0; q < nparts; ++q) {
      RadPrepParams pb;
      memset(&pb, 0, sizeof pb);
      pb.part[0] = B->re;
      pb.part[1] = cplx ? B->im : B->re;
      pb.nparts = nparts;
      pb.lines = N; pb.len = K; pb.off = B->off; pb.line_stride = B->cs; pb.elem_stride = B->rs;
      pb.mode = !cplx ? 0 : (q == 0 ? 1 : 2);
      pb.side = 1;
      pb.v0 = (double *)rb;
      pb.v1 = (double *)rb + nb;
      pb.scale = (int32_t *)((double *)rb + 2 * nb);
      if ((e = launch_rad_prep(pb, s)) != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "rad prep: %s", hipGetErrorString(e));
      RadGemmParams rg;
      rg.a_m = pa.v0; rg.a_r = pa.v1; rg.b_mr = pb.v0; rg.b_r = pb.v1;
      rg.a_s = pa.scale; rg.b_s = pb.scale;
      rg.M = M; rg.N = N; rg.Kt = Kt;
      rad_out_m[q] = (double *)ro + (size_t)q * M * N;
      rad_out_e[q] = (int32_t *)((double *)ro + (size_t)nparts * M * N) + (size_t)q * M * N;
      rg.out_m = rad_out_m[q];
      rg.out_e = rad_out_e[q];
      KernelTimer tg(ctx, "rad_gemm", s);
      if ((e = launch_rad_gemm(rg, s)) != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "rad gemm: %s", hipGetErrorString(e));
    }
  }

  // ---- slicing ----------------------------------------------------------------
  SliceParams sa;
  memset(&sa, 0, sizeof sa);
  sa.part[0] = A->re;
  sa.part[1] = cplx ? A->im : A->re;
  sa.lines = M; sa.len = K; sa.off = A->off; sa.line_stride = A->rs; sa.elem_stride = A->cs; sa.k0 = 0;
  sa.mode = cplx ? 3 : 0;
  sa.lines_pad = Mp; sa.k_pad = Kp; sa.L = LA; sa.v2 = rv2; sa.planes = planesA;
  {
    KernelTimer t_slice(ctx, "slice", s);
    e = launch_slice(sa, s);
    for (int q = 0; q < nparts && e == hipSuccess; ++q) {
      SliceParams sb = sa;
      sb.part[0] = B->re;
      sb.part[1] = cplx ? B->im : B->re;
      sb.lines = N; sb.off = B->off; sb.line_stride = B->cs; sb.elem_stride = B->rs;
      sb.mode = !cplx ? 0 : (q == 0 ? 1 : 2);
      sb.lines_pad = Np; sb.L = LB; sb.v2 = cv2; sb.planes = q == 0 ? planesB : planesB2;
      e = launch_slice(sb, s);
    }
  }
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "slice: %s", hipGetErrorString(e));

  // ---- product and recombination per output part ------------------------------
  const arbgpu_out *cparts[2] = {&C->re, &C->im};
  for (int q = 0; q < nparts; ++q) {
    MfmaParams mp;
    mp.A = planesA;
    mp.B = q == 0 ? planesB : planesB2;
    mp.D = D;
    mp.groups = dgroups;
    mp.M = M; mp.N = N; mp.Mp = Mp; mp.Np = Np; mp.Kp = Kp;
    mp.ntm = (int)(Mp / kTile); mp.ntn = (int)(Np / kTile);
    mp.ngroups = (int)groups.size();
    hipError_t em;
    {
      KernelTimer tm(ctx, "mfma", s);
      em = launch_mfma(mp, s);
    }
    if ((e = em) != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "mfma: %s", hipGetErrorString(e));
    RecombParams rp;
    rp.D = D; rp.slot_of = dslot; rp.Lc = Lc; rp.M = M; rp.N = N; rp.T = T; rp.nT = nT;
    rp.rowv2 = rv2; rp.colv2 = cv2;
    rp.C = *cparts[q];
    rp.c_off = C->off; rp.c_rs = C->rs; rp.c_cs = C->cs;
    rp.p = (int)p;
    rp.approx = approx;
    rp.rin_m = rad_out_m[q];
    rp.rin_e = rad_out_e[q];
    KernelTimer tr(ctx, "recombine", s);
    if ((e = launch_recombine(rp, s)) != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "recombine: %s", hipGetErrorString(e));
  }
  return ARBGPU_OK;
}

}  // namespace arbgpu_impl
