// Host orchestration of the scaled-integer INT8-MFMA matrix product
// (Algorithm 2, Johansson 2019, Section 4): statistics, block partition,
// slicing, diagonal-group schedule, MFMA product, recombination, radius
// products, and the exact merge when the inner range splits into blocks.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sliced.hpp"

namespace arbgpu_impl {

namespace {

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Shape {
  bool cplx, approx;
  int nparts;
  int64_t M, N, K;   // C is M x N, inner dimension K (per part)
  int tile = 0;      // residue MFMA tile edge (0: rns_tile's choice)
};

#define ARB_TRY(expr, what)                                                                          \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "%s: %s", what, hipGetErrorString(e_)); \
  } while (0)

// Statistics workspace: rtop[M], rv2[M], ctop[N], cv2[N], gA[4], gB[4].
int32_t *stats_ws(arbgpu_ctx *ctx, const Shape &sh) {
  return (int32_t *)ws_get(ctx, WS_STATS, sizeof(int32_t) * (size_t)(2 * sh.M + 2 * sh.N + 8));
}

struct Lines;
int b_lines(arbgpu_ctx *ctx, const arbgpu_mat *B, bool cplx, int64_t k0, int64_t k1, hipStream_t s, Lines &L);

// Line statistics of A's rows and B's columns over the inner range [k0, k1):
// per-line lowest set bit (left in the workspace for slicing) and the
// global maxima g[0..3] (A) and g[4..7] (B) as described in StatsParams.
// Waits for the maxima to read them back.  With `pre` (not for a context
// on fixed scratch), B's lines for [k0, k1) are also prepared, their copy
// queued behind the readback so that it runs while the host waits and
// plans; *pre_ok tells whether that was done.
int line_stats(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, const Shape &sh, int64_t k0, int64_t k1,
               int32_t *st, hipStream_t s, int32_t g[8], Lines *pre = nullptr, bool *pre_ok = nullptr) {
  int32_t *rtop = st, *rv2 = st + sh.M, *ctop = st + 2 * sh.M, *cv2 = st + 2 * sh.M + sh.N;
  int32_t *gA = st + 2 * sh.M + 2 * sh.N, *gB = gA + 4;
  ARB_TRY(launch_fill_i32(gA, 0, 8, s), "fill");
  StatsParams sp;
  memset(&sp, 0, sizeof sp);
  sp.part[0] = A->re;
  sp.part[1] = sh.cplx ? A->im : A->re;
  sp.nparts = sh.nparts;
  sp.lines = sh.M; sp.len = k1 - k0; sp.off = A->off; sp.line_stride = A->rs; sp.elem_stride = A->cs; sp.k0 = k0;
  sp.out = LineStats{rtop, rv2};
  sp.gmax = gA;
  StatsParams sq = sp;
  sq.part[0] = B->re;
  sq.part[1] = sh.cplx ? B->im : B->re;
  sq.lines = sh.N; sq.off = B->off; sq.line_stride = B->cs; sq.elem_stride = B->rs;
  sq.out = LineStats{ctop, cv2};
  sq.gmax = gB;
  {
    KernelTimer t_stats(ctx, "stats", s);
    ARB_TRY(launch_stats_rows(sp, s), "stats");
    ARB_TRY(launch_stats_cols(sq, s), "stats");
  }
  if (pre_ok) *pre_ok = false;
  if (pre && ctx->bump_size == 0) {
    if (!ctx->stats_host) ARB_TRY(hipHostMalloc((void **)&ctx->stats_host, 8 * sizeof(int32_t)), "stats readback");
    if (!ctx->ev_stats) ARB_TRY(hipEventCreateWithFlags(&ctx->ev_stats, hipEventDisableTiming), "stats readback");
    ARB_TRY(hipMemcpyAsync(ctx->stats_host, gA, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s), "stats readback");
    ARB_TRY(hipEventRecord(ctx->ev_stats, s), "stats readback");
    {
      KernelTimer t_slice(ctx, "slice", s);
      const int rc = b_lines(ctx, B, sh.cplx, k0, k1, s, *pre);
      if (rc) return rc;
    }
    ARB_TRY(hipEventSynchronize(ctx->ev_stats), "stats readback");
    memcpy(g, ctx->stats_host, 8 * sizeof(int32_t));
    if (pre_ok) *pre_ok = true;
    return ARBGPU_OK;
  }
  ARB_TRY(hipMemcpyAsync(g, gA, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s), "stats readback");
  ARB_TRY(hipStreamSynchronize(s), "stats readback");
  return ARBGPU_OK;
}

// Balanced base-256 digits (each in [-128, 127]) for the scaled integers of
// a line of the given height, |Y| <= 2^height - 1.  L digits reach
// 127 (256^L - 1) / 255 above zero, a little under 256^L / 2, so they hold
// 2^h - 1 exactly when 8 L >= h + 2; the single digit of heights up to 7
// holds 127 = 2^7 - 1.  (8 L = h + 1 would turn Y = 2^h - 1 into
// Y - 256^L for every h = 8 L - 1 >= 15.)
inline int slices_for(int height) { return height <= 7 ? 1 : (height + 2 + 7) / 8; }

// B's lines (columns) for slicing the inner range [k0, k1): when the inner
// index is strided and the columns are not (row-major B), a line-major copy
// of the block, else B in place.
struct Lines {
  arbgpu_arr part[2];
  int64_t off, line_stride, elem_stride, k0;
};

int b_lines(arbgpu_ctx *ctx, const arbgpu_mat *B, bool cplx, int64_t k0, int64_t k1, hipStream_t s, Lines &L) {
  L.part[0] = B->re;
  L.part[1] = cplx ? B->im : B->re;
  L.off = B->off; L.line_stride = B->cs; L.elem_stride = B->rs; L.k0 = k0;
  const int64_t N = B->cols, Kb = k1 - k0;
  if (!(B->cs == 1 && B->rs != 1) || N == 0 || Kb == 0) return ARBGPU_OK;
  const int nparts = cplx ? 2 : 1;
  const size_t elems = (size_t)N * Kb;
  size_t bytes = 0;
  for (int q = 0; q < nparts; ++q) bytes += 4 * elems * (size_t)(L.part[q].cap + 2);
  char *w = (char *)ws_get(ctx, WS_GATHER, bytes);
  if (!w) return ARBGPU_ENOMEM;
  for (int q = 0; q < nparts; ++q) {
    GatherParams gp;
    gp.src = L.part[q];
    gp.off = B->off; gp.line_stride = B->cs; gp.elem_stride = B->rs; gp.k0 = k0;
    gp.lines = N; gp.len = Kb;
    gp.limbs = (uint32_t *)w;
    gp.exp = (int32_t *)(w + 4 * elems * (size_t)L.part[q].cap);
    gp.nls = gp.exp + elems;
    w += 4 * elems * (size_t)(L.part[q].cap + 2);
    ARB_TRY(launch_gather(gp, s), "gather");
    L.part[q] = arbgpu_arr{gp.limbs, (int64_t)elems, L.part[q].cap, gp.exp, gp.nls, nullptr, nullptr};
  }
  if (!cplx) L.part[1] = L.part[0];
  L.off = 0; L.line_stride = Kb; L.elem_stride = 1; L.k0 = 0;
  return ARBGPU_OK;
}

// B's lines for the inner range from k0 on, from lines prepared for the
// whole inner range (b_lines from 0).
int lines_of(const Lines &whole, int64_t k0, Lines &L) {
  L = whole;
  L.k0 = whole.k0 + k0;
  return ARBGPU_OK;
}

// Odd primes between 2^14 and 2^15, largest first (residue moduli).
const std::vector<int32_t> &rns_primes() {
  static const std::vector<int32_t> v = [] {
    std::vector<char> comp(1 << 15, 0);
    std::vector<int32_t> out;
    for (int i = 2; i < (1 << 15); ++i) {
      if (comp[i]) continue;
      for (int j = 2 * i; j < (1 << 15); j += i) comp[j] = 1;
    }
    for (int i = (1 << 15) - 1; i > (1 << 14); --i)
      if (!comp[i]) out.push_back(i);
    return out;
  }();
  return v;
}

// Number of primes whose product exceeds 2^bits.
int rns_count(int64_t bits) {
  // cumulative log2 of the product of the first j + 1 primes, computed once
  static const std::vector<double> cum = [] {
    const std::vector<int32_t> &pr = rns_primes();
    std::vector<double> c(pr.size());
    double acc = 0.0;
    for (size_t j = 0; j < pr.size(); ++j) c[j] = acc += log2((double)pr[j]);
    return c;
  }();
  const auto it = std::upper_bound(cum.begin(), cum.end(), (double)bits + 1.0);
  return it == cum.end() ? -1 : (int)(it - cum.begin()) + 1;
}

int64_t modinv(int64_t a, int64_t p) {   // a^-1 mod p, gcd(a, p) = 1
  int64_t t = 0, nt = 1, r = p, nr = ((a % p) + p) % p;
  while (nr) {
    const int64_t q = r / nr;
    int64_t x = t - q * nt; t = nt; nt = x;
    x = r - q * nr; r = nr; nr = x;
  }
  return t < 0 ? t + p : t;
}

// Balanced base-256 digits d_0 .. d_{n-1} (each in [-128, 128)) of X mod
// 256^n, X given as little-endian limbs.
void balanced_digits(const std::vector<uint32_t> &X, int n, int8_t *d) {
  int c = 0;
  for (int i = 0; i < n; ++i) {
    const int q = i >> 2;
    const int byte = q < (int)X.size() ? (int)((X[q] >> (8 * (i & 3))) & 0xFFu) : 0;
    const int v = byte + c;
    c = v >= 128;
    d[i] = (int8_t)(v - 256 * c);
  }
}

// Byte layout of the residue tables for m primes, nw digit words and W
// limbs of T (offsets of the arrays of RnsTables in one buffer).
struct RnsLayout {
  int kc, ncc, kd, nrt;
  size_t o_mu, o_kp, o_rp, o_c, o_cp, o_wd, o_qd, bytes;
};

RnsLayout rns_layout(int m, int nw, int W) {
  RnsLayout l;
  l.kc = (int)round_up(2 * (int64_t)m + 2, 32);
  l.ncc = (W + 7) / 8;
  l.kd = (int)round_up(4 * (int64_t)nw, 32);
  l.nrt = (m + 15) / 16;
  l.o_mu = 4 * (size_t)m;
  l.o_kp = l.o_mu + 4 * (size_t)m;
  l.o_rp = (l.o_kp + 4 * (size_t)m + 7) & ~(size_t)7;
  l.o_c = l.o_rp + 8 * (size_t)m;
  l.o_cp = (l.o_c + 4 * (size_t)m + 31) & ~(size_t)31;
  l.o_wd = (l.o_cp + sizeof(RnsCrtPrime) * (size_t)m + 15) & ~(size_t)15;
  l.o_qd = l.o_wd + (size_t)l.nrt * 32 * l.kd;
  l.bytes = l.o_qd + (size_t)l.ncc * 32 * l.kc;
  return l;
}

// Residue tables for m primes, nw words of base-256 digits and W limbs of
// T, uploaded to the context workspace (kept while m, nw and W stay the
// same): primes and reduction constants, the digit weights 256^a mod p_j
// as balanced int8 pairs, and the Chinese remainder constants
// (P / p_j)^-1 mod p_j and the digits of P / p_j and P.
int rns_tables(arbgpu_ctx *ctx, int m, int nw, int W, hipStream_t s, RnsTables &tab) {
  const std::vector<int32_t> &pr = rns_primes();
  const RnsLayout lay = rns_layout(m, nw, W);
  const int kc = lay.kc, ncc = lay.ncc, kd = lay.kd;
  const size_t o_mu = lay.o_mu, o_kp = lay.o_kp, o_rp = lay.o_rp, o_c = lay.o_c, o_cp = lay.o_cp, o_wd = lay.o_wd,
               o_qd = lay.o_qd, bytes = lay.bytes;
  char *d = (char *)ws_get(ctx, WS_RNS, bytes);
  if (!d) return ARBGPU_ENOMEM;
  tab.prime = (const int32_t *)d;
  tab.mu = (const uint32_t *)(d + o_mu);
  tab.kp = (const uint32_t *)(d + o_kp);
  tab.wd = (const int8_t *)(d + o_wd);
  tab.rp = (const double *)(d + o_rp);
  tab.c = (const uint32_t *)(d + o_c);
  tab.crt = (const RnsCrtPrime *)(d + o_cp);
  tab.qd = (const int8_t *)(d + o_qd);
  tab.m = m;
  tab.nw = nw;
  tab.kd = kd;
  tab.kc = kc;
  tab.ncc = ncc;
  const int64_t key = (int64_t)m | ((int64_t)nw << 16) | ((int64_t)W << 32);
  if (ctx->rns_key == key && ctx->ws[WS_RNS].ptr == d) return ARBGPU_OK;
  // P = prod p_j and Q_j = P / p_j as little-endian limbs
  std::vector<uint32_t> P(1, 1u);
  for (int j = 0; j < m; ++j) {
    uint64_t c = 0;
    for (auto &l : P) {
      const uint64_t t = (uint64_t)l * (uint32_t)pr[j] + c;
      l = (uint32_t)t;
      c = t >> 32;
    }
    if (c) P.push_back((uint32_t)c);
  }
  std::vector<char> h(bytes, 0);
  int32_t *hp = (int32_t *)h.data();
  uint32_t *hmu = (uint32_t *)(h.data() + o_mu);
  uint32_t *hkp = (uint32_t *)(h.data() + o_kp);
  int8_t *hwd = (int8_t *)(h.data() + o_wd);
  double *hrp = (double *)(h.data() + o_rp);
  uint32_t *hc = (uint32_t *)(h.data() + o_c);
  RnsCrtPrime *hcp = (RnsCrtPrime *)(h.data() + o_cp);
  int8_t *hqd = (int8_t *)(h.data() + o_qd);
  const int nd = 32 * ncc;                 // digit columns
  std::vector<int8_t> dig((size_t)nd + 1);
  // digits of X and of 256 X into inner rows 2i, 2i + 1 of the permuted table
  auto put = [&](int row2, const std::vector<uint32_t> &X) {
    balanced_digits(X, nd, dig.data());
    for (int cc = 0; cc < ncc; ++cc)
      for (int r = 0; r < 32; ++r) {
        const int col = 32 * cc + 16 * ((r >> 2) & 1) + 4 * (r >> 3) + (r & 3);
        int8_t *t = hqd + ((size_t)cc * 32 + r) * kc;
        t[row2] = dig[col];
        t[row2 + 1] = col > 0 ? dig[col - 1] : (int8_t)0;
      }
  };
  std::vector<uint32_t> Q(P.size());
  for (int j = 0; j < m; ++j) {
    const int64_t p = pr[j];
    hp[j] = (int32_t)p;
    hmu[j] = (uint32_t)((((uint64_t)1) << 32) / (uint64_t)p);
    hkp[j] = (uint32_t)((((int64_t)1 << 30) + p - 1) / p * p);
    hrp[j] = 1.0 / (double)p;
    // weight digits of prime j: tile j / 16, row 2 (j % 16) lo, + 1 hi
    const int rlo = 2 * (j % 16);
    int8_t *wlo = hwd + ((size_t)(j / 16) * 32 + rlo) * kd, *whi = wlo + kd;
    int64_t w = 1;   // 256^a mod p
    for (int a = 0; a < 4 * nw; ++a) {
      const int64_t bal = w > p / 2 ? w - p : w;
      const int64_t lo = ((bal + 128) & 255) - 128;
      wlo[a] = (int8_t)lo;
      whi[a] = (int8_t)((bal - lo) >> 8);
      w = w * 256 % p;
    }
    // Q_j = P / p_j (exact), its residue mod p_j, and that residue's inverse
    uint64_t rem = 0;
    for (int q = (int)P.size() - 1; q >= 0; --q) {
      const uint64_t cur = (rem << 32) | P[q];
      Q[q] = (uint32_t)(cur / (uint64_t)p);
      rem = cur % (uint64_t)p;
    }
    uint64_t qm = 0;
    for (int q = (int)P.size() - 1; q >= 0; --q) qm = ((qm << 32) | Q[q]) % (uint64_t)p;
    hc[j] = (uint32_t)modinv((int64_t)qm, p);
    RnsCrtPrime &cr = hcp[j];
    cr.p = (uint32_t)p;
    cr.mu = hmu[j];
    cr.cb = (int32_t)(hc[j] > (uint32_t)(p >> 1) ? (int64_t)hc[j] - p : (int64_t)hc[j]);
    cr.kp2 = 2u * hkp[j];
    cr.rp = hrp[j];
    cr.half = (uint32_t)(p >> 1);
    cr.pad = 0u;
    put(2 * j, Q);
  }
  put(2 * m, P);
  hipError_t e = hipMemcpyAsync(d, h.data(), bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(ctx, ARBGPU_EDEVICE, "residue tables: %s", hipGetErrorString(e));
  ctx->rns_key = key;
  return ARBGPU_OK;
}

// Two's-complement bits of the exact block value: |T| < Kt 2^(HA + HB).
int64_t t_bits(int HA, int HB, int64_t Kt) {
  int lg = 0;
  while (((int64_t)1 << lg) < std::max<int64_t>(Kt, 1)) ++lg;
  return (int64_t)HA + HB + lg + 1;
}

// Block values of `bits` two's-complement bits fit the reconstruction: the
// kernel keeps 32 entries' digit rows and limbs in LDS.
bool rns_fits_bits(int64_t bits) {
  const int m = rns_count(bits);
  if (m < 1) return false;
  const int W = (int)((bits + 1 + 31) / 32) + 1;
  return rns_crt_lds(32, (int)round_up(2 * (int64_t)m + 2, 32), W) <= kRnsCrtLds;
}

// The residue form applies when the on-chip Horner chain of the digit
// products stays below 2^31 (K_pad < 2^16), the residue sums of the slicer
// (at most 4 nw <= 508 digits) below 2^30, and the block values fit the
// reconstruction.
bool rns_fits(int HA, int HB, int64_t Kt) {
  const int64_t Kp = round_up(std::max<int64_t>(Kt, 1), kKStep);
  if (((int64_t)0x7FFFFFFF) / (Kp << 14) < 2) return false;
  const int nw = (std::max(slices_for(HA), slices_for(HB)) + 3) / 4;
  return nw <= 127 && rns_fits_bits(t_bits(HA, HB, Kt));
}

// MFMA work of the two forms (digit pairs): base-256 slices L_A L_B, the
// residue form 4 m; the residue form also pays its conversions, about the
// cost of 4 more pairs per prime at these shapes.
bool rns_better(int HA, int HB, int64_t Kt) {
  if (!rns_fits(HA, HB, Kt)) return false;
  const int64_t m = rns_count(t_bits(HA, HB, Kt));
  return 8 * m < (int64_t)slices_for(HA) * slices_for(HB);
}

int ceil_log2(int64_t v) {
  int l = 0;
  while (((int64_t)1 << l) < v) ++l;
  return l;
}

// Output tile edge of the residue MFMA kernel for an M x N result over
// `groups` (product, prime) pairs: 128 when it cuts the padded area by a
// fifth or when 256 tiles would give fewer than two work items per
// compute unit, else 256 (twice the MACs per staged byte).
int rns_tile(int64_t M, int64_t N, int64_t groups) {
  const int64_t a256 = round_up(std::max<int64_t>(M, 1), 256) * round_up(std::max<int64_t>(N, 1), 256);
  const int64_t a128 = round_up(std::max<int64_t>(M, 1), 128) * round_up(std::max<int64_t>(N, 1), 128);
  const int64_t items256 = groups * (a256 / (256 * 256));
  return (5 * a128 < 4 * a256 || items256 < 512) ? 128 : 256;
}

// Limbs of the exact block result T for the given digit-plane counts.
inline int t_limbs(int LA, int LB) { return (LA + LB - 1 + 3) / 4 + 2; }

// One scaled-integer block over the inner range [k0, k1) whose line
// statistics are in `st`: slices, MFMA product and recombination into
// out[q] (q = output part) truncated to p bits.
int rns_block_product(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, const Shape &sh, int64_t k0,
                      int64_t k1, const int32_t *st, int HA, int HB, const arbgpu_out *out, int64_t o_off,
                      int64_t o_rs, int64_t o_cs, int p, bool out_approx, double *const rin_m[2],
                      int32_t *const rin_e[2], hipStream_t s, bool four, const TSink *ts, const Lines *pre);

// Copies the exact T of output part q (limbs [n][M N] in the workspace) to
// the caller's sink, when there is one.
int t_to_sink(arbgpu_ctx *ctx, const TSink *ts, int q, const uint32_t *T, int n, int64_t mn, hipStream_t s) {
  if (!ts) return ARBGPU_OK;
  ARB_TRY(launch_t_copy(T, n, mn, ts->T[q], ts->ld, ts->cap, s), "exact T copy");
  return ARBGPU_OK;
}

// Headroom of the truncated diagonal set: the left-out diagonals stay
// below 2^(bits of |T|'s bound - p - kTruncSlack), so every entry within
// kTruncSlack - 3 bits of that bound certifies its truncation.  Entries
// further below it (cancellation) are recomputed exactly, a wave each; at
// 32 bits they are rare, and each 8 bits less leave out about one more
// diagonal of slice pairs.
constexpr int kTruncSlack = 32;

int block_product(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, const Shape &sh, int64_t k0, int64_t k1,
                  const int32_t *st, int HA, int HB, const arbgpu_out *out, int64_t o_off, int64_t o_rs, int64_t o_cs,
                  int p, bool out_approx, double *const rin_m[2], int32_t *const rin_e[2], hipStream_t s,
                  bool rns, bool four = false, const TSink *ts = nullptr, bool trunc = false,
                  const Lines *pre = nullptr) {
  if (rns)
    return rns_block_product(ctx, A, B, sh, k0, k1, st, HA, HB, out, o_off, o_rs, o_cs, p, out_approx, rin_m, rin_e,
                             s, four, ts, pre);
  const int32_t *rv2 = st + sh.M, *cv2 = st + 2 * sh.M + sh.N;
  const int64_t Kb = k1 - k0;
  const int64_t Kt = sh.cplx ? 2 * Kb : Kb;
  const int64_t Kp = round_up(std::max<int64_t>(Kt, 1), kKStep);
  // int32 partial planes: P pairs of Kp terms of |d d'| <= 2^14 each
  const int64_t pmax = ((int64_t)0x7FFFFFFF) / (Kp << 14);
  const int64_t Mp = round_up(std::max<int64_t>(sh.M, 1), kTile), Np = round_up(std::max<int64_t>(sh.N, 1), kTile);
  const int LA = slices_for(HA), LB = slices_for(HB);

  const int Lc = LA + LB - 1;
  // The truncated diagonal set (the slice-pair analogue of the products
  // truncated below the window, Section 3.4): the diagonals c < c0, whose
  // total sum_{c < c0} 256^c D_c (|D_c| <= pairs_c K_pad 2^14) stays below
  // 2^ebits, are left out when that is far below the p bits the output
  // keeps; the recombination certifies each entry's truncation against
  // 2^ebits, and entries it cannot certify are recomputed exactly.
  int c0 = 0, ebits = -1;
  LimbShape fb_shape{0, 0};
  if (trunc && !ts) {
    int cap = std::max(A->re.cap, B->re.cap);
    if (sh.cplx) cap = std::max(cap, std::max(A->im.cap, B->im.cap));
    const int64_t limit = t_bits(HA, HB, Kt) - p - kTruncSlack;
    double sc = 0.0;   // sum_{c' <= c} pairs_c' 256^(c' - c)
    for (int c = 0; c < Lc && limit > 0 && limb_shape_for(p, sh.K * sh.nparts, cap, &fb_shape); ++c) {
      const int np = std::min(c, LA - 1) + 1 - std::max(0, c - LB + 1);
      sc = sc / 256.0 + (double)np;
      const int64_t eb = (int64_t)floor(8.0 * c + log2(sc) + log2((double)Kp) + 14.0) + 2;
      if (eb > limit) break;
      c0 = c + 1;
      ebits = (int)eb;
    }
  }
  // diagonal groups of at most pmax slice pairs, each one exact int32 plane
  std::vector<DiagGroup> groups;
  std::vector<int32_t> slot_of(Lc + 1, 0);
  int nslots = 0;
  for (int c = 0; c < Lc; ++c) {
    const int lo = std::max(0, c - LB + 1), hi = std::min(c, LA - 1) + 1;
    slot_of[c] = nslots;
    if (c < c0) continue;
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
  const int nT = t_limbs(LA, LB);
  {
    int64_t pairs = 0;
    for (const DiagGroup &g : groups) pairs += g.a1 - g.a0;
    const int64_t plan[10] = {LA, LB, nslots, ngroups_real, Kt, sh.M, sh.N, sh.nparts, 0, pairs};
    memcpy(ctx->last_plan, plan, sizeof plan);
  }

  const size_t bytesA = (size_t)LA * Mp * Kp, bytesB = (size_t)LB * Np * Kp;
  int8_t *planesA = (int8_t *)ws_get(ctx, WS_PLANES_A, bytesA);
  int8_t *planesB = (int8_t *)ws_get(ctx, WS_PLANES_B, bytesB);
  int8_t *planesB2 = sh.cplx ? (int8_t *)ws_get(ctx, WS_PLANES_B2, bytesB) : nullptr;
  const int64_t ds = plane_stride(sh.M * sh.N);
  int32_t *D = (int32_t *)ws_get(ctx, WS_D, sizeof(int32_t) * (size_t)nslots * ds);
  uint32_t *T = (uint32_t *)ws_get(ctx, WS_T, sizeof(uint32_t) * (size_t)nT * sh.M * sh.N);
  // tables, then (truncated set) the fallback counter and entry list
  const size_t tab_bytes = sizeof(DiagGroup) * groups.size() + sizeof(int32_t) * slot_of.size();
  const size_t fb_off = (tab_bytes + 7) & ~(size_t)7;
  char *tabs = (char *)ws_get(ctx, WS_TABLES, fb_off + (ebits >= 0 ? 8 + 8 * (size_t)sh.M * sh.N : 0));
  if (!planesA || !planesB || (sh.cplx && !planesB2) || !D || !T || !tabs) return ARBGPU_ENOMEM;
  DiagGroup *dgroups = (DiagGroup *)tabs;
  int32_t *dslot = (int32_t *)(tabs + sizeof(DiagGroup) * groups.size());
  int32_t *fb_count = ebits >= 0 ? (int32_t *)(tabs + fb_off) : nullptr;
  int64_t *fb_list = ebits >= 0 ? (int64_t *)(tabs + fb_off + 8) : nullptr;
  ARB_TRY(hipMemcpyAsync(dgroups, groups.data(), sizeof(DiagGroup) * groups.size(), hipMemcpyHostToDevice, s),
          "table upload");
  ARB_TRY(hipMemcpyAsync(dslot, slot_of.data(), sizeof(int32_t) * slot_of.size(), hipMemcpyHostToDevice, s),
          "table upload");
  // the host tables must outlive their asynchronous uploads
  ARB_TRY(hipStreamSynchronize(s), "table upload");

  SliceParams sa;
  memset(&sa, 0, sizeof sa);
  sa.part[0] = A->re;
  sa.part[1] = sh.cplx ? A->im : A->re;
  sa.lines = sh.M; sa.len = Kb; sa.off = A->off; sa.line_stride = A->rs; sa.elem_stride = A->cs; sa.k0 = k0;
  sa.mode = sh.cplx ? 3 : 0;
  sa.lines_pad = Mp; sa.k_pad = Kp; sa.L = LA; sa.v2 = rv2; sa.planes = planesA;
  Lines bl;
  {
    KernelTimer t_slice(ctx, "slice", s);
    int rc = pre ? lines_of(*pre, k0, bl) : b_lines(ctx, B, sh.cplx, k0, k1, s, bl);
    if (rc) return rc;
    ARB_TRY(launch_slice(sa, s), "slice");
    for (int q = 0; q < sh.nparts; ++q) {
      SliceParams sb = sa;
      sb.part[0] = bl.part[0];
      sb.part[1] = bl.part[1];
      sb.lines = sh.N; sb.off = bl.off; sb.line_stride = bl.line_stride; sb.elem_stride = bl.elem_stride;
      sb.k0 = bl.k0;
      sb.mode = !sh.cplx ? 0 : (q == 0 ? 1 : 2);
      sb.lines_pad = Np; sb.L = LB; sb.v2 = cv2; sb.planes = q == 0 ? planesB : planesB2;
      ARB_TRY(launch_slice(sb, s), "slice");
    }
  }
  for (int q = 0; q < sh.nparts; ++q) {
    MfmaParams mp;
    mp.A = planesA;
    mp.B = q == 0 ? planesB : planesB2;
    mp.D = D;
    mp.ds = ds;
    mp.groups = dgroups;
    mp.M = sh.M; mp.N = sh.N; mp.Mp = Mp; mp.Np = Np; mp.Kp = Kp;
    mp.ntm = (int)(Mp / kTile); mp.ntn = (int)(Np / kTile);
    mp.ngroups = (int)groups.size();
    {
      KernelTimer tm(ctx, "mfma", s);
      ARB_TRY(launch_mfma(mp, s), "mfma");
    }
    RecombParams rp;
    rp.D = D; rp.ds = ds; rp.slot_of = dslot; rp.Lc = Lc; rp.M = sh.M; rp.N = sh.N; rp.T = T; rp.nT = nT;
    rp.rowv2 = rv2; rp.colv2 = cv2;
    rp.C = out[q];
    rp.c_off = o_off; rp.c_rs = o_rs; rp.c_cs = o_cs;
    rp.p = p;
    rp.approx = out_approx;
    rp.rin_m = rin_m[q];
    rp.rin_e = rin_e[q];
    rp.ebits = ebits;
    rp.fb_list = fb_list;
    rp.fb_count = fb_count;
    if (fb_count) ARB_TRY(launch_fill_i32(fb_count, 0, 1, s), "fill");
    {
      KernelTimer tr(ctx, "recombine", s);
      ARB_TRY(launch_recombine(rp, s), "recombine");
    }
    if (fb_count) {   // the entries whose truncation was not certified, exactly
      MmParams mm;
      memset(&mm, 0, sizeof mm);
      mm.A[0] = A->re;
      mm.A[1] = sh.cplx ? A->im : A->re;
      mm.B[0] = B->re;
      mm.B[1] = sh.cplx ? B->im : B->re;
      mm.C = out[q];
      mm.M = sh.M; mm.N = sh.K; mm.K = sh.N;
      mm.a_off = A->off; mm.a_rs = A->rs; mm.a_cs = A->cs;
      mm.b_off = B->off; mm.b_rs = B->rs; mm.b_cs = B->cs;
      mm.c_off = o_off; mm.c_rs = o_rs; mm.c_cs = o_cs;
      mm.p = p;
      mm.approx = out_approx;
      mm.ct = !sh.cplx ? comp_real() : (q == 0 ? comp_re() : comp_im());
      KernelTimer tf(ctx, "fallback", s);
      ARB_TRY(launch_limb_mm_list(mm, fb_shape, fb_list, fb_count, sh.M * sh.N, s), "fallback");
    }
    int rc = t_to_sink(ctx, ts, q, T, nT, sh.M * sh.N, s);
    if (rc) return rc;
  }
  return ARBGPU_OK;
}

// The block product in residue form: residue digit planes of every operand
// part modulo m primes, per prime the residues of the block products
// reduced on chip, Chinese remainder reconstruction and rounding per entry.
// A complex block takes three real products, AC, BD and (A + B)(C + D),
// with Re = AC - BD and Im = (A + B)(C + D) - AC - BD formed on the
// residues (eq. (2), Section 3.6); `four` takes AC, BD, AD and BC instead.
// Both are exact, and so give the same T.
int rns_block_product(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, const Shape &sh, int64_t k0,
                      int64_t k1, const int32_t *st, int HA, int HB, const arbgpu_out *out, int64_t o_off,
                      int64_t o_rs, int64_t o_cs, int p, bool out_approx, double *const rin_m[2],
                      int32_t *const rin_e[2], hipStream_t s, bool four, const TSink *ts, const Lines *pre) {
  const int32_t *rv2 = st + sh.M, *cv2 = st + 2 * sh.M + sh.N;
  const int64_t Kb = k1 - k0;
  const int64_t Kt = sh.cplx ? 2 * Kb : Kb;   // terms of one output value
  const int64_t Kp = round_up(std::max<int64_t>(Kb, 1), kKStep);
  const int nprod = !sh.cplx ? 1 : (four ? 4 : 3);
  const int64_t bits = t_bits(HA, HB, Kt);
  const int m = rns_count(bits);
  const int tile = sh.tile ? sh.tile : rns_tile(sh.M, sh.N, (int64_t)nprod * ((m + 7) / 8 * 8));
  const int64_t Mp = round_up(std::max<int64_t>(sh.M, 1), tile), Np = round_up(std::max<int64_t>(sh.N, 1), tile);
  const int W = (int)((bits + 1 + 31) / 32) + 1;
  const int LA = slices_for(HA), LB = slices_for(HB);
  const int nw = (std::max(LA, LB) + 3) / 4;
  if (m < 1) return set_error(ctx, ARBGPU_EINVAL, "residue form: %lld-bit block values", (long long)bits);
  RnsTables tab;
  int rc = rns_tables(ctx, m, nw, W, s, tab);
  if (rc) return rc;
  // plane sets per operand: real 1; complex re, im (and re + im)
  const int nsets = !sh.cplx ? 1 : (four ? 2 : 3);
  const int mpad = (m + 7) / 8 * 8;
  {
    const int64_t plan[10] = {2 * m, 2 * m, (int64_t)nprod * m, (int64_t)nprod * m, Kp, sh.M, sh.N, sh.nparts, m,
                              4 * (int64_t)nprod * m};
    memcpy(ctx->last_plan, plan, sizeof plan);
  }
  const int64_t setA = 2 * (int64_t)m * Mp * Kp, setB = 2 * (int64_t)m * Np * Kp;
  int8_t *planesA = (int8_t *)ws_get(ctx, WS_PLANES_A, (size_t)(nsets * setA));
  int8_t *planesB = (int8_t *)ws_get(ctx, WS_PLANES_B, (size_t)(nsets * setB));
  const int64_t ds = plane_stride(sh.M * sh.N);
  int16_t *Y = (int16_t *)ws_get(ctx, WS_D, sizeof(int16_t) * (size_t)nprod * m * ds);
  uint32_t *Tw = ts ? (uint32_t *)ws_get(ctx, WS_T, sizeof(uint32_t) * (size_t)W * sh.M * sh.N) : nullptr;
  if (!planesA || !planesB || !Y || (ts && !Tw)) return ARBGPU_ENOMEM;

  RnsSliceParams sa;
  memset(&sa, 0, sizeof sa);
  sa.part[0] = sa.part[1] = A->re;
  sa.lines = sh.M; sa.len = Kb; sa.off = A->off; sa.line_stride = A->rs; sa.elem_stride = A->cs; sa.k0 = k0;
  sa.mode = 0;
  sa.lines_pad = Mp; sa.k_pad = Kp; sa.L = LA; sa.v2 = rv2; sa.tab = tab; sa.planes = planesA;
  Lines bl;
  {
    KernelTimer t_slice(ctx, "slice", s);
    rc = pre ? lines_of(*pre, k0, bl) : b_lines(ctx, B, sh.cplx, k0, k1, s, bl);
    if (rc) return rc;
    for (int q = 0; q < sh.nparts; ++q) {
      RnsSliceParams pa = sa;
      pa.part[0] = pa.part[1] = q == 0 ? A->re : A->im;
      pa.planes = planesA + q * setA;
      if (nsets == 3 && q == 1) {   // the imaginary part also forms re + im
        pa.addend = planesA;
        pa.sum = planesA + 2 * setA;
      }
      ARB_TRY(launch_rns_slice(pa, s), "residue slice");
      RnsSliceParams pb = sa;
      pb.part[0] = pb.part[1] = bl.part[q];
      pb.lines = sh.N; pb.off = bl.off; pb.line_stride = bl.line_stride; pb.elem_stride = bl.elem_stride;
      pb.k0 = bl.k0;
      pb.lines_pad = Np; pb.L = LB; pb.v2 = cv2; pb.planes = planesB + q * setB;
      if (nsets == 3 && q == 1) {
        pb.addend = planesB;
        pb.sum = planesB + 2 * setB;
      }
      ARB_TRY(launch_rns_slice(pb, s), "residue slice");
    }
  }
  MfmaRnsParams mp;
  memset(&mp, 0, sizeof mp);
  // products: real A B; complex AC, BD, then (A + B)(C + D), or AD and BC
  const int pa_of[4] = {0, 1, four ? 0 : 2, 1}, pb_of[4] = {0, 1, four ? 1 : 2, 0};
  for (int q = 0; q < nprod; ++q) {
    mp.A[q] = planesA + pa_of[q] * setA;
    mp.B[q] = planesB + pb_of[q] * setB;
  }
  mp.Y = Y;
  mp.prime = tab.prime;
  mp.mu = tab.mu;
  mp.nprod = nprod; mp.m = m; mp.mpad = mpad;
  mp.M = sh.M; mp.N = sh.N; mp.Mp = Mp; mp.Np = Np; mp.Kp = Kp; mp.ds = ds;
  mp.tile = tile;
  mp.ntm = (int)(Mp / tile); mp.ntn = (int)(Np / tile);
  {
    KernelTimer tm(ctx, "mfma", s);
    ARB_TRY(launch_mfma_rns(mp, s), "mfma");
  }
  for (int q = 0; q < sh.nparts; ++q) {
    RnsCrtParams cp;
    memset(&cp, 0, sizeof cp);
    cp.Y = Y; cp.ds = ds;
    if (!sh.cplx) {
      cp.nsrc = 1; cp.src[0] = 0; cp.sgn[0] = 1;
    } else if (q == 0) {   // AC - BD
      cp.nsrc = 2; cp.src[0] = 0; cp.sgn[0] = 1; cp.src[1] = 1; cp.sgn[1] = -1;
    } else if (four) {     // AD + BC
      cp.nsrc = 2; cp.src[0] = 2; cp.sgn[0] = 1; cp.src[1] = 3; cp.sgn[1] = 1;
    } else {               // (A + B)(C + D) - AC - BD
      cp.nsrc = 3; cp.src[0] = 2; cp.sgn[0] = 1; cp.src[1] = 0; cp.sgn[1] = -1; cp.src[2] = 1; cp.sgn[2] = -1;
    }
    cp.tab = tab; cp.M = sh.M; cp.N = sh.N; cp.W = W;
    cp.rowv2 = rv2; cp.colv2 = cv2;
    cp.C = out[q];
    cp.c_off = o_off; cp.c_rs = o_rs; cp.c_cs = o_cs;
    cp.p = p;
    cp.approx = out_approx;
    cp.rin_m = rin_m[q];
    cp.rin_e = rin_e[q];
    cp.t_out = Tw;
    cp.t_ld = sh.M * sh.N;
    {
      KernelTimer tr(ctx, "recombine", s);
      ARB_TRY(launch_rns_crt(cp, s), "residue reconstruction");
    }
    rc = t_to_sink(ctx, ts, q, Tw, W, sh.M * sh.N, s);
    if (rc) return rc;
  }
  return ARBGPU_OK;
}

// Radius products over the whole inner range (Section 4.1, last
// paragraph): rho = |A| R_B + R_A (|B| + R_B), FP64 rounded upward, with a
// per-entry fallback when a value does not fit its line's frame.
int radius_products(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, const Shape &sh, double *rin_m[2],
                    int32_t *rin_e[2], hipStream_t s) {
  const int64_t Kt = sh.cplx ? 2 * sh.K : sh.K;
  const size_t na = (size_t)sh.M * Kt, nb = (size_t)sh.N * Kt, mn = (size_t)sh.M * sh.N;
  char *ra = (char *)ws_get(ctx, WS_RAD_A, 2 * sizeof(double) * na + 2 * sizeof(int32_t) * sh.M);
  char *rb = (char *)ws_get(ctx, WS_RAD_B, 2 * sizeof(double) * nb + 2 * sizeof(int32_t) * sh.N);
  char *ro = (char *)ws_get(ctx, WS_RAD_OUT, (size_t)sh.nparts * (sizeof(double) + sizeof(int32_t)) * mn + 8);
  if (!ra || !rb || !ro) return ARBGPU_ENOMEM;
  int32_t *tiny = (int32_t *)((double *)ro + (size_t)sh.nparts * mn) + (size_t)sh.nparts * mn;
  ARB_TRY(launch_fill_i32(tiny, 0, 1, s), "fill");
  RadPrepParams pa;
  memset(&pa, 0, sizeof pa);
  pa.part[0] = A->re;
  pa.part[1] = sh.cplx ? A->im : A->re;
  pa.nparts = sh.nparts;
  pa.lines = sh.M; pa.len = sh.K; pa.off = A->off; pa.line_stride = A->rs; pa.elem_stride = A->cs;
  pa.mode = sh.cplx ? 3 : 0;
  pa.side = 0;
  pa.v0 = (double *)ra;
  pa.v1 = (double *)ra + na;
  pa.scale0 = (int32_t *)((double *)ra + 2 * na);
  pa.scale1 = pa.scale0 + sh.M;
  pa.tiny = tiny;
  ARB_TRY(launch_rad_prep(pa, s), "rad prep");
  for (int q = 0; q < sh.nparts; ++q) {
    RadPrepParams pb;
    memset(&pb, 0, sizeof pb);
    pb.part[0] = B->re;
    pb.part[1] = sh.cplx ? B->im : B->re;
    pb.nparts = sh.nparts;
    pb.lines = sh.N; pb.len = sh.K; pb.off = B->off; pb.line_stride = B->cs; pb.elem_stride = B->rs;
    pb.mode = !sh.cplx ? 0 : (q == 0 ? 1 : 2);
    pb.side = 1;
    pb.v0 = (double *)rb;
    pb.v1 = (double *)rb + nb;
    pb.scale0 = (int32_t *)((double *)rb + 2 * nb);
    pb.scale1 = pb.scale0 + sh.N;
    pb.tiny = tiny;
    ARB_TRY(launch_rad_prep(pb, s), "rad prep");
    rin_m[q] = (double *)ro + (size_t)q * mn;
    rin_e[q] = (int32_t *)((double *)ro + (size_t)sh.nparts * mn) + (size_t)q * mn;
    RadGemmParams rg;
    rg.a_m = pa.v0; rg.a_r = pa.v1; rg.b_mr = pb.v0; rg.b_r = pb.v1;
    rg.a_s0 = pa.scale0; rg.a_s1 = pa.scale1; rg.b_s0 = pb.scale0; rg.b_s1 = pb.scale1;
    rg.tiny = tiny;
    rg.M = sh.M; rg.N = sh.N; rg.Kt = Kt;
    rg.out_m = rin_m[q];
    rg.out_e = rin_e[q];
    rg.splits = rad_gemm_splits(sh.M, sh.N, Kt);
    rg.kchunk = round_up((Kt + rg.splits - 1) / rg.splits, 16);
    rg.part = nullptr;
    if (rg.splits > 1) {
      rg.part = (double *)ws_get(ctx, WS_RAD_PART, sizeof(double) * 2 * (size_t)rg.splits * mn);
      if (!rg.part) return ARBGPU_ENOMEM;
    }
    RadExactParams rx;
    memset(&rx, 0, sizeof rx);
    rx.A[0] = A->re;
    rx.A[1] = sh.cplx ? A->im : A->re;
    rx.B[0] = B->re;
    rx.B[1] = sh.cplx ? B->im : B->re;
    rx.a_mode = pa.mode;
    rx.b_mode = pb.mode;
    rx.len = sh.K; rx.Kt = Kt; rx.M = sh.M; rx.N = sh.N;
    rx.a_off = A->off; rx.a_rs = A->rs; rx.a_cs = A->cs;
    rx.b_off = B->off; rx.b_rs = B->rs; rx.b_cs = B->cs;
    rx.tiny = tiny;
    rx.out_m = rin_m[q];
    rx.out_e = rin_e[q];
    KernelTimer tg(ctx, "rad_gemm", s);
    ARB_TRY(launch_rad_gemm(rg, s), "rad gemm");
    ARB_TRY(launch_rad_exact(rx, s), "rad exact");
  }
  return ARBGPU_OK;
}

// Height bound of Algorithm 2, h = 1.25 min(p, max(p_A, p_B)) + 192; block
// heights are integers, so the admissible maximum is floor(h).
int height_bound(int64_t p, int pA, int pB) {
  const int64_t m = std::min<int64_t>(p, std::max(pA, pB));
  return (int)((5 * m) / 4 + 192);
}

constexpr int kBasecase = 30;   // Algorithm 2: shorter ranges use dot products

// Cost estimates (seconds) of one block of the partition, for the choice
// between its integer product and its terms in the merge: a fixed cost of
// the integer product's launches and host round trips, its MFMA work and
// the exact block values it writes, against window-engine products of the
// operand limbs that reach the window (about 3 ps per 32 x 32 limb product
// per output entry at these sizes).
double block_cost_int8(const Shape &sh, const BlockSpan &b, int p) {
  const int64_t Kb = b.k1 - b.k0, Kt = sh.cplx ? 2 * Kb : Kb, MN = sh.M * sh.N;
  const int64_t bits = t_bits(b.ha, b.hb, Kt);
  const int64_t pairs = rns_better(b.ha, b.hb, Kt) ? 4 * (int64_t)rns_count(bits) * (sh.cplx ? 3 : 1)
                                                  : (int64_t)slices_for(b.ha) * slices_for(b.hb) * sh.nparts;
  const double W = (double)(bits + 63) / 32.0;
  (void)p;
  return 60e-6 + 2.0 * (double)pairs * (double)MN * (double)Kb / 1.5e15 + (double)MN * sh.nparts * 8.0 * W / 1.5e12;
}

double block_cost_base(const Shape &sh, const BlockSpan &b, int p, const arbgpu_mat *A, const arbgpu_mat *B) {
  int cap = std::max(A->re.cap, B->re.cap);
  if (sh.cplx) cap = std::max(cap, std::max(A->im.cap, B->im.cap));
  const double w = (double)std::min<int64_t>(cap, (p + 64 + 31) / 32);
  return (double)(sh.M * sh.N) * (double)(b.k1 - b.k0) * (sh.cplx ? 4.0 : 1.0) * w * w * 3e-12;
}

}  // namespace

// Largest digit-plane counts, partial planes and T limbs the base-256 form
// can take for heights up to hmax: every height pair when the form is
// forced, else the pairs for which the automatic choice gives this form
// (each digit count taken at the largest height it holds, where the
// residue form needs the most primes).  la = 0: the form is never chosen.
struct SliceBound {
  int64_t la, lb, nslots;
  int tl;
};

SliceBound slice_bound(int hmax, int64_t Kt, bool forced) {
  const int64_t Kp = round_up(std::max<int64_t>(Kt, 1), kKStep);
  const int64_t pmax = std::max<int64_t>(1, ((int64_t)0x7FFFFFFF) / (Kp << 14));
  const int lmax = std::min(kMaxSlices, slices_for(hmax));
  auto nslots = [&](int64_t la, int64_t lb) { return (la + lb - 1) + la * lb / pmax; };
  if (forced) return SliceBound{lmax, lmax, nslots(lmax, lmax), t_limbs(lmax, lmax)};
  static std::mutex mu;
  static std::map<std::pair<int, int64_t>, SliceBound> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({hmax, Kt});
    if (it != cache.end()) return it->second;
  }
  SliceBound b{0, 0, 0, 0};
  auto top = [&](int l) { return std::min(hmax, l == 1 ? 7 : 8 * l - 2); };
  for (int la = 1; la <= lmax; ++la)
    for (int lb = 1; lb <= lmax; ++lb) {
      if (rns_better(top(la), top(lb), Kt)) continue;
      b.la = std::max<int64_t>(b.la, la);
      b.lb = std::max<int64_t>(b.lb, lb);
      b.nslots = std::max(b.nslots, nslots(la, lb));
      b.tl = std::max(b.tl, t_limbs(la, lb));
    }
  std::lock_guard<std::mutex> lk(mu);
  cache[{hmax, Kt}] = b;
  return b;
}

void mat_mul_ws_sizes(const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags, size_t out[]) {
  for (int k = 0; k < WS_COUNT; ++k) out[k] = 0;
  const bool cplx = flags & ARBGPU_COMPLEX;
  const int64_t parts = cplx ? 2 : 1;
  const int64_t M = A->rows, N = B->cols, K = A->cols;
  const int64_t Kt = cplx ? 2 * K : K;
  const int64_t MN = M * N, ds = plane_stride(MN);
  if (flags & ARBGPU_ALGO_LIMB) return;   // the limb kernel takes no workspace
  const int64_t Mp = round_up(std::max<int64_t>(M, 1), kTile), Np = round_up(std::max<int64_t>(N, 1), kTile);
  int cap = std::max(A->re.cap, B->re.cap);
  if (cplx) cap = std::max(cap, std::max(A->im.cap, B->im.cap));
  // integer heights of a single block are at most the height bound
  const int hmax = height_bound(p, 32 * cap, 32 * cap);
  auto grow = [&](int slot, int64_t bytes) { out[slot] = std::max(out[slot], (size_t)std::max<int64_t>(bytes, 256)); };
  grow(WS_STATS, 4 * (2 * M + 2 * N + 8));
  if (B->cs == 1 && B->rs != 1) {   // line-major copy of a row-major B
    int64_t g = 4 * N * K * (B->re.cap + 2);
    if (cplx) g += 4 * N * K * (B->im.cap + 2);
    grow(WS_GATHER, g);
  }
  {   // the planner of several blocks: element table, bounds, per-block statistics
    const int64_t maxb = K / kBasecase + 2;
    grow(WS_PLAN, round_up(8 * (M + N) * K + 16 * maxb + 4 * (maxb + 1), 256) +
                      4 * maxb * round_up(2 * M + 2 * N + 8, 64));
  }
  if (!(flags & ARBGPU_ALGO_RNS)) {   // base-256 slices
    const int64_t Kp = round_up(std::max<int64_t>(Kt, 1), kKStep);
    const SliceBound b = slice_bound(hmax, Kt, (flags & ARBGPU_ALGO_SLICED) != 0);
    if (b.la > 0) {
      grow(WS_PLANES_A, b.la * Mp * Kp);
      grow(WS_PLANES_B, b.lb * Np * Kp);
      if (cplx) grow(WS_PLANES_B2, b.lb * Np * Kp);
      grow(WS_D, 4 * b.nslots * ds);
      grow(WS_T, 4 * (int64_t)b.tl * MN);
      // tables and the list of entries the truncated diagonal set leaves
      grow(WS_TABLES, (int64_t)sizeof(DiagGroup) * (b.nslots + 8) + 4 * (b.la + b.lb) + 16 + 8 * MN);
    }
  }
  if (!(flags & ARBGPU_ALGO_SLICED)) {   // residues: the largest heights the form holds
    // every admissible pair of heights up to hmax: at most 4 * 127 digits
    // per operand and the largest block-value width the reconstruction
    // holds
    const int h = std::min(hmax, 4 * 127 * 8 - 2);
    int64_t bits = t_bits(h, h, Kt);
    if (!rns_fits_bits(bits)) {   // the widest fitting values (the limit grows with bits)
      int64_t lo = 0, hi = bits;
      while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        (rns_fits_bits(mid) ? lo : hi) = mid;
      }
      bits = lo;
    }
    const int64_t Kp = round_up(std::max<int64_t>(K, 1), kKStep);
    if (bits >= 1 && rns_fits_bits(bits) && ((int64_t)0x7FFFFFFF) / (round_up(std::max<int64_t>(Kt, 1), kKStep) << 14) >= 2) {
      const int m = rns_count(bits);
      const int W = (int)((bits + 1 + 31) / 32) + 1;
      const int nw = (slices_for(h) + 3) / 4;
      const int64_t nsets = cplx ? 3 : 1, nprod = cplx ? 4 : 1;
      grow(WS_PLANES_A, nsets * 2 * m * Mp * Kp);
      grow(WS_PLANES_B, nsets * 2 * m * Np * Kp);
      grow(WS_D, 2 * nprod * m * ds);
      grow(WS_RNS, (int64_t)rns_layout(m, nw, W).bytes);
    }
  }
  const bool rad = A->re.rad_m || B->re.rad_m || (cplx && (A->im.rad_m || B->im.rad_m));
  if (rad && !(flags & ARBGPU_APPROX)) {
    grow(WS_RAD_A, 16 * M * Kt + 8 * M);
    grow(WS_RAD_B, 16 * N * Kt + 8 * N);
    grow(WS_RAD_OUT, parts * 12 * MN + 8);
    const int sp = rad_gemm_splits(M, N, Kt);
    if (sp > 1) grow(WS_RAD_PART, 16 * (int64_t)sp * MN);
  }
}

size_t mat_mul_footprint(const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags) {
  size_t sz[WS_COUNT];
  mat_mul_ws_sizes(A, B, p, flags, sz);
  size_t t = 0;
  for (int k = 0; k < WS_COUNT; ++k) t += sz[k];
  return t;
}

int plan_blocks(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, bool cplx, int hmax, hipStream_t s,
                std::vector<BlockSpan> &out, int32_t **stats, int64_t *stride) {
  const int64_t M = A->rows, N = B->cols, K = A->cols;
  const int64_t maxb = K / kBasecase + 2;   // every block but the last has >= 30 indices or is basecase-extended
  const int64_t sstride = round_up(2 * M + 2 * N + 8, 64);
  const size_t hl_bytes = sizeof(int2) * (size_t)(M + N) * K;
  const size_t o_st = round_up(hl_bytes + sizeof(int64_t) * 2 * maxb + sizeof(int32_t) * (maxb + 1), 256);
  const size_t bytes = o_st + sizeof(int32_t) * (size_t)(maxb * sstride);
  char *w = (char *)ws_get(ctx, WS_PLAN, bytes);
  if (!w) return ARBGPU_ENOMEM;
  PlanParams pp;
  memset(&pp, 0, sizeof pp);
  pp.A[0] = A->re;
  pp.A[1] = cplx ? A->im : A->re;
  pp.B[0] = B->re;
  pp.B[1] = cplx ? B->im : B->re;
  pp.nparts = cplx ? 2 : 1;
  pp.M = M; pp.N = N; pp.inner = K;
  pp.a_off = A->off; pp.a_rs = A->rs; pp.a_cs = A->cs;
  pp.b_off = B->off; pp.b_rs = B->rs; pp.b_cs = B->cs;
  pp.hmax = hmax;
  pp.basecase = kBasecase;
  pp.hlA = (int2 *)w;
  pp.hlB = pp.hlA + (size_t)M * K;
  pp.bounds = (int64_t *)(w + hl_bytes);
  pp.kinds = (int32_t *)(pp.bounds + 2 * maxb);
  pp.max_blocks = maxb;
  pp.nblocks = pp.kinds + maxb;
  int32_t *bst = (int32_t *)(w + o_st);
  {
    KernelTimer tp(ctx, "plan", s);
    ARB_TRY(launch_plan(pp, s), "plan");
    BlockStatsParams bs{pp.hlA, pp.hlB, M, N, pp.bounds, pp.nblocks, maxb, bst, sstride};
    ARB_TRY(launch_fill_i32(bst, 0, maxb * sstride, s), "fill");
    ARB_TRY(launch_block_stats(bs, s), "block stats");
  }
  int32_t nb = 0;
  ARB_TRY(hipMemcpyAsync(&nb, pp.nblocks, sizeof nb, hipMemcpyDeviceToHost, s), "plan readback");
  ARB_TRY(hipStreamSynchronize(s), "plan readback");
  if (nb < 0 || nb > maxb)
    return set_error(ctx, ARBGPU_EDEVICE, "planner produced %d blocks (bound %lld)", nb, (long long)maxb);
  std::vector<int64_t> b(2 * (size_t)nb + 2);
  std::vector<int32_t> k((size_t)nb + 1), g(8 * (size_t)nb + 8);
  if (nb) {
    ARB_TRY(hipMemcpyAsync(b.data(), pp.bounds, sizeof(int64_t) * 2 * nb, hipMemcpyDeviceToHost, s), "plan readback");
    ARB_TRY(hipMemcpyAsync(k.data(), pp.kinds, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s), "plan readback");
    // the heights gA[0], gB[0] (8 words after the lines) of every block
    ARB_TRY(hipMemcpy2DAsync(g.data(), 8 * sizeof(int32_t), bst + 2 * M + 2 * N, sizeof(int32_t) * sstride,
                             8 * sizeof(int32_t), nb, hipMemcpyDeviceToHost, s),
            "plan readback");
    ARB_TRY(hipStreamSynchronize(s), "plan readback");
  }
  out.clear();
  for (int i = 0; i < nb; ++i) out.push_back(BlockSpan{b[2 * i], b[2 * i + 1], k[i], g[8 * i], g[8 * i + 4]});
  if (stats) *stats = bst;
  if (stride) *stride = sstride;
  return ARBGPU_OK;
}

int plan_partition(arbgpu_ctx *ctx, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags,
                   hipStream_t s, int64_t *bounds, int32_t *kinds, int64_t max_blocks, int64_t *nblocks) {
  Shape sh{(flags & ARBGPU_COMPLEX) != 0, false, (flags & ARBGPU_COMPLEX) ? 2 : 1, A->rows, B->cols, A->cols};
  int32_t *st = stats_ws(ctx, sh);
  if (!st) return ARBGPU_ENOMEM;
  int32_t g[8];
  int rc = line_stats(ctx, A, B, sh, 0, sh.K, st, s, g);
  if (rc) return rc;
  if (g[2] || g[6]) return set_error(ctx, ARBGPU_EINVAL, "an operand exponent is outside (-2^28, 2^28)");
  std::vector<BlockSpan> blocks;
  rc = plan_blocks(ctx, A, B, sh.cplx, height_bound(p, g[1], g[5]), s, blocks);
  if (rc) return rc;
  *nblocks = (int64_t)blocks.size();
  for (int64_t i = 0; i < (int64_t)blocks.size() && i < max_blocks; ++i) {
    bounds[2 * i] = blocks[i].k0;
    bounds[2 * i + 1] = blocks[i].k1;
    kinds[i] = blocks[i].kind;
  }
  return ARBGPU_OK;
}

int sliced_mat_mul(arbgpu_ctx *ctx, const arbgpu_omat *C, const arbgpu_mat *A, const arbgpu_mat *B, int64_t p,
                   uint32_t flags, hipStream_t s, bool forced, int choice) {
  Shape sh{(flags & ARBGPU_COMPLEX) != 0, (flags & ARBGPU_APPROX) != 0, (flags & ARBGPU_COMPLEX) ? 2 : 1,
           A->rows, B->cols, A->cols};
  sh.tile = choice == kChoiceRns256 ? 256 : (choice == kChoiceRns128 ? 128 : 0);
  if (!forced && sh.K < kBasecase) return kNotApplicable;
  const int64_t Kt = sh.cplx ? 2 * sh.K : sh.K;
  if (((int64_t)0x7FFFFFFF) / (round_up(std::max<int64_t>(Kt, 1), kKStep) << 14) < 1) {
    if (forced) return set_error(ctx, ARBGPU_EINVAL, "sliced product: inner length %lld too long", (long long)Kt);
    return kNotApplicable;
  }

  // ---- statistics over the whole inner range --------------------------------
  int32_t *st = stats_ws(ctx, sh);
  if (!st) return ARBGPU_ENOMEM;
  int32_t g[8];
  Lines pre;
  bool pre_ok = false;
  int rc = line_stats(ctx, A, B, sh, 0, sh.K, st, s, g, &pre, &pre_ok);
  if (rc) return rc;
  const Lines *bpre = pre_ok ? &pre : nullptr;
  if (g[2] || g[6]) return kNotApplicable;   // out-of-range exponents: flagged per entry by the limb kernel
  const int hmax = height_bound(p, g[1], g[5]);
  const bool radA = A->re.rad_m || (sh.cplx && A->im.rad_m);
  const bool radB = B->re.rad_m || (sh.cplx && B->im.rad_m);
  const arbgpu_out outs[2] = {C->re, C->im};
  double *rin_m[2] = {nullptr, nullptr};
  int32_t *rin_e[2] = {nullptr, nullptr};
  // The limb kernel takes over what this path does not cover, unless the
  // caller asked for this path explicitly.
  auto not_here = [&](const char *why) {
    return forced ? set_error(ctx, ARBGPU_EINVAL, "sliced product: %s", why) : kNotApplicable;
  };
  // residue form or base-256 slices for a block of heights (ha, hb)
  auto use_rns = [&](int ha, int hb, int64_t kt) {
    if (flags & ARBGPU_ALGO_RNS) return true;
    if (flags & ARBGPU_ALGO_SLICED) return false;
    if (choice == kChoiceSlices) return false;
    if (choice == kChoiceRns256 || choice == kChoiceRns128) return rns_fits(ha, hb, kt);
    return rns_better(ha, hb, kt);
  };

  if (g[0] <= hmax && g[4] <= hmax) {
    // ---- the whole inner range is one block: its exact integer product
    //      rounds straight to the output
    if (slices_for(g[0]) > kMaxSlices || slices_for(g[4]) > kMaxSlices) return not_here("integer height too large");
    const bool rns = use_rns(g[0], g[4], Kt);
    if (rns && !rns_fits(g[0], g[4], Kt)) return not_here("residue form does not fit these heights");
    if (!sh.approx && (radA || radB)) {
      rc = radius_products(ctx, A, B, sh, rin_m, rin_e, s);
      if (rc) return rc;
    }
    return block_product(ctx, A, B, sh, 0, sh.K, st, g[0], g[4], outs, C->off, C->rs, C->cs, (int)p, sh.approx,
                         rin_m, rin_e, s, rns, (flags & ARBGPU_COMPLEX_4M) != 0, nullptr, true, bpre);
  }

  // ---- several blocks (Algorithm 2's greedy partition) ----------------------
  // Every block result T_s 2^(-e_i - f_j) is kept exactly and the merge adds
  // them and the basecase products exactly before the one truncation.  The
  // exact block values need exponents inside the operand format's range.
  if (2 * (int64_t)std::max(g[3], g[7]) + 64 >= (int64_t)(1 << 28)) return not_here("exponents too large for blocks");
  if (slices_for(hmax) > kMaxSlices) return not_here("height bound too large");
  std::vector<BlockSpan> blocks;
  int32_t *bstats = nullptr;
  int64_t bstride = 0;
  rc = plan_blocks(ctx, A, B, sh.cplx, hmax, s, blocks, &bstats, &bstride);
  if (rc) return rc;
  // Per-block choice (unless an ALGO flag fixes the path): a block whose
  // integer product costs more than its terms on the window engine becomes
  // basecase indices of the merge.
  if (!(flags & (ARBGPU_ALGO_SLICED | ARBGPU_ALGO_RNS)))
    for (BlockSpan &b : blocks)
      if (b.kind == 0 && block_cost_int8(sh, b, (int)p) > block_cost_base(sh, b, (int)p, A, B)) b.kind = 1;
  std::vector<int64_t> bk;   // basecase inner indices
  int nS = 0, capT = 1;
  for (const BlockSpan &b : blocks) {
    if (b.kind == 1) {
      for (int64_t k = b.k0; k < b.k1; ++k) bk.push_back(k);
      continue;
    }
    capT = std::max(capT, t_limbs(slices_for(b.ha), slices_for(b.hb)));
    ++nS;
  }
  if (nS == 0 && !forced) return kNotApplicable;   // only dot products: the limb kernel
  int cap = std::max(A->re.cap, B->re.cap);
  if (sh.cplx) cap = std::max(cap, std::max(A->im.cap, B->im.cap));
  LimbShape ls;
  if (!limb_shape_for((int)p, nS + (int64_t)bk.size() * sh.nparts, cap, &ls)) return not_here("precision too large");
  if (!sh.approx && (radA || radB)) {
    rc = radius_products(ctx, A, B, sh, rin_m, rin_e, s);
    if (rc) return rc;
  }
  const int64_t MN = sh.M * sh.N;
  const size_t tcount = (size_t)sh.nparts * nS * MN;   // exact block values
  const size_t tbytes = tcount * (sizeof(uint32_t) * capT + 2 * sizeof(int32_t));
  char *tw = (char *)ws_get(ctx, WS_BLOCKS, round_up(tbytes, 8) + sizeof(int64_t) * (bk.size() + 1));
  if (!tw) return ARBGPU_ENOMEM;
  uint32_t *tl = (uint32_t *)tw;
  int32_t *te = (int32_t *)(tl + tcount * capT);
  int32_t *tn = te + tcount;
  int64_t *dbk = (int64_t *)(tw + round_up(tbytes, 8));
  if (!bk.empty()) {
    ARB_TRY(hipMemcpyAsync(dbk, bk.data(), sizeof(int64_t) * bk.size(), hipMemcpyHostToDevice, s), "basecase upload");
    ARB_TRY(hipStreamSynchronize(s), "basecase upload");
  }
  // part q, block si: limb plane k of entry ij at tl[q*nS*MN*capT + k*nS*MN + si*MN + ij]
  const int64_t ldT = (int64_t)nS * MN;
  int si = 0;
  for (size_t bi = 0; bi < blocks.size(); ++bi) {
    const BlockSpan &b = blocks[bi];
    if (b.kind == 1) continue;
    const int32_t *bst = bstats + (int64_t)bi * bstride;
    arbgpu_out tout[2];
    for (int q = 0; q < sh.nparts; ++q) {
      const size_t e0 = (size_t)q * nS * MN + (size_t)si * MN;
      tout[q] = arbgpu_out{tl + (size_t)q * nS * MN * capT + (size_t)si * MN, ldT, capT, te + e0, tn + e0,
                           nullptr, nullptr, nullptr};
    }
    double *no_m[2] = {nullptr, nullptr};
    int32_t *no_e[2] = {nullptr, nullptr};
    const int64_t ktb = sh.cplx ? 2 * (b.k1 - b.k0) : b.k1 - b.k0;
    const bool rns = use_rns(b.ha, b.hb, ktb) && rns_fits(b.ha, b.hb, ktb);
    rc = block_product(ctx, A, B, sh, b.k0, b.k1, bst, b.ha, b.hb, tout, 0, sh.N, 1, 32 * capT, true, no_m, no_e, s,
                       rns, (flags & ARBGPU_COMPLEX_4M) != 0, nullptr, false, bpre);
    if (rc) return rc;
    ++si;
  }
  for (int q = 0; q < sh.nparts; ++q) {
    MergeParams mp;
    memset(&mp, 0, sizeof mp);
    mp.T = arbgpu_arr{tl + (size_t)q * nS * MN * capT, ldT, capT, te + (size_t)q * nS * MN,
                      tn + (size_t)q * nS * MN, nullptr, nullptr};
    mp.nS = nS;
    mp.A[0] = A->re;
    mp.A[1] = sh.cplx ? A->im : A->re;
    mp.B[0] = B->re;
    mp.B[1] = sh.cplx ? B->im : B->re;
    mp.a_off = A->off; mp.a_rs = A->rs; mp.a_cs = A->cs;
    mp.b_off = B->off; mp.b_rs = B->rs; mp.b_cs = B->cs;
    mp.bk = dbk;
    mp.nbk = (int64_t)bk.size();
    mp.ct = !sh.cplx ? comp_real() : (q == 0 ? comp_re() : comp_im());
    mp.M = sh.M; mp.N = sh.N;
    mp.C = outs[q];
    mp.c_off = C->off; mp.c_rs = C->rs; mp.c_cs = C->cs;
    mp.p = (int)p;
    mp.approx = sh.approx;
    mp.rin_m = rin_m[q];
    mp.rin_e = rin_e[q];
    KernelTimer tmg(ctx, "merge", s);
    ARB_TRY(launch_merge(mp, ls.ns, s), "merge");
  }
  return ARBGPU_OK;
}

int exact_block_product(arbgpu_ctx *ctx, uint32_t *T_re, uint32_t *T_im, int64_t ldT, int32_t capT, int32_t *row_v2,
                        int32_t *col_v2, const arbgpu_mat *A, const arbgpu_mat *B, uint32_t flags, hipStream_t s) {
  Shape sh{(flags & ARBGPU_COMPLEX) != 0, true, (flags & ARBGPU_COMPLEX) ? 2 : 1, A->rows, B->cols, A->cols};
  const int64_t Kt = sh.cplx ? 2 * sh.K : sh.K;
  int32_t *st = stats_ws(ctx, sh);
  if (!st) return ARBGPU_ENOMEM;
  int32_t g[8];
  int rc = line_stats(ctx, A, B, sh, 0, sh.K, st, s, g);
  if (rc) return rc;
  if (g[2] || g[6]) return set_error(ctx, ARBGPU_ERANGE, "an operand exponent is outside (-2^28, 2^28)");
  if (slices_for(g[0]) > kMaxSlices || slices_for(g[4]) > kMaxSlices)
    return set_error(ctx, ARBGPU_EINVAL, "exact block product: integer height too large");
  bool rns;
  if (flags & ARBGPU_ALGO_RNS) rns = true;
  else if (flags & ARBGPU_ALGO_SLICED) rns = false;
  else rns = rns_better(g[0], g[4], Kt);
  if (rns && !rns_fits(g[0], g[4], Kt))
    return set_error(ctx, ARBGPU_EINVAL, "exact block product: the residue form does not fit these heights");
  if (!rns && ((int64_t)0x7FFFFFFF) / (round_up(std::max<int64_t>(Kt, 1), kKStep) << 14) < 1)
    return set_error(ctx, ARBGPU_EINVAL, "exact block product: inner length %lld too long", (long long)Kt);
  const int need = rns ? (int)((t_bits(g[0], g[4], Kt) + 1 + 31) / 32) + 1 : t_limbs(slices_for(g[0]), slices_for(g[4]));
  if (capT < need) return set_error(ctx, ARBGPU_EINVAL, "exact block product: T needs %d limbs, cap is %d", need, capT);
  if (ldT < sh.M * sh.N) return set_error(ctx, ARBGPU_EINVAL, "exact block product: ldT below rows * cols");
  ARB_TRY(launch_v2_out(st + sh.M, sh.M, row_v2, s), "scalings");
  ARB_TRY(launch_v2_out(st + 2 * sh.M + sh.N, sh.N, col_v2, s), "scalings");
  const TSink ts{{T_re, T_im}, ldT, capT};
  // the rounded outputs are not wanted: a sink without exponents writes none
  const arbgpu_out none[2] = {arbgpu_out{nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr},
                              arbgpu_out{nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr}};
  double *no_m[2] = {nullptr, nullptr};
  int32_t *no_e[2] = {nullptr, nullptr};
  return block_product(ctx, A, B, sh, 0, sh.K, st, g[0], g[4], none, 0, sh.N, 1, 2, true, no_m, no_e, s, rns,
                       (flags & ARBGPU_COMPLEX_4M) != 0, &ts);
}

std::string mat_mul_class(const arbgpu_mat *A, const arbgpu_mat *B, int64_t p, uint32_t flags) {
  const bool cplx = flags & ARBGPU_COMPLEX;
  const bool rad = !(flags & ARBGPU_APPROX) && (A->re.rad_m || B->re.rad_m || (cplx && (A->im.rad_m || B->im.rad_m)));
  return std::string("mat_mul:") + (cplx ? "c" : "r") + (rad ? "b" : "m") + ":n" +
         std::to_string(ceil_log2(std::max(A->rows, B->cols))) + ":k" + std::to_string(ceil_log2(A->cols)) + ":p" +
         std::to_string(ceil_log2(p));
}

}  // namespace arbgpu_impl
