"""GPU parity of the limb-window kernels (Algorithm 1 per output) against
the exact oracle, through the C-ABI."""

import random

import numpy as np
import pytest

import oracle
from paper_1901_04289_amd import arbgpu, gen
from tests.arbcheck import compare_entry

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = arbgpu.Context(0)
    yield c
    c.close()


def _sync():
    import torch
    torch.cuda.synchronize()


def say(msg):
    print(msg, flush=True)


def run_matmul(ctx, A, B, M, N, K, p, flags=0, Ai=None, Bi=None):
    dA, dB = arbgpu.DeviceArray.from_host(A), arbgpu.DeviceArray.from_host(B)
    dAi = arbgpu.DeviceArray.from_host(Ai) if Ai is not None else None
    dBi = arbgpu.DeviceArray.from_host(Bi) if Bi is not None else None
    rad = not (flags & arbgpu.APPROX)
    C = arbgpu.DeviceOut.empty(M * K, p, radius=rad)
    Ci = arbgpu.DeviceOut.empty(M * K, p, radius=rad) if flags & arbgpu.COMPLEX else None
    ctx.mat_mul(C, dA, dB, M, N, K, p, flags, Ci=Ci, Ai=dAi, Bi=dBi)
    _sync()
    return C.to_host(), (Ci.to_host() if Ci is not None else None)


def check_real(out, status, want, entries, K, approx=False):
    bad = []
    for (i, j) in entries:
        e = compare_entry(gen.to_canonical(out, i * K + j), want(i, j), int(status[i * K + j]), approx)
        if e:
            bad.append(((i, j), e))
    assert not bad, bad[:5]


def test_config0_full_parity(ctx):
    w = gen.config0()
    say(f"config0 limb matmul {w.M}x{w.N}x{w.K} p={w.p}")
    (out, st), _ = run_matmul(ctx, w.A, w.B, w.M, w.N, w.K, w.p, arbgpu.ALGO_LIMB)
    Ac = gen.canonical_matrix(w.A, w.M, w.N, w.N, 1)
    Bc = gen.canonical_matrix(w.B, w.N, w.K, w.K, 1)
    C = oracle.mat_mul(Ac, Bc, w.p)
    check_real(out, st, lambda i, j: C[i][j], [(i, j) for i in range(w.M) for j in range(w.K)], w.K)
    # exact inputs: every radius is the truncation ulp only
    assert (st <= 1).all()


@pytest.mark.parametrize("seed,M,N,K,p,prec,erange,rshift", [
    (1, 5, 37, 70, 100, 120, 20, 110),
    (2, 9, 1, 65, 2, 64, 3, None),
    (3, 66, 13, 3, 333, 400, 60, 300),
    (4, 4, 200, 4, 64, 200, 5, None),
    (5, 1, 64, 1, 1000, 1100, 10, 1000),
])
def test_random_matmul_parity(ctx, seed, M, N, K, p, prec, erange, rshift):
    rng = gen.rng_for(10, seed)
    A = gen.random_operands(rng, M * N, rng.integers(1, prec + 1, M * N), -erange, erange,
                            radius_shift=rshift, zero_frac=0.1)
    B = gen.random_operands(rng, N * K, rng.integers(1, prec + 1, N * K), -erange, erange, zero_frac=0.1)
    if M > 2:
        A.limbs[:, N:2 * N] = 0   # an all-zero row
        A.nls[N:2 * N] = 0
    say(f"random matmul seed={seed} {M}x{N}x{K} p={p}")
    (out, st), _ = run_matmul(ctx, A, B, M, N, K, p)
    Ac = gen.canonical_matrix(A, M, N, N, 1)
    Bc = gen.canonical_matrix(B, N, K, K, 1)
    ent = [(i, j) for i in range(M) for j in range(K)]
    if len(ent) > 300:
        ent = random.Random(seed).sample(ent, 300)
    cols = {j: [Bc[k][j] for k in range(N)] for j in range(K)}
    check_real(out, st, lambda i, j: oracle.dot(Ac[i], cols[j], p), ent, K)


def test_approx_and_strided_views(ctx):
    rng = gen.rng_for(11, 0)
    M, N, K, p = 6, 20, 9, 80
    A = gen.random_operands(rng, M * N, 100, -10, 10, radius_shift=90)
    B = gen.random_operands(rng, K * N, 100, -10, 10)   # stored K x N; used transposed
    dA, dB = arbgpu.DeviceArray.from_host(A), arbgpu.DeviceArray.from_host(B)
    C = arbgpu.DeviceOut.empty(M * K, p, radius=False)
    am = arbgpu.Mat(dA.arr(), dA.arr(), M, N, 0, N, 1)
    bm = arbgpu.Mat(dB.arr(), dB.arr(), N, K, 0, 1, N)          # B^T view
    cm = arbgpu.OMat(C.out(), C.out(), M, K, (M - 1) * K, -K, 1)  # rows written bottom-up
    say("approx strided matmul")
    ctx.mat_mul_raw(cm, am, bm, p, arbgpu.APPROX)
    _sync()
    out, st = C.to_host()
    Ac = gen.canonical_matrix(A, M, N, N, 1)
    Bt = gen.canonical_matrix(B, K, N, N, 1)
    for i in range(M):
        for j in range(K):
            want = oracle.dot(Ac[i], Bt[j], p, approx=True)
            idx = (M - 1 - i) * K + j
            assert compare_entry(gen.to_canonical(out, idx), want, int(st[idx]), approx=True) is None


def test_complex_matmul(ctx):
    rng = gen.rng_for(12, 0)
    M, N, K, p = 4, 15, 5, 90
    parts = [gen.random_operands(rng, c, 100, -12, 12, radius_shift=95, zero_frac=0.1)
             for c in (M * N, M * N, N * K, N * K)]
    say("complex matmul")
    (out, st), (outi, sti) = run_matmul(ctx, parts[0], parts[2], M, N, K, p, arbgpu.COMPLEX,
                                         Ai=parts[1], Bi=parts[3])
    A = [[(gen.to_canonical(parts[0], i * N + k), gen.to_canonical(parts[1], i * N + k)) for k in range(N)]
         for i in range(M)]
    B = [[(gen.to_canonical(parts[2], k * K + j), gen.to_canonical(parts[3], k * K + j)) for j in range(K)]
         for k in range(N)]
    C = oracle.cmat_mul(A, B, p)
    for i in range(M):
        for j in range(K):
            re, im = C[i][j]
            assert compare_entry(gen.to_canonical(out, i * K + j), re, int(st[i * K + j])) is None
            assert compare_entry(gen.to_canonical(outi, i * K + j), im, int(sti[i * K + j])) is None


def _dot_case(ctx, X, Y, I, N, p, xoff, xstep, yoff, ystep, sub, flags, Xi=None, Yi=None, Ii=None):
    dX, dY = arbgpu.DeviceArray.from_host(X), arbgpu.DeviceArray.from_host(Y)
    parts_x, parts_y = [dX.arr()], [dY.arr()]
    dI = arbgpu.DeviceArray.from_host(I) if I is not None else None
    parts_i = [dI.arr()] if dI is not None else None
    keep = [dX, dY, dI]
    if flags & arbgpu.COMPLEX:
        dXi, dYi = arbgpu.DeviceArray.from_host(Xi), arbgpu.DeviceArray.from_host(Yi)
        keep += [dXi, dYi]
        parts_x.append(dXi.arr())
        parts_y.append(dYi.arr())
        if I is not None:
            dIi = arbgpu.DeviceArray.from_host(Ii)
            keep.append(dIi)
            parts_i.append(dIi.arr())
    rad = not (flags & arbgpu.APPROX)
    outs = [arbgpu.DeviceOut.empty(3, p, radius=rad) for _ in parts_x]
    ctx.dot_raw([o.out() for o in outs], 1, parts_i, 0, sub, parts_x, xoff, xstep, parts_y, yoff, ystep, N, p,
                flags)
    _sync()
    return [o.to_host() for o in outs]


@pytest.mark.parametrize("seed", range(6))
def test_dot_variants(ctx, seed):
    r = random.Random(seed)
    rng = gen.rng_for(13, seed)
    N = [0, 1, 7, 64, 200, 1500][seed]
    L = max(N * 3, 1) + 2
    p = [2, 53, 128, 300, 700, 64][seed]
    cplx = seed % 2 == 1
    approx = seed == 4
    X = gen.random_operands(rng, L, rng.integers(1, 2 * p + 2, L), -30, 30, radius_shift=p + 5, zero_frac=0.05)
    Y = gen.random_operands(rng, L, rng.integers(1, 2 * p + 2, L), -30, 30, zero_frac=0.05)
    Xi = gen.random_operands(rng, L, rng.integers(1, 2 * p + 2, L), -30, 30, radius_shift=p + 3) if cplx else None
    Yi = gen.random_operands(rng, L, rng.integers(1, 2 * p + 2, L), -30, 30) if cplx else None
    I = gen.random_operands(rng, 1, p + 10, -5, 5, radius_shift=p) if seed % 3 != 0 else None
    Ii = gen.random_operands(rng, 1, p + 10, -5, 5) if (cplx and I is not None) else None
    xstep, ystep = [(1, 1), (-1, 2), (0, 1), (3, -2), (1, 1), (2, -1)][seed]
    xoff = 0 if xstep >= 0 else (N - 1) * -xstep
    yoff = 0 if ystep >= 0 else (N - 1) * -ystep
    sub = seed % 2 == 0
    flags = (arbgpu.COMPLEX if cplx else 0) | (arbgpu.APPROX if approx else 0)
    say(f"dot seed={seed} N={N} p={p} cplx={cplx} approx={approx}")
    res = _dot_case(ctx, X, Y, I, N, p, xoff, xstep, yoff, ystep, sub, flags, Xi, Yi, Ii)
    xs = [xoff + t * xstep for t in range(N)]
    ys = [yoff + t * ystep for t in range(N)]
    if not cplx:
        want = oracle.dot([gen.to_canonical(X, k) for k in xs], [gen.to_canonical(Y, k) for k in ys], p,
                          initial=gen.to_canonical(I, 0) if I is not None else None, sub=sub, approx=approx)
        (out, st), = res
        assert compare_entry(gen.to_canonical(out, 1), want, int(st[1]), approx) is None
    else:
        xc = [(gen.to_canonical(X, k), gen.to_canonical(Xi, k)) for k in xs]
        yc = [(gen.to_canonical(Y, k), gen.to_canonical(Yi, k)) for k in ys]
        ic = (gen.to_canonical(I, 0), gen.to_canonical(Ii, 0)) if I is not None else None
        wre, wim = oracle.cdot(xc, yc, p, initial=ic, sub=sub, approx=approx)
        (o_re, s_re), (o_im, s_im) = res
        assert compare_entry(gen.to_canonical(o_re, 1), wre, int(s_re[1]), approx) is None
        assert compare_entry(gen.to_canonical(o_im, 1), wim, int(s_im[1]), approx) is None


ONE = (0, 1, 1)


def _balls_dot(ctx, xb, yb, p, sub=False, cap=None):
    X = gen.from_canonical(xb, cap)
    Y = gen.from_canonical(yb, cap)
    (out, st), = _dot_case(ctx, X, Y, None, len(xb), p, 0, 1, 0, 1, sub, 0)
    if int(st[1]) == arbgpu.ST_ERANGE:
        return None, int(st[1])
    return gen.to_canonical(out, 1), int(st[1])


def test_adversarial_dots(ctx):
    x = (0, (1 << 127) | 12345, 3)
    cases = [
        ("cancel below window", [(x, None), ((0, 1, -700), None), ((1, 1, -700), None)], [(ONE, None)] * 3, 128),
        ("near boundary +", [(x, None), ((0, 1, -300), None)], [(ONE, None)] * 2, 128),
        ("near boundary -", [(x, None), ((1, 1, -300), None)], [(ONE, None)] * 2, 128),
        ("near boundary - p120", [(x, None), ((1, 1, -300), None)], [(ONE, None)] * 2, 120),
        ("power of two minus tiny", [((0, 1, 10), None), ((1, 1, -500), None)], [(ONE, None)] * 2, 128),
        ("terms miss window", [((0, 3, 100), None), ((0, 5, -5000), None), ((1, 7, -9000), None)],
         [(ONE, None)] * 3, 64),
        ("cancel to tiny", [((0, (1 << 100) | 1, 50), None), ((1, (1 << 100) | 1, 50), None), ((0, 3, -3000), None)],
         [(ONE, None)] * 3, 64),
        ("p=2 N=1", [((0, 0b10111, 4), None)], [((0, 0b111, 3), None)], 2),
        ("zero mids with radii", [((0, 0, 0), (5, -20)), ((0, 3, 2), (1, -40))], [(ONE, (3, -30)), ((0, 0, 0), None)], 64),
        ("exact zero with radius", [(x, (1, -200)), ((1,) + x[1:], None)], [(ONE, None)] * 2, 64),
    ]
    for name, xb, yb, p in cases:
        say(f"adversarial dot: {name}")
        got = _balls_dot(ctx, xb, yb, p)
        want = oracle.dot(xb, yb, p)
        e = compare_entry(got[0], want, got[1])
        assert e is None, (name, e)


def test_refinement_with_wide_operands(ctx):
    # operands wider than the register limbs: cancellation forces the exact
    # streaming path
    r = random.Random(5)
    for t in range(12):
        n = r.randint(2, 9)
        xb = [(oracle.fmake(r.getrandbits(1), r.getrandbits(1500) | (1 << 1499) | 1, r.randint(-20, 20)), None)
              for _ in range(n)]
        yb = [(oracle.fmake(r.getrandbits(1), r.getrandbits(1500) | (1 << 1499) | 1, r.randint(-20, 20)), None)
              for _ in range(n)]
        xb[1] = (oracle.fneg(xb[0][0]), None)
        yb[1] = yb[0]
        p = r.randint(2, 100)
        say(f"wide-operand refinement t={t} n={n} p={p}")
        got = _balls_dot(ctx, xb, yb, p)
        want = oracle.dot(xb, yb, p)
        assert compare_entry(got[0], want, got[1]) is None, t


def test_exponent_out_of_range_is_flagged(ctx):
    xb = [((0, 1, 2**28), None), ((0, 1, 1), None)]
    yb = [(ONE, None), (ONE, None)]
    say("erange dot")
    got = _balls_dot(ctx, xb, yb, 64)
    assert got[1] == arbgpu.ST_ERANGE


def test_config1_sampled(ctx):
    w = gen.config1()
    say(f"config1 limb matmul {w.M}x{w.N}x{w.K} p={w.p}")
    (out, st), _ = run_matmul(ctx, w.A, w.B, w.M, w.N, w.K, w.p, arbgpu.ALGO_LIMB)
    r = random.Random(1)
    ent = [(r.randrange(w.M), r.randrange(w.K)) for _ in range(40)]
    rows = {i: [gen.to_canonical(w.A, i * w.N + k) for k in range(w.N)] for i, _ in ent}
    cols = {j: [gen.to_canonical(w.B, k * w.K + j) for k in range(w.N)] for _, j in ent}
    check_real(out, st, lambda i, j: oracle.dot(rows[i], cols[j], w.p), ent, w.K)
    assert (st <= 1).all()


def test_config2_row_block_sampled(ctx):
    w = gen.config2()
    M = 64   # a row block of the 2048 x 2048 x 2048 product, full inner length
    A = gen.Operands(w.A.limbs[:, :M * w.N].copy(), w.A.exp[:M * w.N].copy(), w.A.nls[:M * w.N].copy(), None, None)
    say(f"config2 limb matmul row block {M}x{w.N}x{w.K} p={w.p}")
    (out, st), _ = run_matmul(ctx, A, w.B, M, w.N, w.K, w.p, arbgpu.ALGO_LIMB)
    r = random.Random(2)
    ent = [(r.randrange(M), r.randrange(w.K)) for _ in range(12)]
    rows = {i: [gen.to_canonical(A, i * w.N + k) for k in range(w.N)] for i, _ in ent}
    cols = {j: [gen.to_canonical(w.B, k * w.K + j) for k in range(w.N)] for _, j in ent}
    check_real(out, st, lambda i, j: oracle.dot(rows[i], cols[j], w.p), ent, w.K)
    assert (st <= 1).all()


def test_long_dot_on_four_waves_equals_batch_and_oracle(ctx):
    # a single dot of 1024 real terms or more runs on a workgroup of four
    # waves; the same dot inside a batch runs on one wave: window sums are
    # modular and the radius sum exact, so every bit agrees
    import torch
    rng = gen.rng_for(37, 0)
    for N, p, cplx in ((1500, 200, False), (5000, 64, False), (700, 512, True)):
        nparts = 2 if cplx else 1
        X = [gen.random_operands(rng, N, rng.integers(1, p + 40, N), -20, 20, radius_shift=p, zero_frac=0.02)
             for _ in range(nparts)]
        Y = [gen.random_operands(rng, N, rng.integers(1, p + 40, N), -20, 20, radius_shift=p - 5)
             for _ in range(nparts)]
        dX = [arbgpu.DeviceArray.from_host(x) for x in X]
        dY = [arbgpu.DeviceArray.from_host(y) for y in Y]
        flags = arbgpu.COMPLEX if cplx else 0
        single = [arbgpu.DeviceOut.empty(1, p) for _ in range(nparts)]
        batched = [arbgpu.DeviceOut.empty(1, p) for _ in range(nparts)]
        say(f"four-wave dot N={N} p={p} complex={cplx}")
        ctx.dot_raw([o.out() for o in single], 0, None, 0, False, [d.arr() for d in dX], 0, 1,
                    [d.arr() for d in dY], 0, 1, N, p, flags)
        b = arbgpu.Batch(ctx, [arbgpu.dot_job([o.out() for o in batched], 0, [d.arr() for d in dX], 0, 1,
                                              [d.arr() for d in dY], 0, 1, N, p, flags)])
        b.launch()
        torch.cuda.synchronize()
        b.close()
        for q in range(nparts):
            (a, sa), (c, sc) = single[q].to_host(), batched[q].to_host()
            assert np.array_equal(a.limbs, c.limbs) and np.array_equal(a.exp, c.exp)
            assert np.array_equal(a.nls, c.nls) and np.array_equal(sa, sc)
            assert np.array_equal(a.rad_m, c.rad_m) and np.array_equal(a.rad_e, c.rad_e)
        if cplx:
            xs = [(gen.to_canonical(X[0], k), gen.to_canonical(X[1], k)) for k in range(N)]
            ys = [(gen.to_canonical(Y[0], k), gen.to_canonical(Y[1], k)) for k in range(N)]
            want = oracle.cdot(xs, ys, p)
        else:
            want = (oracle.dot([gen.to_canonical(X[0], k) for k in range(N)],
                               [gen.to_canonical(Y[0], k) for k in range(N)], p),)
        for q in range(nparts):
            ops, st = single[q].to_host()
            assert compare_entry(gen.to_canonical(ops, 0), want[q], int(st[0])) is None, (N, p, q)


def test_small_products_wave_per_entry_match_oracle(ctx):
    # products with few entries run a wave per entry (terms split over the
    # lanes); every entry against the oracle, real and complex, balls
    rng = gen.rng_for(38, 0)
    for M, N, K, p, cplx in ((3, 200, 5, 128, False), (7, 33, 2, 300, True), (1, 1, 1, 64, False)):
        parts = [gen.random_operands(rng, c, rng.integers(1, p + 30, c), -8, 8, radius_shift=p, zero_frac=0.05)
                 for c in ((M * N, N * K) * (2 if cplx else 1))]
        A, B = parts[0], parts[1]
        Ai, Bi = (parts[2], parts[3]) if cplx else (None, None)
        say(f"wave-per-entry product {M}x{N}x{K} p={p} complex={cplx}")
        (out, st), im = run_matmul(ctx, A, B, M, N, K, p, arbgpu.ALGO_LIMB | (arbgpu.COMPLEX if cplx else 0),
                                   Ai=Ai, Bi=Bi)
        for i in range(M):
            for j in range(K):
                if cplx:
                    x = [(gen.to_canonical(A, i * N + k), gen.to_canonical(Ai, i * N + k)) for k in range(N)]
                    y = [(gen.to_canonical(B, k * K + j), gen.to_canonical(Bi, k * K + j)) for k in range(N)]
                    re, imv = oracle.cdot(x, y, p)
                    assert compare_entry(gen.to_canonical(out, i * K + j), re, int(st[i * K + j])) is None
                    (oi, si) = im
                    assert compare_entry(gen.to_canonical(oi, i * K + j), imv, int(si[i * K + j])) is None
                else:
                    want = oracle.dot([gen.to_canonical(A, i * N + k) for k in range(N)],
                                      [gen.to_canonical(B, k * K + j) for k in range(N)], p)
                    assert compare_entry(gen.to_canonical(out, i * K + j), want, int(st[i * K + j])) is None
