"""GPU parity of the digit-product dot kernel (a dot as one small exact INT8
matrix product of operand digits, certified or handed back to the limb
kernel) against the exact oracle and against the limb kernel alone
(ARBGPU_ALGO_LIMB), through the C-ABI."""

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


def _run(ctx, dev, N, p, xoff, xstep, yoff, ystep, sub, flags, cplx):
    xs = [dev[0].arr()] + ([dev[1].arr()] if cplx else [])
    ys = [dev[2].arr()] + ([dev[3].arr()] if cplx else [])
    rad = not (flags & arbgpu.APPROX)
    outs = [arbgpu.DeviceOut.empty(3, p, radius=rad) for _ in xs]
    ctx.dot_raw([o.out() for o in outs], 1, None, 0, sub, xs, xoff, xstep, ys, yoff, ystep, N, p, flags)
    _sync()
    return [o.to_host() for o in outs]


def _want(host, N, p, xoff, xstep, yoff, ystep, sub, flags, cplx):
    xi = [xoff + t * xstep for t in range(N)]
    yi = [yoff + t * ystep for t in range(N)]
    approx = bool(flags & arbgpu.APPROX)
    red = bool(flags & arbgpu.REDUCE_PREC)
    if not cplx:
        return [oracle.dot([gen.to_canonical(host[0], k) for k in xi], [gen.to_canonical(host[2], k) for k in yi], p,
                           sub=sub, approx=approx, reduce_prec=red)]
    xc = [(gen.to_canonical(host[0], k), gen.to_canonical(host[1], k)) for k in xi]
    yc = [(gen.to_canonical(host[2], k), gen.to_canonical(host[3], k)) for k in yi]
    return list(oracle.cdot(xc, yc, p, sub=sub, approx=approx, reduce_prec=red))


def _same(a, b, approx):
    (oa, sa), (ob, sb) = a, b
    assert int(sa[1]) in (0, 1) and int(sb[1]) in (0, 1)
    assert np.array_equal(oa.limbs[:, 1], ob.limbs[:, 1]) and oa.exp[1] == ob.exp[1] and oa.nls[1] == ob.nls[1]
    if not approx:
        assert oa.rad_m[1] == ob.rad_m[1] and oa.rad_e[1] == ob.rad_e[1]


CASES = [
    # N, p, complex, flags, exponent range, strides (x, y)
    (1, 64, False, 0, 16, (1, 1)),
    (5, 30, True, 0, 16, (1, 1)),
    (64, 128, True, 0, 16, (1, 1)),
    (100, 200, False, arbgpu.APPROX, 16, (2, -1)),
    (300, 512, True, 0, 16, (1, 3)),
    (131, 700, True, arbgpu.REDUCE_PREC, 8, (1, 1)),
    (1500, 1000, True, 0, 16, (1, 1)),
    (2100, 350, False, 0, 30, (-1, 1)),
    (4096, 100, True, 0, 16, (0, 1)),
    (999, 900, False, arbgpu.REDUCE_PREC, 4, (1, 1)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_digit_dot_matches_oracle_and_limb_kernel(ctx, case):
    N, p, cplx, flags, er, (xstep, ystep) = CASES[case]
    rng = gen.rng_for(60, case)
    L = max(N * abs(xstep), N * abs(ystep), 1) + 3
    host = [gen.random_operands(rng, L, rng.integers((p + 1) // 2, 2 * p + 1, L), -er, er,
                                radius_shift=(p + 7 if k % 2 == 0 else None), zero_frac=0.03) for k in range(4)]
    dev = [arbgpu.DeviceArray.from_host(h) for h in host]
    xoff = 1 if xstep >= 0 else 1 + (N - 1) * -xstep
    yoff = 2 if ystep >= 0 else 2 + (N - 1) * -ystep
    sub = case % 3 == 1
    fl = flags | (arbgpu.COMPLEX if cplx else 0)
    say(f"digit dot case={case} N={N} p={p} cplx={cplx} flags={flags:#x}")
    got = _run(ctx, dev, N, p, xoff, xstep, yoff, ystep, sub, fl, cplx)
    ref = _run(ctx, dev, N, p, xoff, xstep, yoff, ystep, sub, fl | arbgpu.ALGO_LIMB, cplx)
    approx = bool(flags & arbgpu.APPROX)
    for a, b in zip(got, ref):
        _same(a, b, approx)
    want = _want(host, N, p, xoff, xstep, yoff, ystep, sub, fl, cplx)
    for (o, st), w in zip(got, want):
        assert compare_entry(gen.to_canonical(o, 1), w, int(st[1]), approx) is None


def _balls(ctx, xb, yb, p, cplx=False, xbi=None, ybi=None, flags=0):
    host = [gen.from_canonical(xb), gen.from_canonical(xbi) if cplx else None,
            gen.from_canonical(yb), gen.from_canonical(ybi) if cplx else None]
    dev = [arbgpu.DeviceArray.from_host(h) if h is not None else None for h in host]
    fl = flags | (arbgpu.COMPLEX if cplx else 0)
    return host, _run(ctx, dev, len(xb), p, 0, 1, 0, 1, False, fl, cplx)


def test_digit_dot_hands_back_what_it_cannot_certify(ctx):
    r = random.Random(61)
    cases = []
    # long sums that cancel exactly down to one tiny term: the window cannot
    # decide, the limb kernel refines
    for n, p in [(300, 200), (900, 700)]:
        xs = [((r.randrange(2), r.getrandbits(p + 100) | 1 | (1 << (p + 99)), r.randrange(-10, 11)), None)
              for _ in range(n)]
        ys = [((0, r.getrandbits(p) | 1 | (1 << (p - 1)), r.randrange(-10, 11)), None) for _ in range(n)]
        X = xs + [((1 - s, M, e), rad) for (s, M, e), rad in xs] + [((0, 1, -400), None)]
        Y = ys + ys + [((0, 1, 1), None)]
        cases.append(("cancel", X, Y, p))
    # terms far below the top one: cut by the frame, counted in the bound
    X = [((0, r.getrandbits(120) | (1 << 119), e), None) for e in (300, -300, 5, 0)]
    Y = [((1, r.getrandbits(120) | (1 << 119), e), None) for e in (2, 280, -9, 700)]
    cases.append(("spread", X, Y, 100))
    # near a power of two: the sum sits just below one
    X = [((0, 1, 1), None), ((1, 1, -600), None)]
    Y = [((0, 1, 1), None), ((0, 1, 1), None)]
    cases.append(("below one", X, Y, 128))
    for name, X, Y, p in cases:
        say(f"digit hand-back: {name} n={len(X)} p={p}")
        host, got = _balls(ctx, X, Y, p)
        want = oracle.dot(X, Y, p)
        (o, st), = got
        assert compare_entry(gen.to_canonical(o, 1), want, int(st[1])) is None, name
    say("digit dot: exponent out of range")
    host, got = _balls(ctx, [((0, 1, 2**28), None), ((0, 1, 1), None)], [((0, 1, 1), None)] * 2, 64)
    (o, st), = got
    assert int(st[1]) == arbgpu.ST_ERANGE and np.isinf(o.rad_m[1])


def test_digit_dot_complex_cancellation_per_part(ctx):
    # the real part cancels exactly (handed back), the imaginary part does not
    r = random.Random(62)
    n, p = 200, 300
    xr = [((0, r.getrandbits(p) | 1 | (1 << (p - 1)), r.randrange(-5, 6)), None) for _ in range(n)]
    yr = [((0, r.getrandbits(p) | 1 | (1 << (p - 1)), r.randrange(-5, 6)), None) for _ in range(n)]
    xi, yi = list(xr), list(yr)   # re = sum xr yr - xi yi = 0 exactly
    host, got = _balls(ctx, xr, yr, p, cplx=True, xbi=xi, ybi=yi)
    xc = list(zip(xr, xi))
    yc = list(zip(yr, yi))
    wre, wim = oracle.cdot(xc, yc, p)
    (o_re, s_re), (o_im, s_im) = got
    assert compare_entry(gen.to_canonical(o_re, 1), wre, int(s_re[1])) is None
    assert compare_entry(gen.to_canonical(o_im, 1), wim, int(s_im[1])) is None
    # the parts' exponents 400 bits apart: no frame of blocks holds both, the
    # whole job goes back to the limb kernel
    xr = [((0, r.getrandbits(p) | (1 << (p - 1)), 200), None) for _ in range(9)]
    yi = [((1, r.getrandbits(p) | (1 << (p - 1)), 200), None) for _ in range(9)]
    xi = [((0, r.getrandbits(p) | (1 << (p - 1)), -200), None) for _ in range(9)]
    yr = [((0, r.getrandbits(p) | (1 << (p - 1)), -200), None) for _ in range(9)]
    host, got = _balls(ctx, xr, yr, p, cplx=True, xbi=xi, ybi=yi)
    wre, wim = oracle.cdot(list(zip(xr, xi)), list(zip(yr, yi)), p)
    (o_re, s_re), (o_im, s_im) = got
    assert compare_entry(gen.to_canonical(o_re, 1), wre, int(s_re[1])) is None
    assert compare_entry(gen.to_canonical(o_im, 1), wim, int(s_im[1])) is None


def test_long_digit_dot_equals_limb_kernel(ctx):
    rng = gen.rng_for(63, 0)
    N, p = 40000, 160
    host = [gen.random_operands(rng, N, rng.integers(80, 321, N), -16, 16, radius_shift=p + 3) for _ in range(4)]
    dev = [arbgpu.DeviceArray.from_host(h) for h in host]
    say(f"long digit dot N={N} p={p}")
    got = _run(ctx, dev, N, p, 0, 1, 0, 1, False, arbgpu.COMPLEX, True)
    ref = _run(ctx, dev, N, p, 0, 1, 0, 1, False, arbgpu.COMPLEX | arbgpu.ALGO_LIMB, True)
    for a, b in zip(got, ref):
        _same(a, b, False)


def test_batch_runs_digit_jobs_and_their_hand_backs(ctx):
    # a config-3 shaped batch plus jobs that cancel: digit runs, fallback
    # runs, and single calls agree bit for bit
    w = gen.config3(seed_salt=5, ndots=300, max_len=200)
    dev = [arbgpu.DeviceArray.from_host(o) for o in (w.x_re, w.x_im, w.y_re, w.y_im)]
    n = len(w.lengths)
    r = random.Random(64)
    m = 6
    X, Y = [], []
    for _ in range(m):
        xs = [((r.randrange(2), r.getrandbits(300) | 1 | (1 << 299), r.randrange(-5, 6)), None) for _ in range(40)]
        ys = [((0, r.getrandbits(300) | 1 | (1 << 299), r.randrange(-5, 6)), None) for _ in range(40)]
        X += xs + [((1 - s, M, e), rad) for (s, M, e), rad in xs] + [((0, 3, -500), None)]
        Y += ys + ys + [((0, 1, 1), None)]
    dX, dY = arbgpu.DeviceArray.from_host(gen.from_canonical(X)), arbgpu.DeviceArray.from_host(gen.from_canonical(Y))
    outs = [arbgpu.DeviceOut.empty(n + m, 1024), arbgpu.DeviceOut.empty(n + m, 1024)]
    refs = [arbgpu.DeviceOut.empty(n + m, 1024), arbgpu.DeviceOut.empty(n + m, 1024)]

    def jobs_for(o):
        jobs = []
        for i in range(n):
            jobs.append(arbgpu.dot_job([o[0].out(), o[1].out()], i, [dev[0].arr(), dev[1].arr()], int(w.offsets[i]), 1,
                                       [dev[2].arr(), dev[3].arr()], int(w.offsets[i]), 1, int(w.lengths[i]),
                                       int(w.precs[i]), arbgpu.COMPLEX))
        for k in range(m):
            jobs.append(arbgpu.dot_job([o[0].out()], n + k, [dX.arr()], 81 * k, 1, [dY.arr()], 81 * k, 1, 81, 250))
        return jobs

    b = arbgpu.Batch(ctx, jobs_for(outs))
    shapes = b.info()["shapes"]
    assert any(s["ns"] < 0 for s in shapes), shapes
    b.tune()
    b.launch()
    _sync()
    for j in jobs_for(refs):
        nparts = 2 if j.flags & arbgpu.COMPLEX else 1
        ctx.dot_raw([j.res[q] for q in range(nparts)], j.res_idx, None, 0, False, [j.x[q] for q in range(nparts)],
                    j.xoff, j.xstep, [j.y[q] for q in range(nparts)], j.yoff, j.ystep, j.N, j.p, j.flags)
    _sync()
    for o, rr in zip(outs, refs):
        (a, sa), (c, sc) = o.to_host(), rr.to_host()
        rows = slice(0, n) if o is outs[1] else slice(0, n + m)
        assert np.array_equal(a.limbs[:, rows], c.limbs[:, rows]) and np.array_equal(a.exp[rows], c.exp[rows])
        assert np.array_equal(a.nls[rows], c.nls[rows]) and np.array_equal(sa[rows], sc[rows])
        assert np.array_equal(a.rad_m[rows], c.rad_m[rows]) and np.array_equal(a.rad_e[rows], c.rad_e[rows])
    host, st = outs[0].to_host()
    for k in range(m):
        xb, yb = X[81 * k:81 * k + 81], Y[81 * k:81 * k + 81]
        assert compare_entry(gen.to_canonical(host, n + k), oracle.dot(xb, yb, 250), int(st[n + k])) is None
    b.close()
