"""GPU parity of dot products beyond the register windows (the LDS-window
kernel, any p up to its limit; Table 1 of the paper goes to 13568 bits)
against the exact oracle, through the C-ABI: real and complex, initial
values, sub, balls, cancellation that needs the exact window, the
precision cut, and wide dots inside a resident batch."""

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


def say(msg):
    print(msg, flush=True)


def dev(ops):
    return arbgpu.DeviceArray.from_host(ops)


def run_dot(ctx, xs, ys, N, p, flags=0, init=None, sub=False, xstep=1, ystep=1, xoff=0, yoff=0):
    import torch
    n = len(xs)
    outs = [arbgpu.DeviceOut.empty(1, p, radius=not (flags & arbgpu.APPROX)) for _ in range(n)]
    ctx.dot_raw([o.out() for o in outs], 0, [i.arr() for i in init] if init else None, 0, sub,
                [x.arr() for x in xs], xoff, xstep, [y.arr() for y in ys], yoff, ystep, N, p, flags)
    torch.cuda.synchronize()
    return [o.to_host() for o in outs]


@pytest.mark.parametrize("seed,N,p,prec,cplx,rad,with_init,sub", [
    (1, 1, 1300, 1400, False, False, False, False),
    (2, 7, 2048, 2100, False, True, True, False),
    (3, 100, 4096, 4200, False, True, False, True),
    (4, 30, 4096, 3000, True, True, True, False),
    (5, 12, 13568, 13600, False, False, True, True),
    (6, 3, 13568, 14000, True, True, False, False),
])
def test_wide_dot_matches_oracle(ctx, seed, N, p, prec, cplx, rad, with_init, sub):
    rng = gen.rng_for(80, seed)
    nparts = 2 if cplx else 1
    rs = p - 8 if rad else None
    X = [gen.random_operands(rng, N, rng.integers(1, prec + 1, N), -30, 30, radius_shift=rs, zero_frac=0.05)
         for _ in range(nparts)]
    Y = [gen.random_operands(rng, N, rng.integers(1, prec + 1, N), -30, 30, radius_shift=rs, zero_frac=0.05)
         for _ in range(nparts)]
    I = [gen.random_operands(rng, 1, prec, -20, 20, radius_shift=rs) for _ in range(nparts)] if with_init else None
    say(f"wide dot seed={seed} N={N} p={p} complex={cplx}")
    flags = arbgpu.COMPLEX if cplx else 0
    res = run_dot(ctx, [dev(x) for x in X], [dev(y) for y in Y], N, p, flags,
                  init=[dev(i) for i in I] if I else None, sub=sub)
    if cplx:
        xs = [(gen.to_canonical(X[0], k), gen.to_canonical(X[1], k)) for k in range(N)]
        ys = [(gen.to_canonical(Y[0], k), gen.to_canonical(Y[1], k)) for k in range(N)]
        init = (gen.to_canonical(I[0], 0), gen.to_canonical(I[1], 0)) if I else None
        want = oracle.cdot(xs, ys, p, initial=init, sub=sub)
    else:
        xs = [gen.to_canonical(X[0], k) for k in range(N)]
        ys = [gen.to_canonical(Y[0], k) for k in range(N)]
        init = gen.to_canonical(I[0], 0) if I else None
        want = (oracle.dot(xs, ys, p, initial=init, sub=sub),)
    for q, w in enumerate(want):
        ops, st = res[q]
        e = compare_entry(gen.to_canonical(ops, 0), w, int(st[0]))
        assert e is None, (q, e)


def test_wide_dot_cancellation_needs_the_exact_window(ctx):
    # x . y with the second half of the terms the negated first half plus a
    # term 3000 bits below the rest: the window of p + guard bits cancels to
    # nothing, so the exact window decides (status REFINED), and a fully
    # cancelling dot gives an exact zero
    p = 2048
    rng = gen.rng_for(81, 0)
    n = 16
    A = gen.random_operands(rng, n, 2100, -5, 5)
    B = gen.random_operands(rng, n, 2100, -5, 5)
    a = [gen.to_canonical(A, k) for k in range(n)]
    b = [gen.to_canonical(B, k) for k in range(n)]
    xs = a + a + [(oracle.fmake(0, 12345, -3000), None)]
    ys = b + [(oracle.fneg(v[0]), None) for v in b] + [(oracle.fmake(0, 1, 1), None)]
    X, Y = gen.from_canonical(xs), gen.from_canonical(ys)
    for N in (2 * n + 1, 2 * n):
        say(f"wide dot cancellation N={N}")
        (ops, st), = run_dot(ctx, [dev(X)], [dev(Y)], N, p)
        want = oracle.dot(xs[:N], ys[:N], p)
        assert compare_entry(gen.to_canonical(ops, 0), want, int(st[0])) is None
        if N == 2 * n:
            assert ops.nls[0] == 0   # exact zero
        else:
            assert int(st[0]) == arbgpu.ST_REFINED


def test_wide_dot_precision_cut_and_approx(ctx):
    rng = gen.rng_for(82, 0)
    N, p = 40, 3000
    X = gen.random_operands(rng, N, 3000, -4, 4, radius_shift=200)
    Y = gen.random_operands(rng, N, 3000, -4, 4, radius_shift=200)
    xs = [gen.to_canonical(X, k) for k in range(N)]
    ys = [gen.to_canonical(Y, k) for k in range(N)]
    (ops, st), = run_dot(ctx, [dev(X)], [dev(Y)], N, p, arbgpu.REDUCE_PREC)
    want = oracle.dot(xs, ys, p, reduce_prec=True)
    assert compare_entry(gen.to_canonical(ops, 0), want, int(st[0])) is None
    (ops, st), = run_dot(ctx, [dev(X)], [dev(Y)], N, p, arbgpu.APPROX)
    want = oracle.dot(xs, ys, p, approx=True)
    assert compare_entry(gen.to_canonical(ops, 0), want, int(st[0]), True) is None


def test_wide_dots_in_a_batch(ctx):
    # a batch holding dots below and beyond the register windows: every
    # output equals the single call's
    import torch
    rng = gen.rng_for(83, 0)
    L = 300
    X = dev(gen.random_operands(rng, L, rng.integers(1, 3000, L), -10, 10, radius_shift=100))
    Y = dev(gen.random_operands(rng, L, rng.integers(1, 3000, L), -10, 10))
    r = random.Random(3)
    specs = [(r.randrange(0, 100), r.randint(0, 150), r.choice([64, 500, 1500, 2500, 4000])) for _ in range(40)]
    outs = arbgpu.DeviceOut.empty(len(specs), 4000)
    ref = arbgpu.DeviceOut.empty(len(specs), 4000)
    jobs = []
    for i, (off, N, p) in enumerate(specs):
        jobs.append(arbgpu.dot_job([outs.out()], i, [X.arr()], off, 1, [Y.arr()], off, 1, N, p))
        ctx.dot_raw([ref.out()], i, None, 0, False, [X.arr()], off, 1, [Y.arr()], off, 1, N, p)
    b = arbgpu.Batch(ctx, jobs)
    b.launch()
    torch.cuda.synchronize()
    (a, sa), (c, sc) = outs.to_host(), ref.to_host()
    assert np.array_equal(a.limbs, c.limbs) and np.array_equal(a.exp, c.exp) and np.array_equal(a.nls, c.nls)
    assert np.array_equal(sa, sc)
    b.close()
