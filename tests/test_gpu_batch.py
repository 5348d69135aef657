"""GPU parity of the resident dot batch (one graph launch of persistent
per-shape kernels, longest-first work queues) against the exact oracle and
against single arbgpu_dot calls, through the C-ABI."""

import random

import numpy as np
import pytest

import oracle
from paper_1901_04289_amd import arbgpu, gen
from tests.arbcheck import compare_entry

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    say("importing torch")
    import torch
    assert torch.cuda.is_available()
    c = arbgpu.Context(0)
    say("context ready")
    yield c
    c.close()


def say(msg):
    print(msg, flush=True)


def _sync():
    import torch
    torch.cuda.synchronize()


class Pool:
    """Operand arrays on the device and their host copies."""

    def __init__(self, ops):
        self.host = ops
        self.dev = arbgpu.DeviceArray.from_host(ops)
        self.arr = self.dev.arr()

    def ball(self, k):
        return gen.to_canonical(self.host, k)


def random_jobs(seed, njobs, cplx_frac=0.5):
    """A mix of real and complex jobs over shared operand pools: lengths
    0..2100, p 2..1100, narrow and wide operands, strides of both signs,
    initial values, sub, approx and the precision cut."""
    r = random.Random(seed)
    rng = gen.rng_for(40, seed)
    L = 8000   # the longest job (N = 2100, stride 3) reads up to index ~6400
    pools = {}
    for name, prec, rs in (("n", 100, 90), ("w", 2200, 700)):
        parts = [Pool(gen.random_operands(rng, L, rng.integers(1, prec + 1, L), -20, 20,
                                          radius_shift=rs if k % 2 == 0 else None, zero_frac=0.05))
                 for k in range(4)]
        pools[name] = parts
    inits = [Pool(gen.random_operands(rng, 64, 120, -4, 4, radius_shift=100)) for _ in range(2)]
    specs = []
    for i in range(njobs):
        N = r.choice([0, 1, 2, 5, 17, 64, 100, 300, 1500, 2100])
        p = r.choice([2, 30, 64, 100, 128, 200, 512, 700, 1100])
        pool = pools[r.choice("nw")]
        cplx = r.random() < cplx_frac
        xstep = r.choice([1, 1, 2, -1, 0])
        ystep = r.choice([1, 3, -2])
        xoff = r.randrange(0, 100) + (max(N - 1, 0) * -xstep if xstep < 0 else 0)
        yoff = r.randrange(0, 100) + (max(N - 1, 0) * -ystep if ystep < 0 else 0)
        flags = (arbgpu.COMPLEX if cplx else 0)
        if r.random() < 0.15:
            flags |= arbgpu.APPROX
        if r.random() < 0.2:
            flags |= arbgpu.REDUCE_PREC
        init = r.randrange(64) if r.random() < 0.3 else None
        specs.append(dict(N=N, p=p, pool=pool, cplx=cplx, xstep=xstep, ystep=ystep, xoff=xoff, yoff=yoff,
                          flags=flags, init=init, sub=r.random() < 0.3))
    return specs, inits


def make_jobs(specs, inits, outs):
    jobs = []
    for i, s in enumerate(specs):
        X = [s["pool"][0].arr, s["pool"][1].arr] if s["cplx"] else [s["pool"][0].arr]
        Y = [s["pool"][2].arr, s["pool"][3].arr] if s["cplx"] else [s["pool"][2].arr]
        R = [outs[0].out(), outs[1].out()] if s["cplx"] else [outs[0].out()]
        I = None
        if s["init"] is not None:
            I = [inits[0].arr, inits[1].arr] if s["cplx"] else [inits[0].arr]
        jobs.append(arbgpu.dot_job(R, i, X, s["xoff"], s["xstep"], Y, s["yoff"], s["ystep"], s["N"], s["p"],
                                   s["flags"], initial=I, init_idx=s["init"] or 0, sub=s["sub"]))
    return jobs


def oracle_of(s, inits):
    xs = [s["xoff"] + t * s["xstep"] for t in range(s["N"])]
    ys = [s["yoff"] + t * s["ystep"] for t in range(s["N"])]
    P = s["pool"]
    approx = bool(s["flags"] & arbgpu.APPROX)
    red = bool(s["flags"] & arbgpu.REDUCE_PREC)
    if not s["cplx"]:
        init = inits[0].ball(s["init"]) if s["init"] is not None else None
        return [oracle.dot([P[0].ball(k) for k in xs], [P[2].ball(k) for k in ys], s["p"], initial=init,
                           sub=s["sub"], approx=approx, reduce_prec=red)]
    init = (inits[0].ball(s["init"]), inits[1].ball(s["init"])) if s["init"] is not None else None
    return list(oracle.cdot([(P[0].ball(k), P[1].ball(k)) for k in xs], [(P[2].ball(k), P[3].ball(k)) for k in ys],
                            s["p"], initial=init, sub=s["sub"], approx=approx, reduce_prec=red))


def check_jobs(specs, inits, host_outs):
    bad = []
    for i, s in enumerate(specs):
        want = oracle_of(s, inits)
        for q, w in enumerate(want):
            ops, st = host_outs[q]
            e = compare_entry(gen.to_canonical(ops, i), w, int(st[i]), bool(s["flags"] & arbgpu.APPROX))
            if e:
                bad.append((i, q, s["N"], s["p"], s["cplx"], s["flags"], e))
    assert not bad, bad[:5]


@pytest.mark.parametrize("seed", [1, 2])
def test_batch_random_mix_matches_oracle(ctx, seed):
    specs, inits = random_jobs(seed, 160)
    outs = [arbgpu.DeviceOut.empty(len(specs), 1100), arbgpu.DeviceOut.empty(len(specs), 1100)]
    jobs = make_jobs(specs, inits, outs)
    say(f"batch random mix seed={seed} jobs={len(jobs)}")
    b = arbgpu.Batch(ctx, jobs)
    info = b.info()
    assert info["jobs"] == len(jobs) and info["tasks"] == sum(2 if s["cplx"] else 1 for s in specs)
    assert len(info["shapes"]) >= 3
    b.launch()
    _sync()
    say("batch done; checking against the oracle")
    host = [o.to_host() for o in outs]
    check_jobs(specs, inits, host)
    # a second launch of the same graph rewrites identical outputs
    for o in outs:
        o.limbs.zero_()
        o.exp.zero_()
    b.launch()
    _sync()
    again = [o.to_host() for o in outs]
    for (a, sa), (c, sc) in zip(host, again):
        assert np.array_equal(a.limbs, c.limbs) and np.array_equal(a.exp, c.exp) and np.array_equal(sa, sc)
    b.close()


def test_batch_equals_single_calls_and_survives_tuning(ctx):
    specs, inits = random_jobs(3, 120, cplx_frac=0.6)
    outs = [arbgpu.DeviceOut.empty(len(specs), 1100), arbgpu.DeviceOut.empty(len(specs), 1100)]
    ref = [arbgpu.DeviceOut.empty(len(specs), 1100), arbgpu.DeviceOut.empty(len(specs), 1100)]
    jobs = make_jobs(specs, inits, outs)
    rjobs = make_jobs(specs, inits, ref)
    say("batch vs single dots")
    for j in rjobs:
        n = 2 if j.flags & arbgpu.COMPLEX else 1
        init = [j.init[q] for q in range(n)] if j.init[0].limbs else None
        ctx.dot_raw([j.res[q] for q in range(n)], j.res_idx, init, j.init_idx, bool(j.sub),
                    [j.x[q] for q in range(n)], j.xoff, j.xstep, [j.y[q] for q in range(n)], j.yoff, j.ystep,
                    j.N, j.p, j.flags)
    b = arbgpu.Batch(ctx, jobs)
    b.tune()
    for o in outs:
        o.limbs.zero_()
    b.launch()
    _sync()
    for o, r in zip(outs, ref):
        (a, sa), (c, sc) = o.to_host(), r.to_host()
        assert np.array_equal(a.limbs, c.limbs) and np.array_equal(a.exp, c.exp)
        assert np.array_equal(a.nls, c.nls) and np.array_equal(sa, sc)
        assert np.array_equal(a.rad_m, c.rad_m) and np.array_equal(a.rad_e, c.rad_e)
    assert all(s["waves"] in (1, 2, 4, 8, 16) for s in b.info()["shapes"])
    b.close()


def test_batch_rejects_bad_job_with_index(ctx):
    specs, inits = random_jobs(4, 5)
    outs = [arbgpu.DeviceOut.empty(5, 1100), arbgpu.DeviceOut.empty(5, 1100)]
    jobs = make_jobs(specs, inits, outs)
    jobs[3].p = 1
    with pytest.raises(arbgpu.ArbgpuError) as ei:
        arbgpu.Batch(ctx, jobs)
    assert ei.value.code == arbgpu.EINVAL and "job 3" in str(ei.value)
    b = arbgpu.Batch(ctx, [])
    b.launch()
    _sync()
    b.close()


def config3_jobs(w, outs, dev):
    jobs = []
    for i in range(len(w.lengths)):
        jobs.append(arbgpu.dot_job([outs[0].out(), outs[1].out()], i, [dev[0].arr(), dev[1].arr()],
                                   int(w.offsets[i]), 1, [dev[2].arr(), dev[3].arr()], int(w.offsets[i]), 1,
                                   int(w.lengths[i]), int(w.precs[i]), arbgpu.COMPLEX))
    return jobs


def test_config3_small_batch_matches_oracle(ctx):
    w = gen.config3(seed_salt=1, ndots=400, max_len=256)
    say(f"config3-shaped batch: {len(w.lengths)} dots, {int(w.lengths.sum())} terms")
    dev = [arbgpu.DeviceArray.from_host(o) for o in (w.x_re, w.x_im, w.y_re, w.y_im)]
    outs = [arbgpu.DeviceOut.empty(len(w.lengths), 1024), arbgpu.DeviceOut.empty(len(w.lengths), 1024)]
    b = arbgpu.Batch(ctx, config3_jobs(w, outs, dev))
    b.launch()
    _sync()
    host = [o.to_host() for o in outs]
    r = random.Random(7)
    picks = r.sample(range(len(w.lengths)), 60) + [int(np.argmax(w.lengths)), int(np.argmax(w.precs))]
    for i in picks:
        o, n = int(w.offsets[i]), int(w.lengths[i])
        xs = [(gen.to_canonical(w.x_re, k), gen.to_canonical(w.x_im, k)) for k in range(o, o + n)]
        ys = [(gen.to_canonical(w.y_re, k), gen.to_canonical(w.y_im, k)) for k in range(o, o + n)]
        wre, wim = oracle.cdot(xs, ys, int(w.precs[i]))
        for (ops, st), want in zip(host, (wre, wim)):
            e = compare_entry(gen.to_canonical(ops, i), want, int(st[i]))
            assert e is None, (i, n, int(w.precs[i]), e)
    b.close()


@pytest.mark.slow
def test_config3_full_batch_sampled(ctx):
    w = gen.config3()
    say(f"config3 batch: {len(w.lengths)} dots, {int(w.lengths.sum())} terms")
    dev = [arbgpu.DeviceArray.from_host(o) for o in (w.x_re, w.x_im, w.y_re, w.y_im)]
    outs = [arbgpu.DeviceOut.empty(len(w.lengths), 1024), arbgpu.DeviceOut.empty(len(w.lengths), 1024)]
    b = arbgpu.Batch(ctx, config3_jobs(w, outs, dev))
    b.launch()
    _sync()
    host = [o.to_host() for o in outs]
    assert all(int(st.max()) <= 1 for _, st in host)
    r = random.Random(8)
    picks = r.sample(range(len(w.lengths)), 6) + [int(np.argmax(w.lengths))]
    for i in picks:
        o, n = int(w.offsets[i]), int(w.lengths[i])
        xs = [(gen.to_canonical(w.x_re, k), gen.to_canonical(w.x_im, k)) for k in range(o, o + n)]
        ys = [(gen.to_canonical(w.y_re, k), gen.to_canonical(w.y_im, k)) for k in range(o, o + n)]
        wre, wim = oracle.cdot(xs, ys, int(w.precs[i]))
        for (ops, st), want in zip(host, (wre, wim)):
            e = compare_entry(gen.to_canonical(ops, i), want, int(st[i]))
            assert e is None, (i, n, int(w.precs[i]), e)
    b.close()


def test_batch_long_dots_that_cancel(ctx):
    # long dots of 2n + 1 terms whose first 2n cancel exactly: the first
    # window level cannot decide, so the wave refines over all terms; the
    # results are exact
    r = random.Random(41)
    # ~1100-bit operands at p ~ 1000: the widest shape
    outs = arbgpu.DeviceOut.empty(4, 1100)
    jobs, want, keep = [], [], []
    for k, (n, p) in enumerate([(1600, 1000), (700, 1100), (3000, 960), (1200, 1000)]):
        xs, ys = [], []
        for _ in range(n):
            xs.append(((r.randrange(2), r.getrandbits(1100) | 1 | (1 << 1099), r.randrange(-10, 11)), None))
            ys.append(((r.randrange(2), r.getrandbits(1000) | 1 | (1 << 999), r.randrange(-10, 11)), None))
        tiny = ((k % 2, 1, -400 - k), None)
        one = ((0, 1, 1), None)
        X = xs + xs + [tiny]
        Y = ys + [((1 - s, M, e), rad) for (s, M, e), rad in ys] + [one]
        dX = arbgpu.DeviceArray.from_host(gen.from_canonical(X))
        dY = arbgpu.DeviceArray.from_host(gen.from_canonical(Y))
        keep += [dX, dY]
        jobs.append(arbgpu.dot_job([outs.out()], k, [dX.arr()], 0, 1, [dY.arr()], 0, 1, 2 * n + 1, p))
        want.append(oracle.dot(X, Y, p))
    say("batch long dots that cancel")
    b = arbgpu.Batch(ctx, jobs)
    b.launch()
    _sync()
    host, st = outs.to_host()
    for k, w in enumerate(want):
        assert compare_entry(gen.to_canonical(host, k), w, int(st[k])) is None, k
        m, rad = gen.to_canonical(host, k)
        assert m[1] == 1 and rad is None   # exactly the tiny term, zero radius
    b.close()


def test_mixed_batch_of_dots_and_small_matmuls(ctx):
    # one graph launch: 120 dot jobs and 60 small complex ball matrix
    # products of uneven size and precision (tiles of 64 entries of a row
    # on the limb kernel, queued with the dots of their kernel shape)
    import torch
    specs, inits = random_jobs(4, 120)
    outs = [arbgpu.DeviceOut.empty(len(specs), 1100), arbgpu.DeviceOut.empty(len(specs), 1100)]
    jobs = [arbgpu.dot_request(j) for j in make_jobs(specs, inits, outs)]
    r = random.Random(5)
    rng = gen.rng_for(44, 0)
    mms = []
    for k in range(60):
        M, N, K = r.randint(1, 40), r.randint(1, 70), r.randint(1, 90)
        p = r.choice([30, 64, 128, 256, 400])
        host = [gen.random_operands(rng, c, rng.integers(1, p + 20, c), -10, 10, radius_shift=p, zero_frac=0.05)
                for c in (M * N, M * N, N * K, N * K)]
        dev = [arbgpu.DeviceArray.from_host(h) for h in host]
        C = [arbgpu.DeviceOut.empty(M * K, p), arbgpu.DeviceOut.empty(M * K, p)]
        Cr = [arbgpu.DeviceOut.empty(M * K, p), arbgpu.DeviceOut.empty(M * K, p)]
        am = arbgpu.Mat(dev[0].arr(), dev[1].arr(), M, N, 0, N, 1)
        bm = arbgpu.Mat(dev[2].arr(), dev[3].arr(), N, K, 0, K, 1)
        cm = arbgpu.OMat(C[0].out(), C[1].out(), M, K, 0, K, 1)
        crm = arbgpu.OMat(Cr[0].out(), Cr[1].out(), M, K, 0, K, 1)
        ctx.mat_mul_raw(crm, am, bm, p, arbgpu.COMPLEX | arbgpu.ALGO_LIMB)
        jobs.append(arbgpu.matmul_job(cm, am, bm, p, arbgpu.COMPLEX))
        mms.append((M, N, K, p, host, dev, C, Cr))
    r.shuffle(jobs)
    say(f"mixed batch: {len(jobs)} jobs")
    b = arbgpu.Batch(ctx, jobs, mixed=True)
    info = b.info()
    ntiles = sum(2 * M * ((K + 63) // 64) for (M, N, K, *_) in mms)
    assert info["tasks"] == sum(2 if s["cplx"] else 1 for s in specs) + ntiles
    b.tune()
    b.launch()
    _sync()
    check_jobs(specs, inits, [o.to_host() for o in outs])
    for (M, N, K, p, host, dev, C, Cr) in mms:
        got = [c.to_host() for c in C]
        ref = [c.to_host() for c in Cr]
        for (a, sa), (c, sc) in zip(got, ref):
            assert np.array_equal(a.limbs, c.limbs) and np.array_equal(a.exp, c.exp)
            assert np.array_equal(a.nls, c.nls) and np.array_equal(sa, sc)
            assert np.array_equal(a.rad_m, c.rad_m) and np.array_equal(a.rad_e, c.rad_e)
    # and sampled entries of a few products against the oracle
    for (M, N, K, p, host, dev, C, Cr) in mms[:8]:
        (o_re, s_re), (o_im, s_im) = C[0].to_host(), C[1].to_host()
        i, j = r.randrange(M), r.randrange(K)
        x = [(gen.to_canonical(host[0], i * N + k), gen.to_canonical(host[1], i * N + k)) for k in range(N)]
        y = [(gen.to_canonical(host[2], k * K + j), gen.to_canonical(host[3], k * K + j)) for k in range(N)]
        wre, wim = oracle.cdot(x, y, p)
        assert compare_entry(gen.to_canonical(o_re, i * K + j), wre, int(s_re[i * K + j])) is None
        assert compare_entry(gen.to_canonical(o_im, i * K + j), wim, int(s_im[i * K + j])) is None
    b.close()
