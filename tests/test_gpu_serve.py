"""GPU tests of the request loop: each result is the same alone and in a
mix of overlapping requests, results match the oracle, admission by HBM
footprint, and ticket times, through the C-ABI."""

import random

import numpy as np
import pytest

import oracle
from paper_1901_04289_amd import arbgpu, gen
from tests.arbcheck import compare_entry

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    say("importing torch")
    import torch
    assert torch.cuda.is_available()
    c = arbgpu.Context(0)
    say("context ready")
    yield c
    c.close()


def _sync():
    import torch
    torch.cuda.synchronize()


class Request:
    """A complex ball matrix product n x n at precision p with resident
    operands and two output sets (alone, in the mix)."""

    def __init__(self, seed, n, p):
        rng = gen.rng_for(4, 100 + seed)
        self.n, self.p = n, p
        self.host = gen.config4_operands(rng, n, p)
        self.dev = [arbgpu.DeviceArray.from_host(o) for o in self.host]
        self.alone = [arbgpu.DeviceOut.empty(n * n, p), arbgpu.DeviceOut.empty(n * n, p)]
        self.mix = [arbgpu.DeviceOut.empty(n * n, p), arbgpu.DeviceOut.empty(n * n, p)]

    def mats(self, outs):
        n = self.n
        A = arbgpu.Mat(self.dev[0].arr(), self.dev[1].arr(), n, n, 0, n, 1)
        B = arbgpu.Mat(self.dev[2].arr(), self.dev[3].arr(), n, n, 0, n, 1)
        C = arbgpu.OMat(outs[0].out(), outs[1].out(), n, n, 0, n, 1)
        return C, A, B

    def job(self):
        C, A, B = self.mats(self.mix)
        return arbgpu.matmul_job(C, A, B, self.p, arbgpu.COMPLEX)

    def run_alone(self, ctx):
        C, A, B = self.mats(self.alone)
        ctx.mat_mul_raw(C, A, B, self.p, arbgpu.COMPLEX)


class DotRequest:
    def __init__(self, seed, n, p):
        rng = gen.rng_for(4, 200 + seed)
        self.n, self.p = n, p
        prec = rng.integers((p + 1) // 2, 2 * p + 1, n)
        self.host = [gen.random_operands(rng, n, prec, -16, 16, radius_shift=prec) for _ in range(4)]
        self.dev = [arbgpu.DeviceArray.from_host(o) for o in self.host]
        self.alone = [arbgpu.DeviceOut.empty(1, p), arbgpu.DeviceOut.empty(1, p)]
        self.mix = [arbgpu.DeviceOut.empty(1, p), arbgpu.DeviceOut.empty(1, p)]

    def dotjob(self, outs):
        return arbgpu.dot_job([outs[0].out(), outs[1].out()], 0, [self.dev[0].arr(), self.dev[1].arr()], 0, 1,
                              [self.dev[2].arr(), self.dev[3].arr()], 0, 1, self.n, self.p, arbgpu.COMPLEX)

    def job(self):
        return arbgpu.dot_request(self.dotjob(self.mix))

    def run_alone(self, ctx):
        j = self.dotjob(self.alone)
        ctx.dot_raw([j.res[0], j.res[1]], 0, None, 0, False, [j.x[0], j.x[1]], 0, 1, [j.y[0], j.y[1]], 0, 1,
                    self.n, self.p, arbgpu.COMPLEX)


def same(outs_a, outs_b):
    for a, b in zip(outs_a, outs_b):
        (x, sx), (y, sy) = a.to_host(), b.to_host()
        if not (np.array_equal(x.limbs, y.limbs) and np.array_equal(x.exp, y.exp) and np.array_equal(x.nls, y.nls)
                and np.array_equal(x.rad_m, y.rad_m) and np.array_equal(x.rad_e, y.rad_e)
                and np.array_equal(sx, sy)):
            return False
    return True


def test_results_same_alone_and_in_the_mix(ctx):
    r = random.Random(1)
    reqs = []
    shapes = [(16, 2048), (33, 128), (100, 512), (257, 256), (64, 1024), (200, 2048), (16, 128), (120, 1024),
              (45, 512), (300, 128)]
    for k, (n, p) in enumerate(shapes):
        reqs.append(Request(k, n, p))
    for k in range(24):
        reqs.append(DotRequest(k, r.choice([4, 50, 300, 1000]), r.choice([64, 128, 300, 700, 1024])))
    r.shuffle(reqs)
    say(f"{len(reqs)} requests: running each alone")
    for q in reqs:
        q.run_alone(ctx)
        _sync()
    say("submitting the mix")
    ctx.serve_config(slots=4)
    tickets = []
    for k in range(0, len(reqs), 5):   # arrivals in small groups
        tickets += ctx.submit([q.job() for q in reqs[k:k + 5]])
    for t in tickets:
        ctx.wait(t)
    say("mix done; comparing")
    for q in reqs:
        assert same(q.alone, q.mix), (type(q).__name__, q.n, q.p)
    # times are ordered for every ticket
    for t in tickets:
        s, b, e = ctx.ticket_times(t)
        assert 0 < s <= b <= e
    # the mix overlapped: some request started before another one ended
    spans = sorted(ctx.ticket_times(t)[1:] for t in tickets)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))


def test_request_results_match_oracle(ctx):
    ctx.serve_config(slots=2)
    reqs = [Request(50, 16, 2048), Request(51, 40, 256)]
    t = ctx.submit([q.job() for q in reqs])
    for x in t:
        ctx.wait(x)
    for q in reqs:
        n, p = q.n, q.p
        A = [[(gen.to_canonical(q.host[0], i * n + k), gen.to_canonical(q.host[1], i * n + k)) for k in range(n)]
             for i in range(n)]
        B = [[(gen.to_canonical(q.host[2], k * n + j), gen.to_canonical(q.host[3], k * n + j)) for j in range(n)]
             for k in range(n)]
        (o_re, s_re), (o_im, s_im) = q.mix[0].to_host(), q.mix[1].to_host()
        rr = random.Random(n)
        for _ in range(12):
            i, j = rr.randrange(n), rr.randrange(n)
            wre, wim = oracle.cdot(A[i], [B[k][j] for k in range(n)], p)
            assert compare_entry(gen.to_canonical(o_re, i * n + j), wre, int(s_re[i * n + j])) is None
            assert compare_entry(gen.to_canonical(o_im, i * n + j), wim, int(s_im[i * n + j])) is None


def test_admission_by_footprint(ctx):
    big = Request(60, 512, 1024)
    other = Request(61, 512, 1024)
    ctx.serve_config(slots=2, budget=1 << 20)
    rc, _ = ctx.submit([big.job()], check=False)
    assert rc == arbgpu.ENOMEM
    say("admission: measuring the footprint")
    one = None
    # one slot: it holds the whole budget, so a job is admitted alone once
    # its footprint fits the budget
    for mib in (256, 512, 1024, 2048, 4096, 8192, 16384):
        ctx.serve_config(slots=1, budget=mib << 20)
        rc, t = ctx.submit([big.job()], check=False)
        if rc == arbgpu.OK:
            one = mib
            ctx.wait(t[0])
            break
    assert one is not None
    # the footprint lies in (one/2, one] MiB: a budget of `one` holds one
    # of these products but not two
    ctx.serve_config(slots=1, budget=one << 20)
    t1 = ctx.submit([big.job()])
    rc, t2 = ctx.submit([other.job()], check=False)
    if rc == arbgpu.OK:
        # only possible when the first product had already finished
        assert ctx.poll(t1[0]) == arbgpu.OK
        ctx.wait(t2[0])
    else:
        assert rc == arbgpu.EAGAIN
        ctx.wait(t1[0])
        t2 = ctx.submit([other.job()])
        ctx.wait(t2[0])
    big.run_alone(ctx)
    other.run_alone(ctx)
    _sync()
    assert same(big.alone, big.mix) and same(other.alone, other.mix)
    ctx.serve_config(slots=4)
