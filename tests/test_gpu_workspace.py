"""Workspace of the C-ABI on the GPU: products on reserved workspace
allocate no device memory, the admission footprint bounds what a product
takes, and serving slots reserved for the largest request allocate nothing
while they serve a mixed stream (results identical to direct calls)."""

import numpy as np
import pytest

from paper_1901_04289_amd import arbgpu, gen

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


class Problem:
    """Row-major device operands and outputs of one matrix product."""

    def __init__(self, seed, M, N, K, p, prec, cplx=False, rshift=None, flags=0):
        rng = gen.rng_for(50, seed)
        self.M, self.N, self.K, self.p, self.cplx = M, N, K, p, cplx
        self.flags = flags | (arbgpu.COMPLEX if cplx else 0)
        n = 2 if cplx else 1
        self.A = [arbgpu.DeviceArray.from_host(gen.random_operands(rng, M * N, prec, -8, 8, radius_shift=rshift,
                                                                   zero_frac=0.05)) for _ in range(n)]
        self.B = [arbgpu.DeviceArray.from_host(gen.random_operands(rng, N * K, prec, -8, 8, radius_shift=rshift,
                                                                   zero_frac=0.05)) for _ in range(n)]
        rad = not (self.flags & arbgpu.APPROX)
        self.C = [arbgpu.DeviceOut.empty(M * K, p, radius=rad) for _ in range(n)]

    def mats(self):
        a, b, c = self.A, self.B, self.C
        am = arbgpu.Mat(a[0].arr(), a[-1].arr(), self.M, self.N, 0, self.N, 1)
        bm = arbgpu.Mat(b[0].arr(), b[-1].arr(), self.N, self.K, 0, self.K, 1)
        cm = arbgpu.OMat(c[0].out(), c[-1].out(), self.M, self.K, 0, self.K, 1)
        return cm, am, bm

    def run(self, ctx):
        import torch
        cm, am, bm = self.mats()
        ctx.mat_mul_raw(cm, am, bm, self.p, self.flags)
        torch.cuda.synchronize()
        return [c.to_host() for c in self.C]

    def job(self):
        cm, am, bm = self.mats()
        return arbgpu.matmul_job(cm, am, bm, self.p, self.flags)


def same(r1, r2):
    for (a, sa), (b, sb) in zip(r1, r2):
        assert np.array_equal(a.limbs, b.limbs) and np.array_equal(a.exp, b.exp)
        assert np.array_equal(a.nls, b.nls) and np.array_equal(sa, sb)
        if a.rad_m is not None:
            assert np.array_equal(a.rad_m, b.rad_m) and np.array_equal(a.rad_e, b.rad_e)


def mixed_problems():
    return [
        Problem(1, 300, 200, 270, 256, 256, rshift=250),                    # automatic INT8 form, balls
        Problem(2, 300, 200, 270, 256, 256, rshift=250, flags=arbgpu.ALGO_SLICED),
        Problem(3, 130, 64, 100, 512, 512, cplx=True, rshift=500),          # complex, three products
        Problem(4, 64, 40, 64, 128, 128, flags=arbgpu.APPROX),
        Problem(5, 20, 10, 20, 100, 100, flags=arbgpu.ALGO_LIMB),
        Problem(6, 9, 33, 7, 2048, 2048, cplx=True, flags=arbgpu.ALGO_RNS),  # wide residues
    ]


def test_reserved_products_allocate_nothing():
    ctx = arbgpu.Context(0)
    probs = mixed_problems()
    for pr in probs:
        cm, am, bm = pr.mats()
        ctx.reserve_raw(am, bm, pr.p, pr.flags)
    a0, b0 = ctx.workspace_info()
    say(f"reserved: {a0} allocations, {b0} bytes")
    first = [pr.run(ctx) for pr in probs]
    for rep in range(2):
        for pr, want in zip(reversed(probs), reversed(first)):
            same(pr.run(ctx), want)
    assert ctx.workspace_info() == (a0, b0)
    ctx.close()


@pytest.mark.parametrize("n,p,cplx", [(16, 128, True), (100, 2048, True), (256, 256, False), (300, 1024, True),
                                      (64, 512, False)])
def test_footprint_bounds_the_workspace(n, p, cplx):
    # a fresh context holds only what the product itself took
    pr = Problem(10 + n + p, n, n, n, p, p, cplx=cplx, rshift=p)
    ctx = arbgpu.Context(0)
    cm, am, bm = pr.mats()
    fp = ctx.footprint_raw(am, bm, pr.p, pr.flags)
    ctx.timing(True)
    pr.run(ctx)
    int8 = ctx.timing_read("mfma")[1] > 0
    ctx.timing(False)
    allocs, held = ctx.workspace_info()
    say(f"n={n} p={p} complex={cplx}: footprint {fp}, held {held} in {allocs} buffers, int8 path {int8}")
    assert held <= fp
    if int8:   # the limb kernel needs no workspace
        assert held > 0
    ctx.close()


def test_reserved_serving_slots_allocate_nothing():
    import torch
    ctx = arbgpu.Context(0)
    ctx.serve_config(4)
    probs = [Problem(20 + k, n, n, n, p, p, cplx=True, rshift=p)
             for k, (n, p) in enumerate([(16, 128), (40, 512), (100, 256), (64, 1024), (128, 128), (33, 2048)])]
    ctx.serve_reserve([pr.job() for pr in probs])
    a0, b0 = ctx.workspace_info()
    want = [pr.run(arbgpu.Context(0)) for pr in probs]
    for rep in range(3):
        tickets = ctx.submit([pr.job() for pr in probs])
        for t in tickets:
            ctx.wait(t)
        torch.cuda.synchronize()
        for pr, w in zip(probs, want):
            same([c.to_host() for c in pr.C], w)
    assert ctx.workspace_info() == (a0, b0)
    ctx.close()
