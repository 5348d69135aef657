"""The allocation-free matrix product (arbgpu_mat_mul_noalloc) through the
C-ABI: two calls in a row, the second on a smaller product, each
bit-identical to arbgpu_mat_mul on the same operands; no device allocation
by the context; products above its fixed scratch are refused."""

import numpy as np
import pytest

from paper_1901_04289_amd import arbgpu, gen

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def problem(seed, M, N, K, p, prec, cplx, rshift):
    rng = gen.rng_for(60, seed)
    n = 2 if cplx else 1
    A = [arbgpu.DeviceArray.from_host(gen.random_operands(rng, M * N, rng.integers(1, prec + 1, M * N), -8, 8,
                                                          radius_shift=rshift, zero_frac=0.05)) for _ in range(n)]
    B = [arbgpu.DeviceArray.from_host(gen.random_operands(rng, N * K, rng.integers(1, prec + 1, N * K), -8, 8,
                                                          radius_shift=rshift, zero_frac=0.05)) for _ in range(n)]
    am = arbgpu.Mat(A[0].arr(), A[-1].arr(), M, N, 0, N, 1)
    bm = arbgpu.Mat(B[0].arr(), B[-1].arr(), N, K, 0, K, 1)
    return A, B, am, bm


def outputs(M, K, p, n):
    C = [arbgpu.DeviceOut.empty(M * K, p) for _ in range(n)]
    return C, arbgpu.OMat(C[0].out(), C[-1].out(), M, K, 0, K, 1)


def host(C):
    return [c.to_host() for c in C]


def same(r1, r2):
    for (a, sa), (b, sb) in zip(r1, r2):
        assert np.array_equal(a.limbs, b.limbs) and np.array_equal(a.exp, b.exp)
        assert np.array_equal(a.nls, b.nls) and np.array_equal(sa, sb)
        assert np.array_equal(a.rad_m, b.rad_m) and np.array_equal(a.rad_e, b.rad_e)


@pytest.mark.parametrize("flags", [0, arbgpu.ALGO_SLICED])
def test_noalloc_equals_mat_mul_on_two_calls(flags):
    import torch
    ctx = arbgpu.Context(0)
    ref = arbgpu.Context(0)
    cases = [(1, 300, 160, 270, 256, 256, True, 250),     # complex, several tiles, ragged
             (2, 40, 33, 50, 128, 140, False, 120)]       # smaller, real
    a0 = ctx.alloc_count()
    for seed, M, N, K, p, prec, cplx, rshift in cases:
        say(f"noalloc seed={seed} {M}x{N}x{K} p={p} complex={cplx} flags={flags:#x}")
        A, B, am, bm = problem(seed, M, N, K, p, prec, cplx, rshift)
        f = flags | (arbgpu.COMPLEX if cplx else 0)
        C1, cm1 = outputs(M, K, p, 2 if cplx else 1)
        C2, cm2 = outputs(M, K, p, 2 if cplx else 1)
        ctx.mat_mul_noalloc_raw(cm1, am, bm, p, f)
        ref.mat_mul_raw(cm2, am, bm, p, f)
        torch.cuda.synchronize()
        same(host(C1), host(C2))
    assert ctx.alloc_count() == a0 == 0
    ctx.close()
    ref.close()


def test_noalloc_refuses_products_above_its_scratch():
    ctx = arbgpu.Context(0)
    M = N = K = 1024
    p = 2048
    A, B, am, bm = problem(3, 4, 4, 4, p, p, True, None)
    # only the shapes and caps decide: a 1024^3 complex product at p = 2048
    # may take several GiB
    big_a = arbgpu.Mat(A[0].arr(), A[1].arr(), M, N, 0, 0, 0)
    big_b = arbgpu.Mat(B[0].arr(), B[1].arr(), N, K, 0, 0, 0)
    C, cm = outputs(1, 1, p, 2)
    cm.rows, cm.cols, cm.rs, cm.cs = M, K, 0, 0
    rc = ctx.mat_mul_noalloc_raw(cm, big_a, big_b, p, arbgpu.COMPLEX, check=False)
    assert rc == arbgpu.EINVAL and "scratch" in ctx.last_error()
    ctx.close()
