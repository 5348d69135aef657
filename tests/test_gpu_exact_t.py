"""GPU parity of the exact integer block product T of Algorithm 2 (Section
4.1), read through arbgpu_mat_mul_exact_t, against the oracle's integer
product, and of the three-product complex form (eq. (2), Section 3.6)
against the four-product form and the oracle."""

import random

import numpy as np
import pytest

import oracle
from paper_1901_04289_amd import arbgpu, gen
from tests.arbcheck import compare_entry

pytestmark = pytest.mark.gpu

ALGOS = [arbgpu.ALGO_SLICED, arbgpu.ALGO_RNS]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = arbgpu.Context(0)
    yield c
    c.close()


def say(msg):
    print(msg, flush=True)


def mids(ops, rows, cols, neg=False):
    m = gen.canonical_matrix(ops, rows, cols, cols, 1)
    return [[oracle.fneg(x[0]) if neg else x[0] for x in r] for r in m]


def decode_t(T, cap, count):
    """Two's-complement integers from int32 limb planes [cap, ld]."""
    a = T.cpu().numpy().view(np.uint32)
    out = []
    for ij in range(count):
        v = 0
        for k in range(cap - 1, -1, -1):
            v = (v << 32) | int(a[k, ij])
        if v >> (32 * cap - 1):
            v -= 1 << (32 * cap)
        out.append(v)
    return out


def exact_t(ctx, parts, M, N, K, flags, cap):
    import torch
    dev = [arbgpu.DeviceArray.from_host(x) for x in parts]
    cplx = bool(flags & arbgpu.COMPLEX)
    am = arbgpu.Mat(dev[0].arr(), dev[1 if cplx else 0].arr(), M, N, 0, N, 1)
    bm = arbgpu.Mat(dev[2 if cplx else 1].arr(), dev[3 if cplx else 1].arr(), N, K, 0, K, 1)
    Tre = torch.zeros((cap, M * K), dtype=torch.int32, device="cuda")
    Tim = torch.zeros((cap, M * K), dtype=torch.int32, device="cuda") if cplx else None
    rv = torch.full((M,), -7, dtype=torch.int32, device="cuda")
    cv = torch.full((K,), -7, dtype=torch.int32, device="cuda")
    ctx.mat_mul_exact_t_raw(Tre, Tim, M * K, cap, rv, cv, am, bm, flags)
    torch.cuda.synchronize()
    ts = [decode_t(Tre, cap, M * K)] + ([decode_t(Tim, cap, M * K)] if cplx else [])
    return ts, rv.cpu().numpy(), cv.cpu().numpy()


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("seed,M,N,K,prec,erange", [
    (1, 40, 90, 33, 200, 6),       # ragged, one tile
    (2, 300, 130, 257, 64, 3),     # several tiles, inner length not a multiple of 128
    (3, 5, 1, 7, 500, 40),         # inner length 1, wide operands
])
def test_exact_t_real(ctx, algo, seed, M, N, K, prec, erange):
    rng = gen.rng_for(40, seed)
    A = gen.random_operands(rng, M * N, rng.integers(1, prec + 1, M * N), -erange, erange, zero_frac=0.1)
    B = gen.random_operands(rng, N * K, rng.integers(1, prec + 1, N * K), -erange, erange, zero_frac=0.1)
    if M > 2:
        A.limbs[:, N:2 * N] = 0       # an all-zero row
        A.nls[N:2 * N] = 0
        A.exp[N:2 * N] = 0
    say(f"exact T real seed={seed} {M}x{N}x{K} algo={algo:#x}")
    cap = 2 * ((prec + 2 * erange + 64) // 32 + 4)
    (T,), rv, cv = exact_t(ctx, [A, B], M, N, K, algo, cap)
    e, f, Tw = oracle.block_product(mids(A, M, N), mids(B, N, K), list(range(N)))
    assert list(rv) == [-x for x in e]
    assert list(cv) == [-x for x in f]
    for i in range(M):
        for j in range(K):
            assert T[i * K + j] == Tw[i][j], (i, j)


@pytest.mark.parametrize("algo,four", [(arbgpu.ALGO_SLICED, False), (arbgpu.ALGO_RNS, False),
                                       (arbgpu.ALGO_RNS, True)])
def test_exact_t_complex(ctx, algo, four):
    # T_re = [A_re A_im] [B_re; -B_im] and T_im = [A_re A_im] [B_im; B_re]
    # with one scaling per row over both parts (and per column)
    rng = gen.rng_for(41, int(four))
    M, N, K = 33, 70, 20
    parts = [gen.random_operands(rng, c, rng.integers(1, 150, c), -9, 9, zero_frac=0.1)
             for c in (M * N, M * N, N * K, N * K)]
    flags = arbgpu.COMPLEX | algo | (arbgpu.COMPLEX_4M if four else 0)
    say(f"exact T complex algo={algo:#x} four={four}")
    (Tr, Ti), rv, cv = exact_t(ctx, parts, M, N, K, flags, 14)
    Ar, Ai = mids(parts[0], M, N), mids(parts[1], M, N)
    Br, Bi, nBi = mids(parts[2], N, K), mids(parts[3], N, K), mids(parts[3], N, K, neg=True)
    Acat = [Ar[i] + Ai[i] for i in range(M)]
    e, f, Twr = oracle.block_product(Acat, Br + nBi, list(range(2 * N)))
    e2, f2, Twi = oracle.block_product(Acat, Bi + Br, list(range(2 * N)))
    assert e == e2 and f == f2
    assert list(rv) == [-x for x in e] and list(cv) == [-x for x in f]
    for i in range(M):
        for j in range(K):
            assert Tr[i * K + j] == Twr[i][j], ("re", i, j)
            assert Ti[i * K + j] == Twi[i][j], ("im", i, j)


def test_exact_t_rejects_short_cap(ctx):
    import torch
    rng = gen.rng_for(42, 0)
    M, N, K = 4, 8, 4
    A = gen.random_operands(rng, M * N, 300, -3, 3)
    B = gen.random_operands(rng, N * K, 300, -3, 3)
    dA, dB = arbgpu.DeviceArray.from_host(A), arbgpu.DeviceArray.from_host(B)
    am = arbgpu.Mat(dA.arr(), dA.arr(), M, N, 0, N, 1)
    bm = arbgpu.Mat(dB.arr(), dB.arr(), N, K, 0, K, 1)
    T = torch.zeros((2, M * K), dtype=torch.int32, device="cuda")
    rv = torch.zeros(M, dtype=torch.int32, device="cuda")
    cv = torch.zeros(K, dtype=torch.int32, device="cuda")
    rc = ctx.mat_mul_exact_t_raw(T, None, M * K, 2, rv, cv, am, bm, arbgpu.ALGO_RNS, check=False)
    assert rc == arbgpu.EINVAL and "limbs" in ctx.last_error()


@pytest.mark.parametrize("seed,M,N,K,p,prec,rshift", [
    (1, 300, 200, 270, 256, 256, 250),     # several tiles, ragged edges, balls
    (2, 9, 3, 11, 700, 800, None),         # short inner length, wide operands
])
def test_complex_three_products_equal_four(ctx, seed, M, N, K, p, prec, rshift):
    import torch
    rng = gen.rng_for(43, seed)
    parts = [gen.random_operands(rng, c, rng.integers(1, prec + 1, c), -8, 8, radius_shift=rshift,
                                 zero_frac=0.05) for c in (M * N, M * N, N * K, N * K)]
    dev = [arbgpu.DeviceArray.from_host(x) for x in parts]
    outs = []
    for four in (False, True):
        C, Ci = arbgpu.DeviceOut.empty(M * K, p), arbgpu.DeviceOut.empty(M * K, p)
        flags = arbgpu.COMPLEX | arbgpu.ALGO_RNS | (arbgpu.COMPLEX_4M if four else 0)
        say(f"complex 3M vs 4M seed={seed} four={four}")
        ctx.mat_mul(C, dev[0], dev[2], M, N, K, p, flags, Ci=Ci, Ai=dev[1], Bi=dev[3])
        torch.cuda.synchronize()
        outs.append((C.to_host(), Ci.to_host()))
    for part in range(2):
        (a, sa), (b, sb) = outs[0][part], outs[1][part]
        assert np.array_equal(a.limbs, b.limbs) and np.array_equal(a.exp, b.exp)
        assert np.array_equal(a.nls, b.nls) and np.array_equal(sa, sb)
        if a.rad_m is not None:
            assert np.array_equal(a.rad_m, b.rad_m) and np.array_equal(a.rad_e, b.rad_e)
    (out, st), (outi, sti) = outs[0]
    r = random.Random(seed)
    ent = [(r.randrange(M), r.randrange(K)) for _ in range(12)] + [(0, 0), (M - 1, K - 1)]
    for i, j in ent:
        x = [(gen.to_canonical(parts[0], i * N + k), gen.to_canonical(parts[1], i * N + k)) for k in range(N)]
        y = [(gen.to_canonical(parts[2], k * K + j), gen.to_canonical(parts[3], k * K + j)) for k in range(N)]
        re, im = oracle.cdot(x, y, p)
        assert compare_entry(gen.to_canonical(out, i * K + j), re, int(st[i * K + j])) is None
        assert compare_entry(gen.to_canonical(outi, i * K + j), im, int(sti[i * K + j])) is None
