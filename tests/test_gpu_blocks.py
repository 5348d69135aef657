"""GPU parity of Algorithm 2's block partition and of the multi-block
matrix product (exact per-block integer products, basecase chunks, one
rounding per entry) against the exact oracle, through the C-ABI."""

import random

import numpy as np
import pytest

import oracle
from paper_1901_04289_amd import arbgpu, gen
from tests.arbcheck import compare_entry
from tests.test_oracle_blocks import TABLE3, _pascal

pytestmark = pytest.mark.gpu

KIND = {"block": 0, "basecase": 1}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = arbgpu.Context(0)
    yield c
    c.close()


def say(msg):
    print(msg, flush=True)


def grade(ops, rows, cols, shift, along_cols):
    """Scale entry (r, c) by 2^shift[c] (along_cols) or 2^shift[r]."""
    e = ops.exp.reshape(rows, cols)
    s = np.asarray(shift, dtype=np.int64)
    e += (s[None, :] if along_cols else s[:, None]).astype(np.int32)
    return ops


class Res:
    """Host copy of one output part: limb planes plus per-entry status."""

    def __init__(self, ops, status):
        self.ops, self.status = ops, status
        self.limbs, self.exp, self.nls = ops.limbs, ops.exp, ops.nls
        self.rad_m, self.rad_e = ops.rad_m, ops.rad_e


def run(ctx, A, B, M, N, K, p, flags, Ai=None, Bi=None):
    import torch
    dA, dB = arbgpu.DeviceArray.from_host(A), arbgpu.DeviceArray.from_host(B)
    dAi = arbgpu.DeviceArray.from_host(Ai) if Ai is not None else None
    dBi = arbgpu.DeviceArray.from_host(Bi) if Bi is not None else None
    rad = not (flags & arbgpu.APPROX)
    C = arbgpu.DeviceOut.empty(M * K, p, radius=rad)
    Ci = arbgpu.DeviceOut.empty(M * K, p, radius=rad) if flags & arbgpu.COMPLEX else None
    ctx.timing(True)
    ctx.mat_mul(C, dA, dB, M, N, K, p, flags, Ci=Ci, Ai=dAi, Bi=dBi)
    torch.cuda.synchronize()
    merges = ctx.timing_read("merge")[1]
    ctx.timing(False)
    return Res(*C.to_host()), (Res(*Ci.to_host()) if Ci is not None else None), merges


def plan(ctx, A, B, M, N, K, p, flags=0, Ai=None, Bi=None):
    dA, dB = arbgpu.DeviceArray.from_host(A), arbgpu.DeviceArray.from_host(B)
    dAi = arbgpu.DeviceArray.from_host(Ai) if Ai is not None else None
    dBi = arbgpu.DeviceArray.from_host(Bi) if Bi is not None else None
    return ctx.plan_blocks(dA, dB, M, N, K, p, flags, Ai=dAi, Bi=dBi)


def oracle_plan(Ac, Bc, p):
    mids = lambda X: [[x[0] for x in r] for r in X]
    return [(a, b, KIND[k]) for a, b, k in oracle.extract_blocks(mids(Ac), mids(Bc), p)]


def mixed_grading(n):
    """Exponent offsets per inner index: gentle, then steep (basecase
    chunks), then gentle again."""
    g, out = 0, []
    for k in range(n):
        out.append(g)
        g += 3 if k < 80 else (45 if k < 130 else 2)
    return out


@pytest.mark.parametrize("n", [100, 300])
def test_plan_pascal_table3(ctx, n):
    for p in (53, 106, 212, 848, 3392):
        A = _pascal(n, p)
        ops = gen.from_canonical([(x, None) for row in A for x in row])
        say(f"plan pascal n={n} p={p}")
        got = plan(ctx, ops, ops, n, n, n, p)
        assert len(got) == TABLE3[(n, p)], (n, p, got)
        want = [(a, b, KIND[k]) for a, b, k in oracle.extract_blocks(A, A, p)]
        assert got == want, (n, p)


@pytest.mark.parametrize("seed,M,N,K,p,prec", [
    (1, 19, 330, 23, 100, 100),
    (2, 3, 500, 1, 64, 60),
    (3, 40, 95, 40, 200, 220),
])
def test_plan_graded_matches_oracle(ctx, seed, M, N, K, p, prec):
    rng = gen.rng_for(30, seed)
    A = gen.random_operands(rng, M * N, rng.integers(1, prec + 1, M * N), -4, 4, zero_frac=0.1)
    B = gen.random_operands(rng, N * K, rng.integers(1, prec + 1, N * K), -4, 4, zero_frac=0.1)
    g = mixed_grading(N)
    grade(A, M, N, g, True)
    grade(B, N, K, [-x for x in g], False)
    say(f"plan graded seed={seed} {M}x{N}x{K} p={p}")
    got = plan(ctx, A, B, M, N, K, p)
    want = oracle_plan(gen.canonical_matrix(A, M, N, N, 1), gen.canonical_matrix(B, N, K, K, 1), p)
    assert got == want
    assert any(k == 0 for _, _, k in got) and len(got) > 1


def test_plan_empty_and_flat(ctx):
    rng = gen.rng_for(31, 0)
    A = gen.random_operands(rng, 4 * 50, 64, -3, 3)
    B = gen.random_operands(rng, 50 * 3, 64, -3, 3)
    assert plan(ctx, A, B, 4, 50, 3, 64) == [(0, 50, 0)]
    # a short inner range is one basecase chunk
    A2 = gen.random_operands(rng, 4 * 7, 64, -3, 3)
    B2 = gen.random_operands(rng, 7 * 3, 64, -3, 3)
    assert plan(ctx, A2, B2, 4, 7, 3, 64) == [(0, 7, 1)]


def test_multiblock_pascal_matches_oracle_and_limb(ctx):
    n, p = 300, 212
    A = _pascal(n, p)
    ops = gen.from_canonical([(x, None) for row in A for x in row])
    say("multi-block pascal n=300 p=212")
    # the residue form on every block (forced), then the automatic choice,
    # which may give some blocks' terms to the merge instead
    out, _, merges = run(ctx, ops, ops, n, n, n, p, arbgpu.ALGO_RNS)
    assert merges == 1
    auto, _, _ = run(ctx, ops, ops, n, n, n, p, 0)
    assert np.array_equal(out.limbs, auto.limbs) and np.array_equal(out.nls, auto.nls)
    assert np.array_equal(out.exp, auto.exp)
    ref, _, m2 = run(ctx, ops, ops, n, n, n, p, arbgpu.ALGO_LIMB)
    assert m2 == 0
    assert np.array_equal(out.limbs, ref.limbs)
    assert np.array_equal(out.exp, ref.exp) and np.array_equal(out.nls, ref.nls)
    assert np.array_equal(out.rad_m, ref.rad_m) and np.array_equal(out.rad_e, ref.rad_e)
    r = random.Random(5)
    ent = [(r.randrange(n), r.randrange(n)) for _ in range(40)] + [(0, 0), (n - 1, n - 1)]
    col = lambda j: [A[k][j] for k in range(n)]
    for i, j in ent:
        want = oracle.dot([(x, None) for x in A[i]], [(x, None) for x in col(j)], p)
        assert compare_entry(gen.to_canonical(out.ops, i * n + j), want, int(out.status[i * n + j])) is None, (i, j)


@pytest.mark.parametrize("algo", [0, arbgpu.ALGO_SLICED, arbgpu.ALGO_RNS])
@pytest.mark.parametrize("seed,M,N,K,p,prec,rshift,approx", [
    (1, 19, 330, 23, 100, 100, 95, False),   # blocks, basecase chunks, balls, zeros
    (2, 33, 260, 2, 150, 180, None, False),  # wide operands, exact
    (3, 5, 200, 70, 90, 100, 80, True),      # midpoints only
])
def test_multiblock_real_parity(ctx, seed, M, N, K, p, prec, rshift, approx, algo):
    rng = gen.rng_for(32, seed)
    A = gen.random_operands(rng, M * N, rng.integers(1, prec + 1, M * N), -4, 4, radius_shift=rshift,
                            zero_frac=0.1)
    B = gen.random_operands(rng, N * K, rng.integers(1, prec + 1, N * K), -4, 4, radius_shift=rshift,
                            zero_frac=0.1)
    g = mixed_grading(N)
    grade(A, M, N, g, True)
    grade(B, N, K, [-x for x in g], False)
    flags = (arbgpu.APPROX if approx else 0) | algo
    say(f"multi-block real seed={seed} {M}x{N}x{K} p={p} algo={algo:#x}")
    out, _, merges = run(ctx, A, B, M, N, K, p, flags)
    # forced INT8 forms take every block; the automatic choice may give
    # blocks (or the whole product) to the window engine
    assert merges == 1 or (algo == 0 and merges == 0)
    Ac = gen.canonical_matrix(A, M, N, N, 1)
    Bc = gen.canonical_matrix(B, N, K, K, 1)
    cols = [[Bc[k][j] for k in range(N)] for j in range(K)]
    for i in range(M):
        for j in range(K):
            want = oracle.dot(Ac[i], cols[j], p, approx=approx)
            e = compare_entry(gen.to_canonical(out.ops, i * K + j), want, int(out.status[i * K + j]), approx)
            assert e is None, ((i, j), e)


@pytest.mark.parametrize("algo", [arbgpu.ALGO_SLICED, arbgpu.ALGO_RNS])
def test_multiblock_complex_parity(ctx, algo):
    rng = gen.rng_for(33, 0)
    M, N, K, p = 7, 170, 9, 120
    parts = [gen.random_operands(rng, c, 130, -6, 6, radius_shift=125, zero_frac=0.05)
             for c in (M * N, M * N, N * K, N * K)]
    g = [4 * k if k < 90 else 360 + 40 * (k - 90) for k in range(N)]
    grade(parts[0], M, N, g, True)
    grade(parts[1], M, N, g, True)
    grade(parts[2], N, K, [-x for x in g], False)
    grade(parts[3], N, K, [-x for x in g], False)
    say("multi-block complex")
    out, outi, merges = run(ctx, parts[0], parts[2], M, N, K, p, arbgpu.COMPLEX | algo, Ai=parts[1], Bi=parts[3])
    assert merges == 2
    A = [[(gen.to_canonical(parts[0], i * N + k), gen.to_canonical(parts[1], i * N + k)) for k in range(N)]
         for i in range(M)]
    B = [[(gen.to_canonical(parts[2], k * K + j), gen.to_canonical(parts[3], k * K + j)) for j in range(K)]
         for k in range(N)]
    C = oracle.cmat_mul(A, B, p)
    for i in range(M):
        for j in range(K):
            re, im = C[i][j]
            assert compare_entry(gen.to_canonical(out.ops, i * K + j), re, int(out.status[i * K + j])) is None
            assert compare_entry(gen.to_canonical(outi.ops, i * K + j), im, int(outi.status[i * K + j])) is None
