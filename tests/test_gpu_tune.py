"""The matrix product's path autotuner and the paths it chooses between:
every path (limb kernel, base-256 slices, residues on 256 and on 128 MFMA
tiles) gives the same bits, forced through the tune-cache file, and the
tuner records a choice that later calls follow."""

import json
import random

import numpy as np
import pytest

import oracle
from paper_1901_04289_amd import arbgpu, gen
from tests.arbcheck import compare_entry

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def operands(seed, M, N, K, prec, cplx, rshift):
    rng = gen.rng_for(70, seed)
    n = 2 if cplx else 1
    hA = [gen.random_operands(rng, M * N, rng.integers(1, prec + 1, M * N), -8, 8, radius_shift=rshift,
                              zero_frac=0.05) for _ in range(n)]
    hB = [gen.random_operands(rng, N * K, rng.integers(1, prec + 1, N * K), -8, 8, radius_shift=rshift,
                              zero_frac=0.05) for _ in range(n)]
    return hA, hB, [arbgpu.DeviceArray.from_host(x) for x in hA], [arbgpu.DeviceArray.from_host(x) for x in hB]


def mats(A, B, C, M, N, K):
    return (arbgpu.OMat(C[0].out(), C[-1].out(), M, K, 0, K, 1),
            arbgpu.Mat(A[0].arr(), A[-1].arr(), M, N, 0, N, 1),
            arbgpu.Mat(B[0].arr(), B[-1].arr(), N, K, 0, K, 1))


def class_key(M, N, K, p, cplx, balls):
    lg = lambda v: max(0, (int(v) - 1).bit_length())
    return f"mat_mul:{'c' if cplx else 'r'}{'b' if balls else 'm'}:n{lg(max(M, K))}:k{lg(N)}:p{lg(p)}"


@pytest.mark.parametrize("seed,M,N,K,p,prec,cplx", [
    (1, 300, 200, 270, 256, 256, True),    # 128 tiles: 3 x 3 with ragged edges
    (2, 520, 64, 130, 512, 500, False),    # 256 tiles: 3 x 1
    (3, 129, 40, 127, 1024, 1024, True),   # one entry past a 128 tile
])
def test_every_path_gives_the_same_bits(tmp_path, seed, M, N, K, p, prec, cplx):
    import torch
    hA, hB, A, B = operands(seed, M, N, K, prec, cplx, prec - 4)
    key = class_key(M, N, K, p, cplx, True)
    outs = {}
    for choice in (arbgpu.CHOICE_LIMB, arbgpu.CHOICE_SLICES, arbgpu.CHOICE_RNS256, arbgpu.CHOICE_RNS128):
        path = tmp_path / f"tune{choice}.json"
        path.write_text(json.dumps({key: choice}))
        ctx = arbgpu.Context(0, tune_cache=str(path))
        C = [arbgpu.DeviceOut.empty(M * K, p) for _ in range(2 if cplx else 1)]
        cm, am, bm = mats(A, B, C, M, N, K)
        say(f"path {choice} seed={seed} {M}x{N}x{K} p={p} complex={cplx}")
        ctx.mat_mul_raw(cm, am, bm, p, arbgpu.COMPLEX if cplx else 0)
        torch.cuda.synchronize()
        outs[choice] = [c.to_host() for c in C]
        ctx.close()
    ref = outs[arbgpu.CHOICE_LIMB]
    for choice, res in outs.items():
        for (a, sa), (b, sb) in zip(res, ref):
            assert np.array_equal(a.limbs, b.limbs) and np.array_equal(a.exp, b.exp), choice
            assert np.array_equal(a.nls, b.nls) and np.array_equal(sa, sb), choice
    # and against the oracle on sampled entries
    r = random.Random(seed)
    for _ in range(6):
        i, j = r.randrange(M), r.randrange(K)
        if cplx:
            x = [(gen.to_canonical(hA[0], i * N + k), gen.to_canonical(hA[1], i * N + k)) for k in range(N)]
            y = [(gen.to_canonical(hB[0], k * K + j), gen.to_canonical(hB[1], k * K + j)) for k in range(N)]
            want = oracle.cdot(x, y, p)
        else:
            x = [gen.to_canonical(hA[0], i * N + k) for k in range(N)]
            y = [gen.to_canonical(hB[0], k * K + j) for k in range(N)]
            want = (oracle.dot(x, y, p),)
        for part, w in enumerate(want):
            (o, st) = outs[arbgpu.CHOICE_RNS128][part]
            assert compare_entry(gen.to_canonical(o, i * K + j), w, int(st[i * K + j])) is None


def test_tuner_records_a_choice_that_later_calls_follow(tmp_path):
    import torch
    M, N, K, p = 200, 96, 180, 256
    hA, hB, A, B = operands(9, M, N, K, 256, True, 250)
    path = tmp_path / "tune.json"
    ctx = arbgpu.Context(0, tune_cache=str(path))
    C = [arbgpu.DeviceOut.empty(M * K, p) for _ in range(2)]
    cm, am, bm = mats(A, B, C, M, N, K)
    ctx.mat_mul_raw(cm, am, bm, p, arbgpu.COMPLEX)
    torch.cuda.synchronize()
    before = [c.to_host() for c in C]
    choice = ctx.tune_mat_mul_raw(cm, am, bm, p, arbgpu.COMPLEX)
    say(f"tuned choice {choice}")
    assert choice in (1, 2, 3, 4)
    saved = json.loads(path.read_text())
    assert saved[class_key(M, N, K, p, True, True)] == choice
    ctx.mat_mul_raw(cm, am, bm, p, arbgpu.COMPLEX)
    torch.cuda.synchronize()
    after = [c.to_host() for c in C]
    for (a, sa), (b, sb) in zip(before, after):
        assert np.array_equal(a.limbs, b.limbs) and np.array_equal(a.nls, b.nls) and np.array_equal(sa, sb)
        assert np.array_equal(a.rad_m, b.rad_m) and np.array_equal(a.rad_e, b.rad_e)
    ctx.close()
