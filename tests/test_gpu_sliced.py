"""GPU parity of the scaled-integer INT8-MFMA matrix product (Algorithm 2)
against the exact oracle and against the limb kernel, through the C-ABI."""

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


def run(ctx, A, B, M, N, K, p, flags, Ai=None, Bi=None):
    import torch
    dA, dB = arbgpu.DeviceArray.from_host(A), arbgpu.DeviceArray.from_host(B)
    dAi = arbgpu.DeviceArray.from_host(Ai) if Ai is not None else None
    dBi = arbgpu.DeviceArray.from_host(Bi) if Bi is not None else None
    rad = not (flags & arbgpu.APPROX)
    C = arbgpu.DeviceOut.empty(M * K, p, radius=rad)
    Ci = arbgpu.DeviceOut.empty(M * K, p, radius=rad) if flags & arbgpu.COMPLEX else None
    ctx.mat_mul(C, dA, dB, M, N, K, p, flags, Ci=Ci, Ai=dAi, Bi=dBi)
    torch.cuda.synchronize()
    return C.to_host(), (Ci.to_host() if Ci is not None else None)


def check(out, st, want, entries, K, approx=False):
    bad = []
    for (i, j) in entries:
        e = compare_entry(gen.to_canonical(out, i * K + j), want(i, j), int(st[i * K + j]), approx)
        if e:
            bad.append(((i, j), e))
    assert not bad, bad[:5]


ALGOS = [arbgpu.ALGO_SLICED, arbgpu.ALGO_RNS]


@pytest.mark.parametrize("algo", ALGOS)
def test_sliced_config0_full(ctx, algo):
    w = gen.config0()
    say(f"sliced config0 64x64x64 p=128 algo={algo:#x}")
    (out, st), _ = run(ctx, w.A, w.B, w.M, w.N, w.K, w.p, algo)
    Ac = gen.canonical_matrix(w.A, w.M, w.N, w.N, 1)
    Bc = gen.canonical_matrix(w.B, w.N, w.K, w.K, 1)
    C = oracle.mat_mul(Ac, Bc, w.p)
    check(out, st, lambda i, j: C[i][j], [(i, j) for i in range(w.M) for j in range(w.K)], w.K)
    assert (st == 0).all()


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("seed,M,N,K,p,prec,erange,rshift", [
    (1, 5, 37, 70, 100, 120, 20, 110),       # ragged everywhere, balls, zeros
    (2, 300, 130, 257, 64, 64, 3, None),     # several tiles, K not a multiple of 128
    (3, 17, 300, 9, 333, 400, 40, 300),      # long inner dimension, wide operands
    (4, 1, 31, 1, 2, 50, 2, None),           # p = 2
])
def test_sliced_random_parity(ctx, seed, M, N, K, p, prec, erange, rshift, algo):
    rng = gen.rng_for(20, seed)
    A = gen.random_operands(rng, M * N, rng.integers(1, prec + 1, M * N), -erange, erange,
                            radius_shift=rshift, zero_frac=0.1)
    B = gen.random_operands(rng, N * K, rng.integers(1, prec + 1, N * K), -erange, erange,
                            radius_shift=rshift, zero_frac=0.1)
    if M > 2:
        A.limbs[:, N:2 * N] = 0
        A.nls[N:2 * N] = 0
    say(f"sliced random seed={seed} {M}x{N}x{K} p={p} algo={algo:#x}")
    (out, st), _ = run(ctx, A, B, M, N, K, p, algo)
    Ac = gen.canonical_matrix(A, M, N, N, 1)
    Bc = gen.canonical_matrix(B, N, K, K, 1)
    ent = [(i, j) for i in range(M) for j in range(K)]
    if len(ent) > 250:
        ent = random.Random(seed).sample(ent, 250)
    cols = {}
    def want(i, j):
        if j not in cols:
            cols[j] = [Bc[k][j] for k in range(N)]
        return oracle.dot(Ac[i], cols[j], p)
    check(out, st, want, ent, K)


@pytest.mark.parametrize("algo", ALGOS)
def test_sliced_exact_T(ctx, algo):
    # p larger than every exact sum: the output mantissa is the whole integer
    # block product T, so this checks T bit for bit
    rng = gen.rng_for(21, 0)
    M, N, K = 40, 90, 33
    A = gen.random_operands(rng, M * N, 200, -6, 6)
    B = gen.random_operands(rng, N * K, 160, -6, 6)
    p = 600
    say(f"sliced exact T algo={algo:#x}")
    (out, st), _ = run(ctx, A, B, M, N, K, p, algo)
    Ac = gen.canonical_matrix(A, M, N, N, 1)
    Bc = gen.canonical_matrix(B, N, K, K, 1)
    e, f, T = oracle.block_product([[x[0] for x in r] for r in Ac], [[x[0] for x in r] for r in Bc],
                                   list(range(N)))
    for i in range(M):
        for j in range(K):
            got = gen.to_canonical(out, i * K + j)
            want = oracle.truncate(T[i][j], -e[i] - f[j], p)
            assert not want[1]
            assert got[0] == want[0], (i, j)
            assert got[1] is None


@pytest.mark.parametrize("algo", ALGOS)
def test_sliced_complex(ctx, algo):
    rng = gen.rng_for(22, 0)
    M, N, K, p = 6, 45, 5, 120
    parts = [gen.random_operands(rng, c, 130, -10, 10, radius_shift=125, zero_frac=0.05)
             for c in (M * N, M * N, N * K, N * K)]
    say(f"sliced complex algo={algo:#x}")
    (out, st), (outi, sti) = run(ctx, parts[0], parts[2], M, N, K, p, arbgpu.COMPLEX | algo,
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


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6, 131])
def test_rns_complex_short_and_ragged_inner(ctx, N):
    # the three-product form adds the residues of the real and imaginary
    # parts and combines three residue planes per prime: inner lengths
    # below 4, not a multiple of 4, and one past a 128-byte step, with
    # residues of both signs (negative and zero entries)
    rng = gen.rng_for(26, N)
    M, K, p = 7, 5, 150
    parts = [gen.random_operands(rng, c, rng.integers(1, 200, c), -12, 12, radius_shift=140, zero_frac=0.1)
             for c in (M * N, M * N, N * K, N * K)]
    say(f"residue form complex inner N={N}")
    (out, st), (outi, sti) = run(ctx, parts[0], parts[2], M, N, K, p, arbgpu.COMPLEX | arbgpu.ALGO_RNS,
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


@pytest.mark.parametrize("cplx", [False, True])
def test_rns_paired_reconstruction(ctx, cplx):
    # 2048-bit operands over 65536 entries: the reconstruction's 64-entry
    # tile needs more than 64 KiB of LDS, so its waves take runs of limb
    # chunks of both 32-entry blocks together (every weight fragment feeding
    # two products) and the runs' carries are added per entry
    rng = gen.rng_for(27, int(cplx))
    M, N, K, p = 256, 40, 256, 2048
    prec = rng.integers(1900, 2049, 4 * M * N)
    A = gen.random_operands(rng, M * N, prec[:M * N], -8, 8, radius_shift=2040, zero_frac=0.05)
    B = gen.random_operands(rng, N * K, prec[M * N:M * N + N * K], -8, 8, zero_frac=0.05)
    Ai = gen.random_operands(rng, M * N, prec[2 * M * N:3 * M * N], -8, 8) if cplx else None
    Bi = gen.random_operands(rng, N * K, prec[3 * M * N:3 * M * N + N * K], -8, 8, radius_shift=2040) if cplx else None
    flags = (arbgpu.COMPLEX if cplx else 0) | arbgpu.ALGO_RNS
    say(f"residue form paired reconstruction complex={cplx}")
    (out, st), im = run(ctx, A, B, M, N, K, p, flags, Ai=Ai, Bi=Bi)
    r = random.Random(27)
    ent = [(r.randrange(M), r.randrange(K)) for _ in range(24)] + [(0, 0), (M - 1, K - 1), (63, 31), (64, 32)]
    if not cplx:
        Ac = gen.canonical_matrix(A, M, N, N, 1)
        Bc = gen.canonical_matrix(B, N, K, K, 1)
        check(out, st, lambda i, j: oracle.dot(Ac[i], [Bc[k][j] for k in range(N)], p), ent, K)
    else:
        (oi, si) = im
        for i, j in ent:
            x = [(gen.to_canonical(A, i * N + k), gen.to_canonical(Ai, i * N + k)) for k in range(N)]
            y = [(gen.to_canonical(B, k * K + j), gen.to_canonical(Bi, k * K + j)) for k in range(N)]
            re, imv = oracle.cdot(x, y, p)
            assert compare_entry(gen.to_canonical(out, i * K + j), re, int(st[i * K + j])) is None
            assert compare_entry(gen.to_canonical(oi, i * K + j), imv, int(si[i * K + j])) is None


@pytest.mark.parametrize("algo", ALGOS)
def test_config1_sliced_equals_limb_and_oracle(ctx, algo):
    w = gen.config1()
    say(f"config1 sliced vs limb 512^3 p=256 algo={algo:#x}")
    (o1, s1), _ = run(ctx, w.A, w.B, w.M, w.N, w.K, w.p, algo)
    (o2, s2), _ = run(ctx, w.A, w.B, w.M, w.N, w.K, w.p, arbgpu.ALGO_LIMB)
    # identical midpoints everywhere
    assert np.array_equal(o1.limbs, o2.limbs)
    assert np.array_equal(o1.exp, o2.exp) and np.array_equal(o1.nls, o2.nls)
    r = random.Random(3)
    ent = [(r.randrange(w.M), r.randrange(w.K)) for _ in range(30)]
    rows = {i: [gen.to_canonical(w.A, i * w.N + k) for k in range(w.N)] for i, _ in ent}
    cols = {j: [gen.to_canonical(w.B, k * w.K + j) for k in range(w.N)] for _, j in ent}
    check(o1, s1, lambda i, j: oracle.dot(rows[i], cols[j], w.p), ent, w.K)


def test_config2_sliced_sampled(ctx):
    w = gen.config2()
    say("config2 sliced 2048^3 p=512")
    (out, st), _ = run(ctx, w.A, w.B, w.M, w.N, w.K, w.p, arbgpu.ALGO_SLICED)
    assert (st == 0).all()
    # the residue form gives the same bits
    (o2, s2), _ = run(ctx, w.A, w.B, w.M, w.N, w.K, w.p, arbgpu.ALGO_RNS)
    assert np.array_equal(out.limbs, o2.limbs) and np.array_equal(out.exp, o2.exp)
    assert np.array_equal(out.nls, o2.nls) and np.array_equal(out.rad_m, o2.rad_m) and np.array_equal(st, s2)
    # an independent check of whole rows: the first 64 rows of the product
    # from the limb-window kernel (no slicing, no residues, no MFMA) are the
    # same bits as the INT8 product's
    R = 64
    Ab = gen.Operands(w.A.limbs[:, :R * w.N].copy(), w.A.exp[:R * w.N].copy(), w.A.nls[:R * w.N].copy(), None, None)
    say("config2 limb-kernel row block 64x2048x2048 p=512")
    (o3, s3), _ = run(ctx, Ab, w.B, R, w.N, w.K, w.p, arbgpu.ALGO_LIMB)
    n = R * w.K
    assert np.array_equal(o3.limbs, out.limbs[:, :n]) and np.array_equal(o3.exp, out.exp[:n])
    assert np.array_equal(o3.nls, out.nls[:n])
    r = random.Random(4)
    ent = [(r.randrange(w.M), r.randrange(w.K)) for _ in range(10)] + [(0, 0), (w.M - 1, w.K - 1)]
    rows = {i: [gen.to_canonical(w.A, i * w.N + k) for k in range(w.N)] for i, _ in ent}
    cols = {j: [gen.to_canonical(w.B, k * w.K + j) for k in range(w.N)] for _, j in ent}
    check(out, st, lambda i, j: oracle.dot(rows[i], cols[j], w.p), ent, w.K)


def full_height_operands(rng, count, h, exp_lo, exp_hi):
    """Operands whose mantissas have exactly h significant bits, a quarter of
    them all ones (the scaled integer 2^h - 1 when the line's exponents
    agree), both signs."""
    ops = gen.random_operands(rng, count, h, exp_lo, exp_hi)
    ones = rng.random(count) < 0.25
    balls = []
    for i in range(count):
        m, r = gen.to_canonical(ops, i)
        if ones[i] and m[1]:
            m = oracle.fmake(m[0], (1 << h) - 1, m[2])
        balls.append((m, r))
    return gen.from_canonical(balls, cap=ops.cap)


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("h", [7, 8, 15, 23, 31, 63, 64, 127, 255, 519, 520])
def test_digit_count_at_every_height_class(ctx, algo, h):
    # rows of A and columns of B of integer height exactly h (one exponent
    # per line, mantissas of h bits, entries up to 2^h - 1 in magnitude):
    # heights 8 L - 1 need L + 1 balanced base-256 digits, the largest
    # values the most.  The exact block product T is compared with the
    # oracle's integer product, and the midpoints with the limb kernel
    rng = gen.rng_for(28, h)
    M, N, K = 9, 6, 7
    A = full_height_operands(rng, M * N, h, 0, 0)
    B = full_height_operands(rng, N * K, h, 0, 0)
    A.exp[:] = np.repeat(rng.integers(-5, 6, M), N).astype(np.int32) * (A.nls != 0)
    B.exp[:] = np.tile(rng.integers(-5, 6, K), N).astype(np.int32) * (B.nls != 0)
    p = 2 * h + 16
    say(f"digit count h={h} algo={algo:#x}")
    (out, st), _ = run(ctx, A, B, M, N, K, p, algo)
    Ac = gen.canonical_matrix(A, M, N, N, 1)
    Bc = gen.canonical_matrix(B, N, K, K, 1)
    e, f, T = oracle.block_product([[x[0] for x in r] for r in Ac], [[x[0] for x in r] for r in Bc],
                                   list(range(N)))
    assert max(abs(x) for row in T for x in row) > 0
    for i in range(M):
        for j in range(K):
            want = oracle.truncate(T[i][j], -e[i] - f[j], p)
            assert not want[1]
            assert gen.to_canonical(out, i * K + j)[0] == want[0], (i, j)
    (o2, s2), _ = run(ctx, A, B, M, N, K, p, arbgpu.ALGO_LIMB)
    assert np.array_equal(out.limbs, o2.limbs) and np.array_equal(out.nls, o2.nls)


@pytest.mark.parametrize("seed,spread,bside", [(1, 700, False), (2, 300, True), (3, 1500, True)])
def test_sliced_radius_wide_range(ctx, seed, spread, bside):
    # radii spread over many binades inside one row (and column): the
    # per-line FP64 frames cannot hold them all, so the per-entry radius
    # kernel takes over; tiny radii next to large midpoints exercise the
    # |b| + r_b bump
    rng = gen.rng_for(23, seed)
    M, N, K, p = 13, 70, 11, 150
    A = gen.random_operands(rng, M * N, 150, -8, 8, radius_shift=140)
    B = gen.random_operands(rng, N * K, 150, -8, 8, radius_shift=140 if bside else None)
    A.rad_e[::2] -= spread
    if bside:
        B.rad_e[1::3] -= spread
    say(f"sliced radius spread={spread} seed={seed}")
    (out, st), _ = run(ctx, A, B, M, N, K, p, arbgpu.ALGO_SLICED)
    Ac = gen.canonical_matrix(A, M, N, N, 1)
    Bc = gen.canonical_matrix(B, N, K, K, 1)
    C = oracle.mat_mul(Ac, Bc, p)
    check(out, st, lambda i, j: C[i][j], [(i, j) for i in range(M) for j in range(K)], K)


@pytest.mark.parametrize("cplx", [False, True])
def test_rns_widest_shapes(ctx, cplx):
    # operands near 4000 bits: ~540 primes, ~252 limbs of T, 126 digit
    # words (the residue sums allow 127); the residue slicer runs with 64
    # elements per workgroup and the reconstruction with 32 entries per
    # workgroup in about 70 KiB of LDS
    rng = gen.rng_for(24, int(cplx))
    M, N, K, p = 4, 9, 3, 4000
    prec = rng.integers(3800, 4001, 4 * M * N)
    A = gen.random_operands(rng, M * N, prec[:M * N], -3, 3, radius_shift=3990, zero_frac=0.05)
    B = gen.random_operands(rng, N * K, prec[M * N:M * N + N * K], -3, 3, zero_frac=0.05)
    Ai = gen.random_operands(rng, M * N, prec[2 * M * N:3 * M * N], -3, 3, radius_shift=3990) if cplx else None
    Bi = gen.random_operands(rng, N * K, prec[3 * M * N:3 * M * N + N * K], -3, 3) if cplx else None
    flags = arbgpu.COMPLEX if cplx else 0
    say(f"residue form widest shapes complex={cplx}")
    (out, st), im = run(ctx, A, B, M, N, K, p, flags | arbgpu.ALGO_RNS, Ai=Ai, Bi=Bi)
    plan = ctx.plan_info()
    assert plan["primes"] > 500, plan
    # the base-256 slices give the same bits
    (o2, s2), im2 = run(ctx, A, B, M, N, K, p, flags | arbgpu.ALGO_SLICED, Ai=Ai, Bi=Bi)
    assert np.array_equal(out.limbs, o2.limbs) and np.array_equal(out.exp, o2.exp)
    assert np.array_equal(out.nls, o2.nls) and np.array_equal(out.rad_m, o2.rad_m)
    ent = [(i, j) for i in range(M) for j in range(K)]
    if not cplx:
        Ac = gen.canonical_matrix(A, M, N, N, 1)
        Bc = gen.canonical_matrix(B, N, K, K, 1)
        check(out, st, lambda i, j: oracle.dot(Ac[i], [Bc[k][j] for k in range(N)], p), ent, K)
    else:
        (oi, si) = im
        Ac = [[(gen.to_canonical(A, i * N + k), gen.to_canonical(Ai, i * N + k)) for k in range(N)]
              for i in range(M)]
        Bc = [[(gen.to_canonical(B, k * K + j), gen.to_canonical(Bi, k * K + j)) for j in range(K)]
              for k in range(N)]
        for i, j in ent:
            re, imv = oracle.cdot(Ac[i], [Bc[k][j] for k in range(N)], p)
            assert compare_entry(gen.to_canonical(out, i * K + j), re, int(st[i * K + j])) is None
            assert compare_entry(gen.to_canonical(oi, i * K + j), imv, int(si[i * K + j])) is None


def test_rns_beyond_its_limits(ctx):
    # 4070-bit operands: 128 digit words, more than the residue sums allow
    # (127), so a forced residue product is refused and the automatic
    # choice takes the base-256 slices (heights < 4095 bits)
    rng = gen.rng_for(25, 0)
    M, N, K, p = 2, 5, 2, 4070
    A = gen.random_operands(rng, M * N, 4070, -3, 3)
    B = gen.random_operands(rng, N * K, 4070, -3, 3)
    with pytest.raises(arbgpu.ArbgpuError, match="residue form does not fit"):
        run(ctx, A, B, M, N, K, p, arbgpu.ALGO_RNS)
    (out, st), _ = run(ctx, A, B, M, N, K, p, 0)
    assert ctx.plan_info()["primes"] == 0
    Ac = gen.canonical_matrix(A, M, N, N, 1)
    Bc = gen.canonical_matrix(B, N, K, K, 1)
    check(out, st, lambda i, j: oracle.dot(Ac[i], [Bc[k][j] for k in range(N)], p),
          [(i, j) for i in range(M) for j in range(K)], K)


def test_truncated_slices_certify_or_fall_back(ctx):
    # Base-256 slices leave out the low diagonals of the integer product
    # when they lie far below the output's p bits.  Rows whose terms cancel
    # in pairs against columns that negate in pairs give exact zeros and
    # tiny sums, which the truncated product cannot certify: those entries
    # are recomputed exactly; every midpoint equals the limb kernel's
    rng = gen.rng_for(29, 0)
    M, N, K, p = 40, 64, 30, 200
    A = gen.random_operands(rng, M * N, 220, -3, 3)
    B = gen.random_operands(rng, N * K, 220, -3, 3)
    a = [gen.to_canonical(A, i) for i in range(M * N)]
    b = [gen.to_canonical(B, i) for i in range(N * K)]
    rows, zero_cols, tiny_cols = (0, 5, 17), (0, 3, 29), (7,)
    for i in rows:
        for t in range(N // 2):
            a[i * N + 2 * t + 1] = a[i * N + 2 * t]
    for j in zero_cols + tiny_cols:
        for t in range(N // 2):
            b[(2 * t + 1) * K + j] = (oracle.fneg(b[2 * t * K + j][0]), None)
    for j in tiny_cols:   # one pair does not cancel: its small leftover is the exact sum
        b[1 * K + j] = (oracle.fmake(0, (1 << 30) + 1, -90), None)
    A, B = gen.from_canonical(a, cap=A.cap), gen.from_canonical(b, cap=B.cap)
    say("truncated slices with cancelling entries")
    (out, st), _ = run(ctx, A, B, M, N, K, p, arbgpu.ALGO_SLICED)
    plan = ctx.plan_info()
    assert plan["pairs"] < plan["slices_a"] * plan["slices_b"]   # the truncated set was used
    (o2, s2), _ = run(ctx, A, B, M, N, K, p, arbgpu.ALGO_LIMB)
    assert np.array_equal(out.limbs, o2.limbs) and np.array_equal(out.exp, o2.exp)
    assert np.array_equal(out.nls, o2.nls)
    Ac = gen.canonical_matrix(A, M, N, N, 1)
    Bc = gen.canonical_matrix(B, N, K, K, 1)
    ent = [(i, j) for i in rows for j in zero_cols + tiny_cols] + [(1, 1), (39, 29)]
    check(out, st, lambda i, j: oracle.dot(Ac[i], [Bc[k][j] for k in range(N)], p), ent, K)
    for i in rows:
        for j in zero_cols:
            assert out.nls[i * K + j] == 0   # exact zeros


@pytest.mark.parametrize("p", [512, 1024])
def test_rns_complex_three_products_equal_four_and_limb(ctx, p):
    # 65536 complex entries: the imaginary parts' slicers form the residues
    # of re + im (128 elements per workgroup), the reconstruction runs 64
    # entries per workgroup (two runs of chunks per block at p = 512, the
    # paired blocks at p = 1024); the three-product form, the four-product
    # form and the limb kernel give the same midpoints everywhere
    rng = gen.rng_for(31, p)
    M, N, K = 256, 64, 256
    prec = rng.integers(p // 2, p + 1, 4 * M * N)
    A = gen.random_operands(rng, M * N, prec[:M * N], -6, 6, radius_shift=p - 8, zero_frac=0.05)
    B = gen.random_operands(rng, N * K, prec[M * N:M * N + N * K], -6, 6, zero_frac=0.05)
    Ai = gen.random_operands(rng, M * N, prec[2 * M * N:3 * M * N], -6, 6, zero_frac=0.05)
    Bi = gen.random_operands(rng, N * K, prec[3 * M * N:3 * M * N + N * K], -6, 6, radius_shift=p - 8)
    say(f"complex 256x64x256 p={p}: three products, four products, limb kernel")
    base = arbgpu.COMPLEX | arbgpu.ALGO_RNS
    (o3, s3), (i3, t3) = run(ctx, A, B, M, N, K, p, base, Ai=Ai, Bi=Bi)
    (o4, s4), (i4, t4) = run(ctx, A, B, M, N, K, p, base | arbgpu.COMPLEX_4M, Ai=Ai, Bi=Bi)
    (ol, sl), (il, tl) = run(ctx, A, B, M, N, K, p, arbgpu.COMPLEX | arbgpu.ALGO_LIMB, Ai=Ai, Bi=Bi)
    for a, b in ((o3, o4), (i3, i4), (o3, ol), (i3, il)):
        assert np.array_equal(a.limbs, b.limbs)
        assert np.array_equal(a.exp, b.exp) and np.array_equal(a.nls, b.nls)
    r = random.Random(31)
    for i, j in [(r.randrange(M), r.randrange(K)) for _ in range(6)] + [(0, 0), (M - 1, K - 1)]:
        x = [(gen.to_canonical(A, i * N + k), gen.to_canonical(Ai, i * N + k)) for k in range(N)]
        y = [(gen.to_canonical(B, k * K + j), gen.to_canonical(Bi, k * K + j)) for k in range(N)]
        re, imv = oracle.cdot(x, y, p)
        assert compare_entry(gen.to_canonical(o3, i * K + j), re, int(s3[i * K + j])) is None
        assert compare_entry(gen.to_canonical(i3, i * K + j), imv, int(t3[i * K + j])) is None
