"""Pins for the oracle's matrix product, scaled integer blocks and greedy
block extraction (Section 4, Algorithm 2, Table 3)."""

import random
from fractions import Fraction

import pytest
from mpmath import libmp

import oracle


def fr(x):
    s, M, e = x
    if M == 0:
        return Fraction(0)
    v = Fraction(M) * Fraction(2) ** (e - M.bit_length())
    return -v if s else v


def rand_float(rng, bits, elo, ehi, zero_p=0.0):
    if rng.random() < zero_p:
        return oracle.ZERO
    M = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    return oracle.fmake(rng.getrandbits(1), M, rng.randint(elo, ehi))


@pytest.mark.parametrize("seed", range(4))
def test_block_product_against_brute_force(seed):
    rng = random.Random(seed)
    M, N, K = 5, 9, 4
    A = [[rand_float(rng, rng.randint(1, 70), -20, 20, 0.15) for _ in range(N)] for _ in range(M)]
    B = [[rand_float(rng, rng.randint(1, 70), -20, 20, 0.15) for _ in range(K)] for _ in range(N)]
    A[2] = [oracle.ZERO] * N     # an all-zero row
    s = [1, 2, 3, 5, 6]
    e, f, T = oracle.block_product(A, B, s)
    for i in range(M):
        for j in range(K):
            exact = sum((fr(A[i][k]) * fr(B[k][j]) for k in s), Fraction(0))
            assert Fraction(T[i][j]) * Fraction(2) ** (-e[i] - f[j]) == exact
    # minimal height: each nonzero row of E_s A_s is integral with an odd entry
    for i in range(M):
        row = [fr(A[i][k]) * Fraction(2) ** e[i] for k in s]
        assert all(v.denominator == 1 for v in row)
        if any(row):
            assert any(v.numerator % 2 for v in row)
        else:
            assert e[i] == 0
    for j in range(K):
        col = [fr(B[k][j]) * Fraction(2) ** f[j] for k in s]
        assert all(v.denominator == 1 for v in col)
        if any(col):
            assert any(v.numerator % 2 for v in col)


@pytest.mark.parametrize("seed", range(3))
def test_matmul_entry_is_dot(seed):
    rng = random.Random(10 + seed)
    A = [[(rand_float(rng, 50, -10, 10), oracle.rmake(rng.getrandbits(20), -90)) for _ in range(6)] for _ in range(3)]
    B = [[(rand_float(rng, 50, -10, 10), None) for _ in range(2)] for _ in range(6)]
    C = oracle.mat_mul(A, B, 33)
    for i in range(3):
        for j in range(2):
            assert C[i][j] == oracle.dot(A[i], [B[k][j] for k in range(6)], 33)


def test_block_partition_does_not_change_product():
    # Splitting the inner dimension into scaled integer blocks and adding the
    # exact block contributions reproduces the exact product (Algorithm 2
    # with one final rounding).
    rng = random.Random(3)
    A = [[rand_float(rng, 40, -600 + 100 * k, -590 + 100 * k) for k in range(12)] for _ in range(4)]
    B = [[rand_float(rng, 40, -5, 5) for _ in range(3)] for _ in range(12)]
    blocks = oracle.extract_blocks(A, B, 30, basecase=2)
    assert len(blocks) > 1
    for i in range(4):
        for j in range(3):
            total = Fraction(0)
            for k0, k1, kind in blocks:
                e, f, T = oracle.block_product(A, B, list(range(k0, k1)))
                total += Fraction(T[i][j]) * Fraction(2) ** (-e[i] - f[j])
            exact = sum((fr(A[i][k]) * fr(B[k][j]) for k in range(12)), Fraction(0))
            assert total == exact


def test_height_bound():
    assert oracle.height_bound(128, 128, 128) == 352
    assert oracle.height_bound(53, 200, 10) == Fraction(5, 4) * 53 + 192
    assert oracle.height_bound(512, 100, 300) == Fraction(5, 4) * 300 + 192


def test_uniform_matrix_is_one_block():
    rng = random.Random(9)
    A = [[rand_float(rng, 64, -4, 4) for _ in range(40)] for _ in range(6)]
    B = [[rand_float(rng, 64, -4, 4) for _ in range(5)] for _ in range(40)]
    assert oracle.extract_blocks(A, B, 64) == [(0, 40, "block")]
    # a short inner dimension is a basecase chunk
    assert oracle.extract_blocks([r[:10] for r in A], B[:10], 64) == [(0, 10, "basecase")]


# ---------------------------------------------------------------- Table 3

def _pascal(N, p):
    """Entries pi * binomial(i+j, i) rounded to p bits (nearest)."""
    pi = libmp.mpf_pi(p + 64)
    row = []
    A = [[None] * N for _ in range(N)]
    for i in range(N):
        c = 1   # binomial(i + j, i) for j = 0
        for j in range(N):
            if j > 0:
                c = c * (i + j) // j
            if j < i:
                A[i][j] = A[j][i]
                continue
            sign, man, exp, bc = libmp.mpf_mul(pi, libmp.from_int(c), p, 'n')
            A[i][j] = oracle.fmake(sign, man, exp + bc)
    return A


TABLE3 = {   # (N, p) -> number of blocks printed in Table 3 (1 where none is printed)
    (100, 53): 1, (100, 106): 1, (100, 212): 1, (100, 848): 1, (100, 3392): 1,
    (300, 53): 3, (300, 106): 3, (300, 212): 3, (300, 848): 2, (300, 3392): 1,
    (1000, 53): 10, (1000, 106): 10, (1000, 212): 9, (1000, 848): 5, (1000, 3392): 2,
}


@pytest.mark.parametrize("N", [100, 300])
def test_table3_pascal_block_counts(N):
    for p in (53, 106, 212, 848, 3392):
        A = _pascal(N, p)
        blocks = oracle.extract_blocks(A, A, p)
        assert len(blocks) == TABLE3[(N, p)], (N, p, blocks)
        assert blocks[0][0] == 0 and blocks[-1][1] == N
        assert all(b[1] == c[0] for b, c in zip(blocks, blocks[1:]))


@pytest.mark.slow
def test_table3_pascal_block_counts_n1000():
    for p in (53, 106, 212, 848, 3392):
        A = _pascal(1000, p)
        blocks = oracle.extract_blocks(A, A, p)
        assert len(blocks) == TABLE3[(1000, p)], (p, [(b[0], b[1], b[2]) for b in blocks])


def test_short_greedy_block_extends_to_basecase():
    # Column k has exponent 40k, so a greedy block holds only 6 columns
    # (height 40m + 40 <= h = 1.25*40 + 192); the basecase rule extends it to
    # 30 indices, and the tail becomes a shorter basecase chunk.
    rng = random.Random(21)
    A = [[oracle.fmake(0, (rng.getrandbits(40) | (1 << 39) | 1), 40 * k) for k in range(50)] for _ in range(3)]
    B = [[oracle.fmake(0, 1, 1) for _ in range(2)] for _ in range(50)]
    assert oracle.extract_blocks(A, B, 40) == [(0, 30, "basecase"), (30, 50, "basecase")]
    assert oracle.extract_blocks(A, B, 40, basecase=1)[0] == (0, 6, "block")
