"""Pins for the exact oracle's dot products.

The oracle is checked against things other than itself: a Fraction-based
brute force that never forms a common denominator, mpmath's round-down
(a library routine), closed forms, invariants that the definition implies
(Section 2 and Section 3: the initial/sub convention, the enclosure, the
zero-radius rule for exact data), and containment of sampled points.
"""

import random
from fractions import Fraction

import pytest
from hypothesis import given, settings, strategies as st
from mpmath import libmp

import oracle
from oracle import arb

# ---------------------------------------------------------------- helpers


def fr(x):
    """Float tuple -> Fraction, written independently of oracle.fvalue."""
    s, M, e = x
    if M == 0:
        return Fraction(0)
    v = Fraction(M) * Fraction(2) ** (e - len(bin(M)) + 2)
    return -v if s else v


def rfr(r):
    if r is None:
        return Fraction(0)
    R, g = r
    return Fraction(R) * Fraction(2) ** g


def trunc_fraction(v: Fraction, p: int):
    """Round-toward-zero of a dyadic Fraction to p bits via mpmath."""
    if v == 0:
        return Fraction(0)
    num, den = v.numerator, v.denominator
    assert den & (den - 1) == 0
    sign, man, exp, bc = libmp.from_man_exp(num, -(den.bit_length() - 1), p, 'd')
    r = Fraction(man) * Fraction(2) ** exp
    return -r if sign else r


floats = st.builds(
    lambda s, M, e: oracle.fmake(s, M, e),
    st.integers(0, 1), st.integers(0, 2**64 - 1), st.integers(-40, 40))
radii = st.one_of(st.none(), st.builds(lambda R, g: oracle.rmake(R, g),
                                       st.integers(0, 2**53 - 1), st.integers(-120, 0)))
balls = st.tuples(floats, radii)


def rand_float(rng, bits, elo, ehi):
    M = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
    return oracle.fmake(rng.getrandbits(1), M, rng.randint(elo, ehi))

# ------------------------------------------------------- brute force pins


@settings(max_examples=300, deadline=None)
@given(st.lists(st.tuples(balls, balls), min_size=0, max_size=8),
       st.integers(2, 140), st.booleans(), st.one_of(st.none(), balls))
def test_dot_matches_fraction_brute_force(pairs, p, sub, initial):
    x = [a for a, _ in pairs]
    y = [b for _, b in pairs]
    res = oracle.dot(x, y, p, initial=initial, sub=sub)
    S = sum((fr(a[0]) * fr(b[0]) for a, b in pairs), Fraction(0))
    if sub:
        S = -S
    if initial is not None:
        S += fr(initial[0])
    want = trunc_fraction(S, p)
    assert fr(res.mid) == want
    assert res.inexact == (want != S)
    # exact enclosure radius
    rho = sum((abs(fr(a[0])) * rfr(b[1]) + abs(fr(b[0])) * rfr(a[1]) + rfr(a[1]) * rfr(b[1])
               for a, b in pairs), Fraction(0))
    if initial is not None:
        rho += rfr(initial[1])
    if res.inexact:
        e_m = res.mid[2]
        rho += Fraction(2) ** (e_m - p)
    assert rfr(res.rad) == rho
    # the midpoint is canonical (odd mantissa) and has at most p bits
    if res.mid[1]:
        assert res.mid[1] & 1 and res.mid[1].bit_length() <= p
        assert Fraction(2) ** (res.mid[2] - 1) <= abs(fr(res.mid)) < Fraction(2) ** res.mid[2]
    # enclosure: |S - m| <= radius
    assert abs(S - fr(res.mid)) <= rfr(res.rad)


@settings(max_examples=200, deadline=None)
@given(floats, floats, st.integers(2, 200))
def test_single_product_matches_mpmath_mul(a, b, p):
    res = oracle.dot([(a, None)], [(b, None)], p)
    ma = libmp.from_man_exp(-a[1] if a[0] else a[1], a[2] - a[1].bit_length()) if a[1] else libmp.fzero
    mb = libmp.from_man_exp(-b[1] if b[0] else b[1], b[2] - b[1].bit_length()) if b[1] else libmp.fzero
    prod = libmp.mpf_mul(ma, mb, p, 'd')
    sign, man, exp, bc = prod
    want = Fraction(man) * Fraction(2) ** exp * (-1 if sign else 1) if man else Fraction(0)
    assert fr(res.mid) == want


def test_truncation_worked_example():
    # 95 = 0b1011111 to 4 bits toward zero is 88 = 0b1011000, both signs
    f, inexact = oracle.truncate(95, 0, 4)
    assert fr(f) == 88 and inexact
    f, inexact = oracle.truncate(-95, 0, 4)
    assert fr(f) == -88 and inexact
    f, inexact = oracle.truncate(88, 0, 4)
    assert fr(f) == 88 and not inexact

# ----------------------------------------------------------- closed forms


@pytest.mark.parametrize("N,p", [(1, 2), (3, 5), (3, 4), (10, 19), (10, 20), (64, 128), (100, 53)])
def test_geometric_closed_form(N, p):
    # sum_{i<N} 2^-i * 2^-i = 1.0101...01 in binary (2N-1 bits)
    x = [((0, 1, 1 - i), None) for i in range(N)]
    res = oracle.dot(x, x, p)
    bits = 2 * N - 1
    full = int("10" * (N - 1) + "1", 2)
    if bits <= p:
        assert fr(res.mid) == Fraction(full, 2 ** (bits - 1)) and not res.inexact
        assert res.rad == (0, 0)
    else:
        top = full >> (bits - p)
        assert fr(res.mid) == Fraction(top, 2 ** (p - 1)) and res.inexact
        assert rfr(res.rad) == Fraction(1, 2 ** (p - 1))


def test_distinct_powers_exact_iff_span_fits():
    ks = [7, 3, -20, -41]
    x = [((0, 1, k + 1), None) for k in ks]
    y = [((0, 1, 1), None)] * len(ks)
    span = max(ks) - min(ks) + 1
    res = oracle.dot(x, y, span)
    assert not res.inexact and fr(res.mid) == sum(Fraction(2) ** k for k in ks)
    res = oracle.dot(x, y, span - 1)
    assert res.inexact and fr(res.mid) == sum(Fraction(2) ** k for k in ks[:-1])


def test_cancellation_gives_exact_zero_ball():
    rng = random.Random(5)
    a = rand_float(rng, 200, -5, 5)
    b = rand_float(rng, 200, -5, 5)
    res = oracle.dot([(a, None), (oracle.fneg(a), None)], [(b, None), (b, None)], 64)
    assert res.mid == oracle.ZERO and res.rad == (0, 0) and not res.inexact


def test_empty_dot_and_initial_only():
    res = oracle.dot([], [], 10)
    assert res.mid == oracle.ZERO and res.rad == (0, 0)
    init = (oracle.fmake(1, 0b1011011, 3), (3, -10))
    res = oracle.dot([], [], 4, initial=init)
    assert fr(res.mid) == trunc_fraction(fr(init[0]), 4)
    assert res.inexact


def test_p_below_two_rejected():
    with pytest.raises(ValueError):
        oracle.dot([], [], 1)

# ------------------------------------------------------------- invariants


def _rand_balls(rng, n, bits=100, erange=30, rad=True):
    out = []
    for _ in range(n):
        m = rand_float(rng, rng.randint(1, bits), -erange, erange)
        r = oracle.rmake(rng.getrandbits(50), rng.randint(-200, -100)) if rad and rng.random() < 0.7 else None
        out.append((m, r))
    return out


@pytest.mark.parametrize("seed", range(8))
def test_permutation_invariance(seed):
    rng = random.Random(seed)
    x, y = _rand_balls(rng, 40), _rand_balls(rng, 40)
    perm = list(range(40))
    rng.shuffle(perm)
    a = oracle.dot(x, y, 77)
    b = oracle.dot([x[i] for i in perm], [y[i] for i in perm], 77)
    assert a == b


@pytest.mark.parametrize("seed", range(6))
def test_power_of_two_scaling(seed):
    rng = random.Random(100 + seed)
    x, y = _rand_balls(rng, 25, rad=False), _rand_balls(rng, 25, rad=False)
    t = rng.randint(-50, 50)
    xs = [((m[0], m[1], m[2] + t), r) for m, r in x]
    a = oracle.dot(x, y, 90)
    b = oracle.dot(xs, y, 90)
    assert b.mid[:2] == a.mid[:2] and b.mid[2] == a.mid[2] + t
    assert b.inexact == a.inexact


@pytest.mark.parametrize("seed", range(6))
def test_sub_is_negation_and_initial_is_extra_term(seed):
    rng = random.Random(200 + seed)
    x, y = _rand_balls(rng, 30), _rand_balls(rng, 30)
    init = _rand_balls(rng, 1)[0]
    a = oracle.dot(x, y, 64)
    b = oracle.dot(x, y, 64, sub=True)
    assert b.mid == oracle.fneg(a.mid) and b.rad == a.rad and b.inexact == a.inexact
    one = ((0, 1, 1), None)
    c = oracle.dot(x, y, 64, initial=init)
    d = oracle.dot(x + [init], y + [one], 64)
    assert c == d
    # initial with sub: initial - sum == initial + sum((-x_i) y_i)
    e = oracle.dot(x, y, 64, initial=init, sub=True)
    f = oracle.dot([(oracle.fneg(m), r) for m, r in x] + [init], y + [one], 64)
    assert e == f


@pytest.mark.parametrize("seed", range(4))
def test_complex_with_zero_imaginary_is_real(seed):
    rng = random.Random(300 + seed)
    x, y = _rand_balls(rng, 20), _rand_balls(rng, 20)
    z = (oracle.ZERO, None)
    re, im = oracle.cdot([(a, z) for a in x], [(b, z) for b in y], 80)
    assert re == oracle.dot(x, y, 80)
    assert im.mid == oracle.ZERO and im.rad == (0, 0)


@pytest.mark.parametrize("seed", range(4))
def test_complex_against_fraction_definition(seed):
    rng = random.Random(400 + seed)
    n = 12
    x = [(b1, b2) for b1, b2 in zip(_rand_balls(rng, n), _rand_balls(rng, n))]
    y = [(b1, b2) for b1, b2 in zip(_rand_balls(rng, n), _rand_balls(rng, n))]
    re, im = oracle.cdot(x, y, 70)
    Sre = sum((fr(a[0]) * fr(c[0]) - fr(b[0]) * fr(d[0]) for (a, b), (c, d) in zip(x, y)), Fraction(0))
    Sim = sum((fr(a[0]) * fr(d[0]) + fr(b[0]) * fr(c[0]) for (a, b), (c, d) in zip(x, y)), Fraction(0))
    assert fr(re.mid) == trunc_fraction(Sre, 70)
    assert fr(im.mid) == trunc_fraction(Sim, 70)
    assert abs(Sre - fr(re.mid)) <= rfr(re.rad)
    assert abs(Sim - fr(im.mid)) <= rfr(im.rad)


def test_zero_radius_iff_exact_inputs_and_exact_result():
    rng = random.Random(7)
    x, y = _rand_balls(rng, 10, bits=20, rad=False), _rand_balls(rng, 10, bits=20, rad=False)
    res = oracle.dot(x, y, 400)          # wide enough: exact
    assert not res.inexact and res.rad == (0, 0)
    res = oracle.dot(x, y, 8)            # inexact: nonzero radius
    assert res.inexact and res.rad[0] > 0
    x[3] = (x[3][0], (1, -300))          # one inexact input: nonzero radius
    res = oracle.dot(x, y, 400)
    assert not res.inexact and res.rad[0] > 0


@pytest.mark.parametrize("seed", range(5))
def test_containment_of_sampled_points(seed):
    rng = random.Random(500 + seed)
    x, y = _rand_balls(rng, 15, bits=60), _rand_balls(rng, 15, bits=60)
    res = oracle.dot(x, y, 40)
    m, R = fr(res.mid), rfr(res.rad)
    for _ in range(50):
        S = Fraction(0)
        for a, b in zip(x, y):
            pa = fr(a[0]) + rfr(a[1]) * Fraction(rng.randint(-8, 8), 8)
            pb = fr(b[0]) + rfr(b[1]) * Fraction(rng.randint(-8, 8), 8)
            S += pa * pb
        assert abs(S - m) <= R


def test_reduced_precision_cut():
    # e_max = 2 (1*1 products with exponent 1+1), e_rad = 2 - 40 + 1 ... :
    one = (0, 1, 1)
    x = [(one, (1, -40))]
    y = [(one, None)]
    # radius product |m_y| r_x has exponent 1 + (-40 + 1) = -38; e_max = 2
    assert oracle.reduced_precision([(0, x[0], y[0])], 200) == 2 - (-38) + 30
    assert oracle.reduced_precision([(0, x[0], y[0])], 20) == 20
    assert oracle.reduced_precision([], 20) == 2
    r = oracle.dot(x, y, 200, reduce_prec=True)
    assert fr(r.mid) == 1


def test_reduced_precision_cut_complex():
    # x = [1 +- 2^-40] + [3 +- 0] i, y = 1 + 1 i (exact): both parts are
    # exact small integers, unchanged by any cut of at least 2 bits
    one = (0, 1, 1)
    three = (0, 3, 2)
    x = [((one, (1, -40)), (three, None))]
    y = [((one, None), (one, None))]
    re, im = oracle.cdot(x, y, 500, reduce_prec=True)
    assert fr(re.mid) == -2 and fr(im.mid) == 4
    # an inexact case: a 200-bit mantissa near 2/3 with zero imaginary
    # parts reduces to the real cut dot
    m = (1 << 200) // 3 | 1
    xm = (0, m, 1)
    x2 = [((xm, (1, -40)), (oracle.ZERO, None))]
    y2 = [((one, None), (oracle.ZERO, None))]
    re2, im2 = oracle.cdot(x2, y2, 500, reduce_prec=True)
    real = oracle.dot([(xm, (1, -40))], [(one, None)], 500, reduce_prec=True)
    assert re2.mid == real.mid and re2.rad == real.rad
    # the real dot is cut to 1 + 38 + 30 = 69 bits (e_max = 1 + 1 = 2, e_rad = 1 - 39 = -38)
    assert oracle.fprec(re2.mid) <= 70 and re2.inexact
    assert im2.mid == oracle.ZERO


def test_badly_scaled_matrix_keeps_entrywise_accuracy():
    # The 3x3 example of Section 2 times the identity and times itself.
    ten = Fraction(10)
    entries = [[(Fraction(123) * ten ** 98, ten ** 80), (Fraction(-3, 2), 0), (0, 0)],
               [(1, 0), (Fraction(234, 100), ten ** -20), (Fraction(345, 100), ten ** -50)],
               [(0, 0), (2, 0), (Fraction(456) * ten ** -102, ten ** -130)]]

    def to_ball(v, r, prec=400):
        if v == 0:
            mid = oracle.ZERO
        else:
            sgn = 1 if v < 0 else 0
            a = abs(v)
            e = a.numerator.bit_length() - a.denominator.bit_length() + 1
            M = (a * Fraction(2) ** (prec - e)).numerator // (a * Fraction(2) ** (prec - e)).denominator
            mid = oracle.fmake(sgn, M, e - prec + M.bit_length())
        if r == 0:
            rad = None
        else:
            e = r.numerator.bit_length() - r.denominator.bit_length() + 1
            R = -(-(r * Fraction(2) ** (53 - e)).numerator // (r * Fraction(2) ** (53 - e)).denominator)
            rad = oracle.rmake(R, e - 53)
        return (mid, rad)

    A = [[to_ball(v, r) for v, r in row] for row in entries]
    I = [[((0, 1, 1) if i == j else oracle.ZERO, None) for j in range(3)] for i in range(3)]
    C = oracle.mat_mul(A, I, 300)
    for i in range(3):
        for j in range(3):
            m, r = A[i][j]
            if m[1]:
                # the midpoint survives to 300 bits, radius is the input radius plus rounding
                assert abs(fr(C[i][j].mid) - fr(m)) <= Fraction(2) ** (m[2] - 300)
                assert rfr(C[i][j].rad) <= rfr(r) + Fraction(2) ** (m[2] - 300)
    C2 = oracle.mat_mul(A, A, 200)
    # (3,3) entry = 2*3.45 + (4.56e-100)^2: tiny entries keep relative accuracy
    m33 = fr(C2[2][2].mid)
    assert abs(m33 - Fraction(69, 10)) < Fraction(1, 10 ** 40)
    assert rfr(C2[2][2].rad) < Fraction(1, 10 ** 40)
    # (2,3) entry = 2.34*3.45 + 3.45*4.56e-100: radius reflects 1e-20 and 1e-50 inputs
    assert rfr(C2[1][2].rad) < Fraction(1, 10 ** 19)


# ------------------------------------------------- approx variants (Section 3)


@settings(max_examples=150, deadline=None)
@given(st.lists(st.tuples(balls, balls), min_size=0, max_size=8),
       st.integers(2, 140), st.booleans(), st.one_of(st.none(), balls))
def test_approx_dot_is_the_truncated_sum_without_radius(pairs, p, sub, initial):
    # the approx variants return only a midpoint: the same truncation of the
    # exact sum (checked against Fraction arithmetic and mpmath's round-down,
    # independently of the full call), no radius, and the same inexact flag
    x = [a for a, _ in pairs]
    y = [b for _, b in pairs]
    res = oracle.dot(x, y, p, initial=initial, sub=sub, approx=True)
    S = sum((fr(a[0]) * fr(b[0]) for a, b in pairs), Fraction(0))
    if sub:
        S = -S
    if initial is not None:
        S += fr(initial[0])
    want = trunc_fraction(S, p)
    assert res.rad is None
    assert fr(res.mid) == want
    assert res.inexact == (want != S)
    full = oracle.dot(x, y, p, initial=initial, sub=sub)
    assert res.mid == full.mid and res.inexact == full.inexact


@pytest.mark.parametrize("seed", range(4))
def test_approx_cdot_against_fraction_definition(seed):
    rng = random.Random(500 + seed)
    n = 10
    x = [(b1, b2) for b1, b2 in zip(_rand_balls(rng, n), _rand_balls(rng, n))]
    y = [(b1, b2) for b1, b2 in zip(_rand_balls(rng, n), _rand_balls(rng, n))]
    re, im = oracle.cdot(x, y, 61, approx=True)
    Sre = sum((fr(a[0]) * fr(c[0]) - fr(b[0]) * fr(d[0]) for (a, b), (c, d) in zip(x, y)), Fraction(0))
    Sim = sum((fr(a[0]) * fr(d[0]) + fr(b[0]) * fr(c[0]) for (a, b), (c, d) in zip(x, y)), Fraction(0))
    assert re.rad is None and im.rad is None
    assert fr(re.mid) == trunc_fraction(Sre, 61) and re.inexact == (fr(re.mid) != Sre)
    assert fr(im.mid) == trunc_fraction(Sim, 61) and im.inexact == (fr(im.mid) != Sim)
    fre, fim = oracle.cdot(x, y, 61)
    assert (re.mid, re.inexact) == (fre.mid, fre.inexact)
    assert (im.mid, im.inexact) == (fim.mid, fim.inexact)


# ------------------------------------------- complex matrix product (Section 4.3)


def _rand_cmat(rng, rows, cols, bits=90, erange=25):
    return [[(b1, b2) for b1, b2 in zip(_rand_balls(rng, cols, bits, erange), _rand_balls(rng, cols, bits, erange))]
            for _ in range(rows)]


@pytest.mark.parametrize("seed", range(3))
def test_cmat_mul_against_fraction_definition(seed):
    # C_ij = sum_k (a + b i)(c + d i) over exact rationals, each part
    # truncated once toward zero (mpmath round-down), with the enclosure
    # radius of Section 2 summed over the part's 2N real products
    rng = random.Random(600 + seed)
    M, N, K, p = 3, 7, 4, 70
    A, B = _rand_cmat(rng, M, N), _rand_cmat(rng, N, K)
    C = oracle.cmat_mul(A, B, p)
    for i in range(M):
        for j in range(K):
            terms = [(A[i][k], B[k][j]) for k in range(N)]
            Sre = sum((fr(a[0]) * fr(c[0]) - fr(b[0]) * fr(d[0]) for (a, b), (c, d) in terms), Fraction(0))
            Sim = sum((fr(a[0]) * fr(d[0]) + fr(b[0]) * fr(c[0]) for (a, b), (c, d) in terms), Fraction(0))

            def prad(u, v):
                return abs(fr(u[0])) * rfr(v[1]) + abs(fr(v[0])) * rfr(u[1]) + rfr(u[1]) * rfr(v[1])

            rho_re = sum((prad(a, c) + prad(b, d) for (a, b), (c, d) in terms), Fraction(0))
            rho_im = sum((prad(a, d) + prad(b, c) for (a, b), (c, d) in terms), Fraction(0))
            re, im = C[i][j]
            for part, S, rho in ((re, Sre, rho_re), (im, Sim, rho_im)):
                m = fr(part.mid)
                assert m == trunc_fraction(S, p)
                assert part.inexact == (m != S)
                if part.inexact:
                    rho += Fraction(2) ** (part.mid[2] - p)
                assert rfr(part.rad) == rho
                assert abs(S - m) <= rfr(part.rad)


@pytest.mark.parametrize("seed", range(2))
def test_cmat_mul_with_zero_imaginary_parts_is_mat_mul(seed):
    rng = random.Random(700 + seed)
    M, N, K, p = 4, 6, 3, 55
    A = [_rand_balls(rng, N) for _ in range(M)]
    B = [_rand_balls(rng, K) for _ in range(N)]
    z = (oracle.ZERO, None)
    C = oracle.cmat_mul([[(a, z) for a in row] for row in A], [[(b, z) for b in row] for row in B], p)
    R = oracle.mat_mul(A, B, p)
    for i in range(M):
        for j in range(K):
            re, im = C[i][j]
            assert re == R[i][j]
            assert im.mid == oracle.ZERO and im.rad == (0, 0) and not im.inexact


@pytest.mark.parametrize("approx", [False, True])
def test_cmat_mul_entry_is_cdot_of_row_and_column(approx):
    rng = random.Random(800 + approx)
    M, N, K = 2, 5, 3
    A, B = _rand_cmat(rng, M, N), _rand_cmat(rng, N, K)
    C = oracle.cmat_mul(A, B, 40, approx=approx)
    R = oracle.mat_mul([[a for a, _ in row] for row in A], [[b for b, _ in row] for row in B], 40, approx=approx)
    for i in range(M):
        for j in range(K):
            assert C[i][j] == oracle.cdot(A[i], [B[k][j] for k in range(N)], 40, approx=approx)
            assert R[i][j] == oracle.dot([a for a, _ in A[i]], [B[k][j][0] for k in range(N)], 40,
                                         approx=approx)
            if approx:
                assert C[i][j][0].rad is None and R[i][j].rad is None
