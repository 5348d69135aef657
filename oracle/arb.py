"""Exact reference semantics (test infrastructure only; see the package
docstring).

Representations (all plain Python integers, no floating point anywhere):

* A *float* is a tuple ``(s, M, e)`` with sign bit ``s``, integer
  mantissa ``M >= 0`` and exponent ``e``; its value is
  ``(-1)**s * M * 2**(e - bitlen(M))`` so that ``2**(e-1) <= |x| < 2**e``
  for ``M > 0``.  This is the midpoint format of Section 3.1, eq. (1), with
  the limb split left out.  Zero is ``ZERO = (0, 0, 0)``.  Canonical floats
  have an odd mantissa (trailing zero bits stripped), so equal values have
  equal tuples.
* A *radius* is a tuple ``(R, g)`` with ``R >= 0``, value ``R * 2**g``
  (an exact dyadic number).  ``None`` means an exact ball (radius 0).
* A *ball* is ``(mid, rad)``; a rectangular complex ball is
  ``(re_ball, im_ball)`` (Section 3.6).

Parity unpinned: nothing.  Every public function is pinned by the CPU
tests in ``tests/test_oracle_*.py`` (brute-force rational sums, a library
rounding routine, closed forms, invariants, and the block counts printed in
Table 3).
"""

from __future__ import annotations

from fractions import Fraction
from typing import List, NamedTuple, Optional, Sequence, Tuple

ZERO = (0, 0, 0)


# ---------------------------------------------------------------------------
# Floats and radii
# ---------------------------------------------------------------------------

def _ctz(n: int) -> int:
    """Number of trailing zero bits of a positive integer."""
    return (n & -n).bit_length() - 1


def fmake(sign: int, M: int, e: int):
    """Canonical float of value (-1)**sign * M * 2**(e - bitlen(M))."""
    if M < 0:
        raise ValueError("mantissa must be non-negative")
    if M == 0:
        return ZERO
    t = _ctz(M)
    return (1 if sign else 0, M >> t, e)


def fvalue(x) -> Tuple[int, int]:
    """Exact value of a float as (N, E) meaning N * 2**E."""
    s, M, e = x
    if M == 0:
        return 0, 0
    return (-M if s else M), e - M.bit_length()


def fneg(x):
    s, M, e = x
    if M == 0:
        return ZERO
    return (1 - s, M, e)


def fexp(x) -> int:
    """Exponent e with 2**(e-1) <= |x| < 2**e (eq. (1))."""
    return x[2]


def fv2(x) -> int:
    """2-adic valuation of a nonzero float: the position of its lowest set bit."""
    s, M, e = x
    if M == 0:
        raise ValueError("v2 of zero")
    return e - M.bit_length() + _ctz(M)


def fprec(x) -> int:
    """Number of significant bits (0 for zero)."""
    M = x[1]
    if M == 0:
        return 0
    return (M >> _ctz(M)).bit_length()


def rmake(R: int, g: int):
    if R < 0:
        raise ValueError("radius must be non-negative")
    if R == 0:
        return (0, 0)
    t = _ctz(R)
    return (R >> t, g + t)


def rvalue(r) -> Tuple[int, int]:
    if r is None:
        return 0, 0
    return r


def _dy_add(a: Tuple[int, int], b: Tuple[int, int]) -> Tuple[int, int]:
    """Exact sum of two dyadic numbers (N, E)."""
    (na, ea), (nb, eb) = a, b
    if na == 0:
        return b
    if nb == 0:
        return a
    if ea <= eb:
        return na + (nb << (eb - ea)), ea
    return (na << (ea - eb)) + nb, eb


def _dy_mul(a: Tuple[int, int], b: Tuple[int, int]) -> Tuple[int, int]:
    return a[0] * b[0], a[1] + b[1]


def _dy_abs(a: Tuple[int, int]) -> Tuple[int, int]:
    return abs(a[0]), a[1]


def _dy_sum(items) -> Tuple[int, int]:
    """Exact sum of dyadic numbers, formed over the common denominator
    2**E_min (the lowest exponent present) as a single integer."""
    items = [it for it in items if it[0] != 0]
    if not items:
        return 0, 0
    emin = min(E for _, E in items)
    total = 0
    for N, E in items:
        total += N << (E - emin)
    return total, emin


# ---------------------------------------------------------------------------
# Truncation to p bits (the defined rounding of the output midpoint)
# ---------------------------------------------------------------------------

def truncate(N: int, E: int, p: int):
    """Round N * 2**E to p significant bits toward zero.

    Returns ``(float, inexact)``.  Algorithm 1 (finalization, step 2) rounds
    the accumulator to p bits without naming the mode; the reading used
    throughout is truncation of the magnitude, which never changes the
    binade and commutes with negation.
    """
    if p < 2:
        raise ValueError("p must be >= 2")
    if N == 0:
        return ZERO, False
    s = 1 if N < 0 else 0
    A = -N if s else N
    b = A.bit_length()
    if b <= p:
        return fmake(s, A, E + b), False
    drop = b - p
    M = A >> drop
    inexact = (A & ((1 << drop) - 1)) != 0
    return fmake(s, M, E + b), inexact


# ---------------------------------------------------------------------------
# Dot products (Section 2, Section 3, Algorithm 1)
# ---------------------------------------------------------------------------

class DotResult(NamedTuple):
    mid: tuple                       # canonical float
    rad: Optional[Tuple[int, int]]   # exact dyadic (R, g); None for approx
    inexact: bool                    # midpoint differs from the exact sum


def _ball_mid(b):
    return b[0]


def _ball_rad(b) -> Tuple[int, int]:
    return rvalue(b[1])


def _prod_rad(u, v) -> Tuple[int, int]:
    """Propagated radius of a ball product: |m_u| r_v + |m_v| r_u + r_u r_v
    (Section 2, the bound on r)."""
    mu, mv = _dy_abs(fvalue(u[0])), _dy_abs(fvalue(v[0]))
    ru, rv = _ball_rad(u), _ball_rad(v)
    return _dy_sum([_dy_mul(mu, rv), _dy_mul(mv, ru), _dy_mul(ru, rv)])


def _exponent_of_radius(r) -> Optional[int]:
    R, g = r
    if R == 0:
        return None
    return g + R.bit_length()


def reduced_precision(products, p: int, initial=None) -> int:
    """Radius-driven precision cut of the setup pass (Section 3.3, step 7(a)
    with 7(c)): p' = max(2, min(p, e_max - e_rad + 30)), where e_max bounds
    the exponents of the midpoint products and e_rad those of the radius
    products (factor exponents added).  ``products`` is a list of
    (sign, u_ball, v_ball).  The initial term counts as the product
    initial * 1.  Only used when the caller asks for the cut."""
    P_RAD = 30
    e_max = None
    e_rad = None

    def upd_max(cur, v):
        return v if cur is None else max(cur, v)

    items = [(u, v) for _, u, v in products]
    one = ((0, 1, 1), None)
    if initial is not None:
        items.append((initial, one))
    for u, v in items:
        mu, mv = u[0], v[0]
        if mu[1] != 0 and mv[1] != 0:
            e_max = upd_max(e_max, fexp(mu) + fexp(mv))
        ru, rv = _ball_rad(u), _ball_rad(v)
        fru, frv = _exponent_of_radius(ru), _exponent_of_radius(rv)
        if mu[1] != 0 and frv is not None:
            e_rad = upd_max(e_rad, fexp(mu) + frv)
        if mv[1] != 0 and fru is not None:
            e_rad = upd_max(e_rad, fexp(mv) + fru)
        if fru is not None and frv is not None:
            e_rad = upd_max(e_rad, fru + frv)
    if e_max is None:
        return 2
    q = p
    if e_rad is not None:
        q = min(q, e_max - e_rad + P_RAD)
    return max(q, 2)


def _real_dot(products, p: int, initial=None, sub: bool = False,
              approx: bool = False, reduce_prec: bool = False) -> DotResult:
    """Core real dot: ``products`` is a list of (sign, u_ball, v_ball) whose
    terms are (-1)**sign * u * v.  Computes initial + (-1)**sub * sum."""
    if p < 2:
        raise ValueError("p must be >= 2")
    terms = []
    for sg, u, v in products:
        N, E = _dy_mul(fvalue(u[0]), fvalue(v[0]))
        if sg:
            N = -N
        terms.append((N, E))
    S_N, S_E = _dy_sum(terms)
    if sub:
        S_N = -S_N
    if initial is not None:
        S_N, S_E = _dy_add((S_N, S_E), fvalue(initial[0]))
    q = reduced_precision(products, p, initial) if reduce_prec else p
    mid, inexact = truncate(S_N, S_E, q)
    if approx:
        return DotResult(mid, None, inexact)
    rads = [_prod_rad(u, v) for _, u, v in products]
    if initial is not None:
        rads.append(_ball_rad(initial))
    if inexact:
        rads.append((1, fexp(mid) - q))
    R, g = _dy_sum(rads)
    return DotResult(mid, rmake(R, g), inexact)


def dot(x: Sequence, y: Sequence, p: int, initial=None, sub: bool = False,
        approx: bool = False, reduce_prec: bool = False) -> DotResult:
    """Ball containing initial + (-1)**sub * sum_i x_i y_i (Section 3, the
    arb_dot problem statement; Section 2 for the enclosure).

    The midpoint is the exact sum truncated toward zero to p bits; the
    radius is the exact dyadic bound  [inexact] * 2**(e_m - p) + r_initial
    + sum_i (|m_i| r'_i + |m'_i| r_i + r_i r'_i).  With ``approx`` only the
    midpoint is returned (the approx variants ignore radii).  Strides are
    applied by the caller (``x``, ``y`` are already the N operands)."""
    if len(x) != len(y):
        raise ValueError("length mismatch")
    return _real_dot([(0, a, b) for a, b in zip(x, y)], p, initial, sub,
                     approx, reduce_prec)


def cdot(x: Sequence, y: Sequence, p: int, initial=None, sub: bool = False,
         approx: bool = False, reduce_prec: bool = False) -> Tuple[DotResult, DotResult]:
    """Complex dot over rectangular complex balls (Section 3.6): the real
    part is the real dot of the 2N terms a_i c_i and -(b_i d_i), the
    imaginary part that of a_i d_i and b_i c_i, each rounded once.  Each
    operand is ((a, ra), (b, rb)) = [a +- ra] + [b +- rb] i.  With
    ``reduce_prec`` each part takes the precision cut of its own 2N-term
    real dot (Section 3.3, step 7(a))."""
    if len(x) != len(y):
        raise ValueError("length mismatch")
    re_terms, im_terms = [], []
    for (a, b), (c, d) in zip(x, y):
        re_terms.append((0, a, c))
        re_terms.append((1, b, d))
        im_terms.append((0, a, d))
        im_terms.append((0, b, c))
    ire = initial[0] if initial is not None else None
    iim = initial[1] if initial is not None else None
    return (_real_dot(re_terms, p, ire, sub, approx, reduce_prec),
            _real_dot(im_terms, p, iim, sub, approx, reduce_prec))


# ---------------------------------------------------------------------------
# Matrix products (Section 4)
# ---------------------------------------------------------------------------

def mat_mul(A: Sequence[Sequence], B: Sequence[Sequence], p: int,
            approx: bool = False) -> List[List[DotResult]]:
    """Entrywise C_ij = dot(row i of A, column j of B, p): the classical
    product of M*K dot products of length N (Section 4).  Any blocking,
    scaling or splitting of the inner dimension must give exactly this
    (one rounding per entry)."""
    M, N = len(A), len(A[0]) if A else 0
    if len(B) != N:
        raise ValueError("inner dimension mismatch")
    K = len(B[0]) if B else 0
    cols = [[B[k][j] for k in range(N)] for j in range(K)]
    return [[dot(A[i], cols[j], p, approx=approx) for j in range(K)]
            for i in range(M)]


def cmat_mul(A, B, p: int, approx: bool = False):
    """Complex matrix product, entrywise cdot (Section 4.3 combines four
    real products exactly before the single rounding of each entry)."""
    M, N = len(A), len(A[0]) if A else 0
    if len(B) != N:
        raise ValueError("inner dimension mismatch")
    K = len(B[0]) if B else 0
    cols = [[B[k][j] for k in range(N)] for j in range(K)]
    return [[cdot(A[i], cols[j], p, approx=approx) for j in range(K)]
            for i in range(M)]


# ---------------------------------------------------------------------------
# Scaled integer blocks (Section 4.1, Algorithm 2)
# ---------------------------------------------------------------------------

def block_scalings(A_mid, B_mid, s: Sequence[int]):
    """Scaling exponents of a block (Section 4.1): e_i makes row i of
    2**e_i A_s an integer row of minimal height (some entry odd), f_j does
    the same for column j of B_s 2**f_j; all-zero rows/columns get 0.
    ``A_mid``/``B_mid`` are matrices of floats (midpoints)."""
    M = len(A_mid)
    K = len(B_mid[0]) if B_mid else 0
    e = []
    for i in range(M):
        v = [fv2(A_mid[i][k]) for k in s if A_mid[i][k][1] != 0]
        e.append(-min(v) if v else 0)
    f = []
    for j in range(K):
        v = [fv2(B_mid[k][j]) for k in s if B_mid[k][j][1] != 0]
        f.append(-min(v) if v else 0)
    return e, f


def _scaled_int(x, shift: int) -> int:
    """x * 2**shift as an exact integer (the caller guarantees it is one)."""
    N, E = fvalue(x)
    E += shift
    if N == 0:
        return 0
    if E >= 0:
        return N << E
    # must be exact
    if N % (1 << -E):
        raise ValueError("not an integer after scaling")
    return N >> -E if N >= 0 else -((-N) >> -E)


def block_product(A_mid, B_mid, s: Sequence[int]):
    """T = (E_s A_s)(B_s F_s) over the integers (Algorithm 2, the matrix
    product over Z), with its scalings.  Returns (e, f, T) where
    sum_{k in s} a_ik b_kj = T_ij * 2**(-e_i - f_j) exactly."""
    e, f = block_scalings(A_mid, B_mid, s)
    M = len(A_mid)
    K = len(B_mid[0]) if B_mid else 0
    As = [[_scaled_int(A_mid[i][k], e[i]) for k in s] for i in range(M)]
    Bs = [[_scaled_int(B_mid[k][j], f[j]) for j in range(K)] for k in s]
    T = [[sum(As[i][t] * Bs[t][j] for t in range(len(s))) for j in range(K)]
         for i in range(M)]
    return e, f, T


def height_bound(p: int, pA: int, pB: int) -> Fraction:
    """Height bound h = 1.25 min(p, max(p_A, p_B)) + 192 (Algorithm 2),
    kept exact."""
    return Fraction(5, 4) * min(p, max(pA, pB)) + 192


def extract_blocks(A_mid, B_mid, p: int, basecase: int = 30):
    """Greedy contiguous partition of the inner index set (Algorithm 2 and
    Section 4.1): starting from the lowest unused index, append indices in
    increasing order while every row of A_s and every column of B_s keeps
    integer height at most h bits (height of a row = highest exponent minus
    lowest set bit over its nonzero entries).  A block shorter than
    ``basecase`` indices is extended to min(basecase, remaining) indices and
    marked 'basecase' (it is evaluated with dot products).  Returns a list
    of (k0, k1, kind)."""
    M = len(A_mid)
    N = len(B_mid)
    K = len(B_mid[0]) if B_mid else 0
    pA = max((fprec(x) for row in A_mid for x in row), default=0)
    pB = max((fprec(x) for row in B_mid for x in row), default=0)
    h = height_bound(p, pA, pB)
    top = [[(fexp(x), fv2(x)) if x[1] else None for x in row] for row in A_mid]
    btop = [[(fexp(x), fv2(x)) if x[1] else None for x in row] for row in B_mid]
    out = []
    start = 0
    while start < N:
        rtop, rlow = [None] * M, [None] * M
        ctop, clow = [None] * K, [None] * K
        end = start
        while end < N:
            ok = True
            for i in range(M):
                tl = top[i][end]
                if tl is None:
                    continue
                t = tl[0] if rtop[i] is None else max(rtop[i], tl[0])
                lo = tl[1] if rlow[i] is None else min(rlow[i], tl[1])
                if t - lo > h:
                    ok = False
                    break
            if ok:
                for j in range(K):
                    tl = btop[end][j]
                    if tl is None:
                        continue
                    t = tl[0] if ctop[j] is None else max(ctop[j], tl[0])
                    lo = tl[1] if clow[j] is None else min(clow[j], tl[1])
                    if t - lo > h:
                        ok = False
                        break
            if not ok:
                break
            for i in range(M):
                tl = top[i][end]
                if tl is not None:
                    rtop[i] = tl[0] if rtop[i] is None else max(rtop[i], tl[0])
                    rlow[i] = tl[1] if rlow[i] is None else min(rlow[i], tl[1])
            for j in range(K):
                tl = btop[end][j]
                if tl is not None:
                    ctop[j] = tl[0] if ctop[j] is None else max(ctop[j], tl[0])
                    clow[j] = tl[1] if clow[j] is None else min(clow[j], tl[1])
            end += 1
        if end - start < basecase:
            end = start + min(basecase, N - start)
            out.append((start, end, "basecase"))
        else:
            out.append((start, end, "block"))
        start = end
    return out
