"""Comparison of library outputs with oracle results (test helper)."""

from fractions import Fraction

TIGHT = Fraction(1, 2**20)


def dyadic_cmp_le(a, b):
    """a <= b for exact dyadic pairs (N, E)."""
    (na, ea), (nb, eb) = a, b
    e = min(ea, eb)
    return (na << (ea - e)) <= (nb << (eb - e))


def compare_entry(got, want, status=None, approx=False):
    """got: canonical ball decoded from the device output; want: oracle
    DotResult.  Returns None when they agree: identical midpoint, and a
    radius r with R <= r <= (1 + 2^-20) R for the oracle's exact bound R."""
    mid, rad = got
    if status is not None and status not in (0, 1):
        return f"status {status}"
    if mid != want.mid:
        return f"midpoint {mid} != {want.mid}"
    if approx:
        return None
    R = want.rad if want.rad is not None else (0, 0)
    if R[0] == 0:
        if rad is not None and rad[0] != 0:
            return f"radius {rad} for an exact result"
        return None
    if rad is None:
        return f"radius 0, expected {R}"
    # R <= r
    if not dyadic_cmp_le(R, rad):
        return f"radius {rad} below the bound {R}"
    # r <= R (1 + 2^-20)  <=>  r * 2^20 <= R * (2^20 + 1)
    if not dyadic_cmp_le((rad[0] << 20, rad[1]), (R[0] * (2**20 + 1), R[1])):
        return f"radius {rad} looser than (1+2^-20) * {R}"
    return None
