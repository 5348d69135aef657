"""Exact CPU oracle for arbitrary-precision ball dot products and matrix
products (Johansson, "Faster arbitrary-precision dot product and matrix
multiplication", 2019).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the GPU
library and imports nothing from it.

Every result is the plain definition written out with Python integers:
the exact sum is formed over a common power-of-two denominator and then
truncated toward zero to p bits.  Nothing here is blocked, windowed or
reordered beyond what that definition needs.
"""

from .arb import (  # noqa: F401
    ZERO,
    fmake,
    fvalue,
    fneg,
    fv2,
    fexp,
    fprec,
    rmake,
    rvalue,
    truncate,
    dot,
    cdot,
    mat_mul,
    cmat_mul,
    block_scalings,
    block_product,
    height_bound,
    extract_blocks,
    reduced_precision,
)
