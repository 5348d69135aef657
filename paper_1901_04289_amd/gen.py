"""Seeded synthetic operands for the dot/matmul workloads.

This module only *draws inputs*: random limbs, exponents, signs and radii
in the limb-plane format, and decodes that format into plain integers.  It
contains none of the dot-product or matrix-product arithmetic, so the GPU
path and the exact oracle can both take their inputs from here without
sharing any of the method.

Format of an operand array (host side, numpy):

* ``limbs``  uint32 ``[cap, count]``: plane-major, plane 0 is the most
  significant limb, value = (-1)**sign * sum_k limbs[k, i] * 2**(exp - 32(k+1))
  (eq. (1) with 32-bit limbs; the top limb has its top bit set).
* ``exp``    int32 ``[count]``: 2**(exp-1) <= |m| < 2**exp.
* ``nls``    int32 ``[count]``: limb count n in bits 0..30 (0 = zero),
  sign in bit 31.
* ``rad_m``  float64 ``[count]`` in [0.5, 1) or 0, ``rad_e`` int32: radius
  rad_m * 2**rad_e; both ``None`` for exact operands.

A mantissa of precision P has its top and bottom bits set and the P-2 bits
between them uniformly random, so its precision is exactly P.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 1901042890
SIGN_BIT = np.int32(-2**31)


@dataclasses.dataclass
class Operands:
    limbs: np.ndarray            # uint32 [cap, count]
    exp: np.ndarray              # int32 [count]
    nls: np.ndarray              # int32 [count]
    rad_m: Optional[np.ndarray]  # float64 [count] or None
    rad_e: Optional[np.ndarray]  # int32 [count] or None

    @property
    def count(self) -> int:
        return int(self.exp.shape[0])

    @property
    def cap(self) -> int:
        return int(self.limbs.shape[0])


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + config + 1000 * salt))


def _draw_mantissas(rng: np.random.Generator, prec: np.ndarray, cap: int) -> np.ndarray:
    """Limb planes of top-aligned mantissas with exact precision ``prec``."""
    count = prec.shape[0]
    n = (prec + 31) // 32
    limbs = rng.integers(0, 2**32, size=(cap, count), dtype=np.uint64).astype(np.uint32)
    k = np.arange(cap, dtype=np.int64)[:, None]
    limbs[k >= n[None, :]] = 0
    # lowest used bit of the last limb: bit position (32n - prec) from the bottom
    low = (32 * n - prec).astype(np.uint64)
    last = n - 1
    cols = np.arange(count)
    lastv = limbs[last, cols].astype(np.uint64)
    lastv = (lastv >> low) << low
    lastv |= (np.uint64(1) << low)
    limbs[last, cols] = lastv.astype(np.uint32)
    limbs[0, :] |= np.uint32(0x80000000)
    return limbs


def _round_up_radius(limbs: np.ndarray, exp: np.ndarray, shift: np.ndarray):
    """Radius RU53(2**-shift * |m|): the magnitude rounded up to 53 bits
    and scaled by 2**-shift, returned as (rad_m in [0.5,1), rad_e)."""
    top = (limbs[0].astype(np.uint64) << np.uint64(32))
    if limbs.shape[0] > 1:
        top |= limbs[1].astype(np.uint64)
    rem = (top & np.uint64(0x7FF)) != 0
    if limbs.shape[0] > 2:
        rem |= np.any(limbs[2:] != 0, axis=0)
    mant = (top >> np.uint64(11)) + rem.astype(np.uint64)   # <= 2**53, exact
    m, ex = np.frexp(mant.astype(np.float64))
    rad_e = (ex.astype(np.int64) + exp.astype(np.int64) - 53 - shift.astype(np.int64))
    return m, rad_e.astype(np.int32)


def random_operands(rng: np.random.Generator, count: int, prec, exp_lo: int, exp_hi: int,
                    cap: Optional[int] = None, radius_shift=None,
                    zero_frac: float = 0.0) -> Operands:
    """``count`` operands of precision ``prec`` (int or array), exponents
    uniform in [exp_lo, exp_hi], random signs.  ``radius_shift`` (int or
    array) gives radii RU53(2**-shift |m|); None gives exact operands."""
    prec = np.broadcast_to(np.asarray(prec, dtype=np.int64), (count,)).copy()
    if np.any(prec < 1):
        raise ValueError("precision must be >= 1")
    n = (prec + 31) // 32
    if cap is None:
        cap = int(n.max()) if count else 1
    if np.any(n > cap):
        raise ValueError("cap too small for the requested precision")
    limbs = _draw_mantissas(rng, prec, cap)
    exp = rng.integers(exp_lo, exp_hi + 1, size=count).astype(np.int32)
    sign = rng.integers(0, 2, size=count).astype(np.int32)
    nls = n.astype(np.int32) | (sign << 31).astype(np.int32)
    if zero_frac > 0:
        z = rng.random(count) < zero_frac
        limbs[:, z] = 0
        exp[z] = 0
        nls[z] = 0
    rad_m = rad_e = None
    if radius_shift is not None:
        sh = np.broadcast_to(np.asarray(radius_shift, dtype=np.int64), (count,))
        rad_m, rad_e = _round_up_radius(limbs, exp, sh)
        if zero_frac > 0:
            rad_m[z] = 0.0
            rad_e[z] = 0
    return Operands(limbs, exp, nls, rad_m, rad_e)


def from_canonical(balls: Sequence, cap: Optional[int] = None) -> Operands:
    """Pack canonical balls ((s, M, e), rad) into the limb-plane format.
    ``rad`` is None (exact) or (R, g) with R < 2**53."""
    count = len(balls)
    ns = []
    for (s, M, e), _ in balls:
        ns.append(0 if M == 0 else (M.bit_length() + 31) // 32)
    if cap is None:
        cap = max(ns + [1])
    limbs = np.zeros((cap, count), dtype=np.uint32)
    exp = np.zeros(count, dtype=np.int32)
    nls = np.zeros(count, dtype=np.int32)
    have_rad = any(r is not None for _, r in balls)
    rad_m = np.zeros(count, dtype=np.float64) if have_rad else None
    rad_e = np.zeros(count, dtype=np.int32) if have_rad else None
    for i, ((s, M, e), r) in enumerate(balls):
        n = ns[i]
        if n > cap:
            raise ValueError("cap too small")
        if M:
            full = M << (32 * n - M.bit_length())
            for k in range(n):
                limbs[k, i] = (full >> (32 * (n - 1 - k))) & 0xFFFFFFFF
            exp[i] = e
            nls[i] = (n - 2**31) if s else n
        if r is not None and r[0] != 0:
            R, g = r
            if R.bit_length() > 53:
                raise ValueError("radius mantissa wider than 53 bits")
            m, ex = math.frexp(float(R))
            rad_m[i] = m
            rad_e[i] = ex + g
    return Operands(limbs, exp, nls, rad_m, rad_e)


def to_canonical(ops: Operands, i: int):
    """Decode operand i into a canonical ball ((s, M, e), rad_or_None)."""
    nl = int(ops.nls[i])
    n = nl & 0x7FFFFFFF
    s = 1 if nl < 0 else 0
    if n == 0:
        mid = (0, 0, 0)
    else:
        M = 0
        for k in range(n):
            M = (M << 32) | int(ops.limbs[k, i])
        if M == 0:
            mid = (0, 0, 0)
        else:
            e = int(ops.exp[i]) - 32 * n + M.bit_length()
            t = (M & -M).bit_length() - 1
            mid = (s, M >> t, e)
    rad = None
    if ops.rad_m is not None and ops.rad_m[i] != 0.0:
        num, den = float(ops.rad_m[i]).as_integer_ratio()
        g = int(ops.rad_e[i]) - (den.bit_length() - 1)
        t = (num & -num).bit_length() - 1
        rad = (num >> t, g + t)
    return mid, rad


def canonical_matrix(ops: Operands, rows: int, cols: int, rs: int, cs: int, off: int = 0):
    return [[to_canonical(ops, off + i * rs + j * cs) for j in range(cols)] for i in range(rows)]


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class MatmulWorkload:
    name: str
    M: int
    N: int   # inner dimension
    K: int
    p: int
    A: Operands   # row-major M x N
    B: Operands   # row-major N x K
    Ai: Optional[Operands] = None   # imaginary parts (complex workloads)
    Bi: Optional[Operands] = None


def config0(seed_salt: int = 0) -> MatmulWorkload:
    """64x64 by 64x64, p = 128, 128-bit mantissas, exponents in [-8, 8], exact."""
    rng = rng_for(0, seed_salt)
    A = random_operands(rng, 64 * 64, 128, -8, 8)
    B = random_operands(rng, 64 * 64, 128, -8, 8)
    return MatmulWorkload("real matmul 64x64x64 p=128 exact", 64, 64, 64, 128, A, B)


def config1(seed_salt: int = 0, n: int = 512) -> MatmulWorkload:
    """N = 512 ball matmul, p = 256, 256-bit mantissas, exponents in [-32, 32],
    radii RU53(2**-250 |m|)."""
    rng = rng_for(1, seed_salt)
    A = random_operands(rng, n * n, 256, -32, 32, radius_shift=250)
    B = random_operands(rng, n * n, 256, -32, 32, radius_shift=250)
    return MatmulWorkload(f"real ball matmul {n}x{n}x{n} p=256", n, n, n, 256, A, B)


def config2(seed_salt: int = 0, n: int = 2048) -> MatmulWorkload:
    """N = 2048 matmul, p = 512, 512-bit mantissas, exponents in [-4, 4], exact."""
    rng = rng_for(2, seed_salt)
    A = random_operands(rng, n * n, 512, -4, 4)
    B = random_operands(rng, n * n, 512, -4, 4)
    return MatmulWorkload(f"real matmul {n}x{n}x{n} p=512 exact", n, n, n, 512, A, B)


@dataclasses.dataclass
class DotBatch:
    lengths: np.ndarray      # int64 [ndots]
    precs: np.ndarray        # int64 [ndots] output precision p
    offsets: np.ndarray      # int64 [ndots] start index of each dot's operands
    x_re: Operands
    x_im: Operands
    y_re: Operands
    y_im: Operands


def config3(seed_salt: int = 0, ndots: int = 10000, max_len: int = 4096) -> DotBatch:
    """Batched complex ball dots: lengths log-uniform in [4, max_len], p
    log-uniform in [64, 1024], each real component of each operand at its
    own precision uniform in [ceil(p/2), 2p], exponents in [-16, 16], radii
    RU53(2**-prec |m|)."""
    rng = rng_for(3, seed_salt)
    lengths = np.floor(np.exp(rng.uniform(np.log(4), np.log(max_len + 1), ndots))).astype(np.int64)
    lengths = np.clip(lengths, 4, max_len)
    precs = np.floor(np.exp(rng.uniform(np.log(64), np.log(1025), ndots))).astype(np.int64)
    precs = np.clip(precs, 64, 1024)
    offsets = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    total = int(lengths.sum())
    p_of_term = np.repeat(precs, lengths)
    comps = []
    for _ in range(4):
        lo = (p_of_term + 1) // 2
        hi = 2 * p_of_term
        pr = rng.integers(lo, hi + 1)
        comps.append(random_operands(rng, total, pr, -16, 16, cap=64, radius_shift=pr))
    return DotBatch(lengths, precs, offsets, *comps)


@dataclasses.dataclass
class Request:
    arrival_s: float
    n: int
    p: int


def config4_requests(seed_salt: int = 0, count: int = 10000, rate: float = 200.0) -> List[Request]:
    """Poisson stream (rate per second) of square complex ball matmul
    requests, N log-uniform in [16, 1024], p uniform over
    {128, 256, 512, 1024, 2048}."""
    rng = rng_for(4, seed_salt)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    ns = np.floor(np.exp(rng.uniform(np.log(16), np.log(1025), count))).astype(np.int64)
    ns = np.clip(ns, 16, 1024)
    ps = rng.choice(np.array([128, 256, 512, 1024, 2048]), count)
    return [Request(float(a), int(n), int(p)) for a, n, p in zip(t, ns, ps)]


def config4_operands(rng: np.random.Generator, n: int, p: int):
    """Operands of one serving request: four n x n parts (A re/im, B re/im),
    precision p, exponents in [-8, 8], radii RU53(2**-p |m|)."""
    cap = (p + 31) // 32
    return [random_operands(rng, n * n, p, -8, 8, cap=cap, radius_shift=p) for _ in range(4)]
