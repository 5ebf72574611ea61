"""Exact rational evaluation of the PP force (eq. 4d with eq. 2) for small
particle sets.  TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

The PP term sums m_p [R(r, b_pp) - R(r, b_f)] D / r over pairs closer than
b_f.  Near the cutoff R(r, b_pp) = 1/r^2 and R(r, b_f) -> 1/r^2, so the
difference cancels: evaluated in FP64 as printed it keeps only a few digits
for r within a few percent of b_f.  Here every quantity is a Python
``Fraction``: the separations D are exact (integer positions in units of
2^-15 fine cells), eq. (2) is evaluated in rational arithmetic, and only the
square root is approximated (integer square root at 2^-140 relative).  The
per-particle sums are rounded to FP64 once.  Cost is O(N^2) candidate tests
plus a rational evaluation per pair in range: meant for a few thousand
particles.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr

import numpy as np


def inner(t: Fr) -> Fr:
    """b^2 R(r, b) on 0 <= t = r/b < 1/2 (eq. 2, first branch)."""
    return (Fr(64, 5) * t - Fr(256, 5) * t ** 3 + 32 * t ** 4 + Fr(1536, 35) * t ** 5
            - Fr(192, 5) * t ** 6)


def outer(t: Fr) -> Fr:
    """b^2 R(r, b) on 1/2 <= t < 1 (eq. 2, second branch)."""
    return (Fr(3, 35) / (t * t) - Fr(32, 5) + Fr(256, 5) * t - 96 * t ** 2 + Fr(256, 5) * t ** 3
            + 32 * t ** 4 - Fr(1536, 35) * t ** 5 + Fr(64, 5) * t ** 6)


def refforce(r: Fr, b: Fr) -> Fr:
    """R(r, b) of eq. (2), exactly."""
    if r >= b:
        return 1 / (r * r)
    t = r / b
    return (inner(t) if 2 * r < b else outer(t)) / (b * b)


def sqrt_units(n2: int, bits: int = 140) -> Fr:
    """sqrt(n2) * 2^-15 for an integer n2 (a squared separation in units of
    2^-30 fine cells^2), truncated to 2^-bits relative: isqrt of n2 4^bits."""
    return Fr(math.isqrt(n2 << (2 * bits)), 1 << (bits + 15))


def pair_g(n2: int, b_pp: Fr, b_f: Fr) -> Fr:
    """g(r) = [R(r, b_pp) - R(r, b_f)] / r at r^2 = n2 2^-30 (0 beyond b_f)."""
    if Fr(n2, 1 << 30) >= b_f * b_f:
        return Fr(0)
    r = sqrt_units(n2)
    return (refforce(r, b_pp) - refforce(r, b_f)) / r


def pp_accel(q: np.ndarray, n_fine: int, b_pp: float, b_f: float) -> np.ndarray:
    """acc_i = sum_{j != i, r < b_f} g(r_ij) D_ij (units: G m_p = 1, fine
    cells) for integer positions q (int64, (3, N), units of 2^-15 fine
    cells), with the exact minimum-image separation."""
    q = np.asarray(q, dtype=np.int64)
    N = q.shape[1]
    L = int(n_fine) << 15
    bpp, bf = Fr(b_pp).limit_denominator(10 ** 12), Fr(b_f).limit_denominator(10 ** 12)
    cut2 = float(bf) ** 2 * (1 + 1e-9) * float(1 << 30)   # squared cutoff in (2^-15)^2 units
    acc = np.zeros((3, N))
    for i in range(N):
        d = q - q[:, i:i + 1]
        d = (d + L // 2) % L - L // 2
        d2 = (d.astype(np.float64) ** 2).sum(axis=0)
        js = np.nonzero((d2 < cut2) & (d2 > 0))[0]
        s = [Fr(0), Fr(0), Fr(0)]
        for j in js:
            dj = [int(d[k, j]) for k in range(3)]
            g = pair_g(dj[0] * dj[0] + dj[1] * dj[1] + dj[2] * dj[2], bpp, bf)
            if g:
                for k in range(3):
                    s[k] += g * Fr(dj[k], 1 << 15)
        for k in range(3):
            acc[k, i] = float(s[k])
    return acc
