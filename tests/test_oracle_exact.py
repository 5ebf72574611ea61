"""Pins of the exact rational PP evaluator (oracle/exact.py).

It is checked against what eq. (2) fixes exactly (continuity of the force
law at b/2 and b, its linear small-r limit), against the enclosed-mass
integral of the profile pair (through the FP64 oracle, which is pinned to
that integral), and against the FP64 oracle's PP sum where the latter does
not cancel; the stored exact fixtures are checked to be current.
"""
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import synthetic
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_force_law_continuous_at_the_breakpoints():
    # both branches of eq. (2) meet at t = 1/2, and the outer one meets the
    # Newtonian law 1/r^2 at t = 1 (b^2 R = 1/t^2 = 1), exactly
    assert exact.inner(Fr(1, 2)) == exact.outer(Fr(1, 2))
    assert exact.outer(Fr(1)) == 1
    # first derivatives as well (difference quotients of exact polynomials)
    h = Fr(1, 10 ** 30)
    d_in = (exact.inner(Fr(1, 2)) - exact.inner(Fr(1, 2) - h)) / h
    d_out = (exact.outer(Fr(1, 2) + h) - exact.outer(Fr(1, 2))) / h
    assert abs(d_in - d_out) < Fr(1, 10 ** 25)
    d_out1 = (exact.outer(Fr(1)) - exact.outer(1 - h)) / h
    assert abs(d_out1 - (-2)) < Fr(1, 10 ** 25)       # d/dt t^-2 at t = 1


def test_small_r_limit_is_linear():
    # the force between two overlapping profiles grows linearly from r = 0
    t = Fr(1, 10 ** 12)
    assert abs(exact.inner(t) / t - Fr(64, 5)) < Fr(1, 10 ** 20)


@pytest.mark.parametrize("b", [Fr(1, 5), Fr(2), Fr(14)])
def test_matches_fp64_oracle_force_law(b):
    for t in (0.013, 0.2, 0.49, 0.5, 0.61, 0.9, 0.999, 1.5):
        r = Fr(t) * b
        R = float(exact.refforce(r, b))
        assert R == pytest.approx(oracle.refforce(float(r), float(b)), rel=1e-13)


def test_square_root_units():
    for n2 in (1, 2, 3, 1 << 30, 123456789):
        r = exact.sqrt_units(n2)
        assert 0 <= Fr(n2, 1 << 30) - r * r < Fr(1, 10 ** 35) * Fr(n2, 1 << 30) + Fr(1, 10 ** 60)


def test_pp_sum_matches_fp64_oracle_and_conserves_momentum():
    x = synthetic.zeldovich(13, 0.25, 103)
    q = oracle.quantize(x, 32)
    a = exact.pp_accel(q, 32, 0.2, 2.0)
    ref = oracle.Oracle(oracle.Params(n_fine=32)).pp_accel(oracle.q_to_fine(q))
    # the FP64 sum differs only through its cancellation near the cutoff
    assert np.linalg.norm(a - ref) <= 1e-9 * np.linalg.norm(a)
    assert np.linalg.norm(a.sum(axis=1)) <= 1e-14 * np.abs(a).sum()


def test_golden_fixture_is_current():
    x = synthetic.zeldovich(13, 0.25, 103)
    a = exact.pp_accel(oracle.quantize(x, 32), 32, 0.2, 2.0)
    g = np.loadtxt(os.path.join(GOLDEN, "pp_exact_zel_32_ragged.txt")).T
    assert np.array_equal(a, g)
