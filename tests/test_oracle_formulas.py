"""Pins of the oracle's closed forms against what the mathematics fixes.

Each test checks an oracle formula against something other than itself:
a numerical integral of the real-space profile, a textbook alias identity,
a continuum limit, or a symmetry.  A dropped term, a wrong sign or a swapped
argument in eqs. (1), (2), (9)-(13) fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle


B = [0.2, 1.0, 2.0, 3.5, 14.0]


@pytest.mark.parametrize("b", B)
def test_profile_unit_mass(b):
    # eq. (1) integrates to one particle mass.
    m, _ = integrate.quad(lambda r: 4 * math.pi * r * r * oracle.profile(r, b), 0, b / 2)
    assert abs(m - 1.0) < 1e-12


@pytest.mark.parametrize("b", [1.0, 2.0, 14.0])
@pytest.mark.parametrize("kb", [0.05, 0.5, 1.9, 2.1, 5.0, 17.0, 60.0])
def test_profile_k_is_fourier_transform(b, kb):
    # eq. (13) equals the 3D Fourier transform of eq. (1):
    # S(k) = int 4 pi r^2 S(r) sin(kr)/(kr) dr.  Both the series branch
    # (u = kb/2 < 1) and the closed form are covered.
    k = kb / b
    f = lambda r: 4 * math.pi * r * r * oracle.profile(r, b) * (
        math.sin(k * r) / (k * r) if k * r > 0 else 1.0)
    ref, _ = integrate.quad(f, 0, b / 2, limit=200, epsabs=1e-14, epsrel=1e-13)
    assert abs(oracle.profile_k(k, b) - ref) < 1e-11


def test_profile_k_infinite_softening_is_zero():
    assert oracle.profile_k(0.3, math.inf) == 0.0


def test_profile_k_series_matches_closed_form_at_switch():
    b = 2.0
    u = 1.0
    k = 2 * u / b
    closed = 12.0 / u ** 4 * (2 - 2 * math.cos(u) - u * math.sin(u))
    assert abs(oracle.profile_k(k * (1 - 1e-12), b) - closed) < 1e-12
    assert abs(oracle.profile_k(k, b) - closed) < 1e-12


def _enclosed_force(r, b):
    """Force of the autoconvolution S*S at radius r, from S(k) numerically:
    M(<r)/r^2 with M(<r) = (2/pi) int S(k)^2 (sin kr - kr cos kr)/k dk."""
    g = lambda k: oracle.profile_k(k, b) ** 2 * (math.sin(k * r) - k * r * math.cos(k * r)) / k
    kmax = 400.0 / b
    m, _ = integrate.quad(g, 0, kmax, limit=4000, epsabs=1e-13)
    return 2 / math.pi * m / r ** 2


@pytest.mark.parametrize("t", [0.1, 0.3, 0.5, 0.7, 0.9, 1.2])
def test_refforce_is_force_between_profiles(t):
    # eq. (2) is the force between two eq.(1) profiles (footnote: coefficients
    # dropped), i.e. the enclosed mass of S*S over r^2.
    b = 2.0
    r = t * b
    assert abs(oracle.refforce(r, b) - _enclosed_force(r, b)) < 2e-8 * max(1, 1 / r ** 2)


@pytest.mark.parametrize("b", B)
def test_refforce_newtonian_beyond_b_and_continuous(b):
    for r in (b, 1.5 * b, 10 * b):
        assert oracle.refforce(r, b) == pytest.approx(1 / r ** 2, rel=1e-15)
    # C^0..C^3 continuity at r = b/2 and r = b (finite-difference of the branches)
    for rc in (b / 2, b):
        h = 1e-6 * b
        lo, hi = oracle.refforce(rc - h, b), oracle.refforce(rc + h, b)
        assert abs(lo - hi) < 1e-5 / b ** 2
    assert oracle.refforce(0.0, b) == 0.0


@pytest.mark.parametrize("b", [0.2, 2.0, 14.0])
def test_refforce_derivative(b):
    for t in (0.05, 0.3, 0.49, 0.51, 0.8, 0.99, 1.01, 2.0):
        r = t * b
        h = 1e-6 * b
        fd = (oracle.refforce(r + h, b) - oracle.refforce(r - h, b)) / (2 * h)
        assert oracle.refforce_dr(r, b) == pytest.approx(fd, rel=1e-6, abs=1e-8 / b ** 3)


def test_pp_kernel_vanishes_smoothly_at_cutoff():
    # R_PP = R(b_pp) - R(b_f) -> 0 like (1 - r/b_f)^5 at r -> b_f.
    b_pp, b_f = 0.2, 2.0
    for eps in (1e-1, 1e-2):
        r = b_f * (1 - eps)
        g = oracle.pp_g(r, b_pp, b_f) * r
        assert abs(g) < 200 * eps ** 5 / b_f ** 2
    assert oracle.pp_g(b_f, b_pp, b_f) == 0.0
    assert oracle.pp_g(0.0, b_pp, b_f) == 0.0
    # g is R(b_pp) - R(b_f) over r
    r = 0.7
    assert oracle.pp_g(r, b_pp, b_f) == pytest.approx(
        (1 / r ** 2 - oracle.refforce(r, b_f)) / r, rel=1e-14)


def test_pp_kernel_derivative():
    b_pp, b_f = 0.2, 2.0
    for r in (0.05, 0.15, 0.5, 1.2, 1.9):
        h = 1e-7
        fd = (oracle.pp_g(r + h, b_pp, b_f) - oracle.pp_g(r - h, b_pp, b_f)) / (2 * h)
        assert oracle.pp_dg(r, b_pp, b_f) == pytest.approx(fd, rel=1e-5, abs=1e-8)


@pytest.mark.parametrize("k", [0.0, 0.3, 1.5, 2.5, math.pi])
def test_alias_sum_cic_identity(k):
    # Textbook identity: sum_n sinc^4((k + 2 pi n)/2) = 1 - (2/3) sin^2(k/2).
    exact = 1 - 2 / 3 * math.sin(k / 2) ** 2
    assert oracle.alias_w2_1d(k, 400, 2) == pytest.approx(exact, abs=2e-8)
    # truncation |n| <= 2 leaves at most 1.5e-3 relative error (CIC)
    assert abs(oracle.alias_w2_1d(k, 2, 2) / exact - 1) < 1.6e-3


@pytest.mark.parametrize("k", [0.0, 0.3, 1.5, math.pi])
def test_alias_sum_tsc_identity(k):
    s = math.sin(k / 2) ** 2
    exact = 1 - s + 2 / 15 * s * s
    assert oracle.alias_w2_1d(k, 400, 3) == pytest.approx(exact, abs=1e-10)


class TestGreen:
    n = 32

    @pytest.fixture(scope="class")
    def G(self):
        return oracle.green_table(self.n, 2.0, math.inf)

    def test_zero_where_difference_operator_vanishes(self, G):
        h = self.n // 2
        for m in [(0, 0, 0), (h, 0, 0), (0, h, h), (h, h, h)]:
            assert G[m[2], m[1], m[0]] == 0.0

    def test_axis_permutation_symmetry(self, G):
        for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0)]:
            assert np.allclose(G, np.transpose(G, perm), rtol=1e-13, atol=0)

    def test_even_in_each_component(self):
        n = self.n
        for m in [(3, 5, 1), (7, 0, 2), (1, 1, 15)]:
            g0 = oracle.green_point(n, m, 2.0, math.inf)
            for flip in [(-1, 1, 1), (1, -1, 1), (1, 1, -1)]:
                mm = [a * b for a, b in zip(m, flip)]
                assert oracle.green_point(n, mm, 2.0, math.inf) == pytest.approx(g0, rel=1e-13)

    def test_table_matches_pointwise(self, G):
        for m in [(1, 2, 3), (16, 0, 5), (4, 4, 4)]:
            assert G[m[2], m[1], m[0]] == oracle.green_point(self.n, m, 2.0, math.inf)

    @pytest.mark.parametrize("n", [64, 256])
    def test_continuum_limit(self, n):
        # k -> 0 on the untruncated level: G -> -4 pi S^2(k, b) / k^2.
        b = 2.0
        k = 2 * math.pi / n
        g = oracle.green_point(n, (1, 0, 0), b, math.inf)
        target = -4 * math.pi * oracle.profile_k(k, b) ** 2 / k ** 2
        assert g / target == pytest.approx(1.0, abs=2e-3 * (64 / n) ** 2)
        assert g < 0  # attractive: phi is a potential well

    def test_truncated_level_vanishes_at_small_k(self):
        # PM2 (b_a=2, truncated at b_prev=14): S^2(k,2)-S^2(k,14) -> 0 as k -> 0,
        # i.e. the fine level carries no long-range force.
        n = 256
        g_small = oracle.green_point(n, (1, 0, 0), 2.0, 14.0)
        g_full = oracle.green_point(n, (1, 0, 0), 2.0, math.inf)
        assert abs(g_small) < 0.05 * abs(g_full)
