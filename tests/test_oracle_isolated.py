"""Pins of the oracle's isolated boundary conditions (appendix A): a mesh
twice the isolation box, the untruncated level's target force cut at half
the box (its transform times 1 - sinc(kL), eq. A2).

* far from the matching scales the force of an isolated pair is the
  softened pair force R(r, b_pp) itself (no periodic images) to well under a
  percent, where the periodic box's images bias it by several percent;
* the factor tends to one for L -> infinity (the periodic table), and it
  leaves the truncated finer levels unchanged (their force vanishes before
  r = L)."""
import numpy as np

import oracle


def _pair_err(o, p, x):
    a = o.accel(x)[:, 0]
    d = x[:, 1] - x[:, 0]
    r = np.linalg.norm(d)
    ref = oracle.refforce(r, p.b_pp) * d / r
    return np.linalg.norm(a - ref) / np.linalg.norm(ref)


def test_isolated_pair_force_is_the_softened_pair_force():
    rng = np.random.default_rng(41)
    iso = oracle.Params(n_fine=64, b_fine=4.0, b_pp=0.4, isolated=True)
    per = oracle.Params(n_fine=64, b_fine=4.0, b_pp=0.4)
    oi, op = oracle.Oracle(iso), oracle.Oracle(per)
    for r in (12.0, 20.0, 28.0):
        for _ in range(3):
            u = np.abs(rng.standard_normal(3))
            u /= np.linalg.norm(u)
            c = 1.0 + rng.random(3)
            x = np.stack([c, c + r * u], axis=1)          # inside [0, 32)^3
            assert _pair_err(oi, iso, x) < 0.005
    # the same pair in the periodic 64^3 box feels its images
    u = np.array([1.0, 0.0, 0.0])
    x = np.stack([np.array([2.0, 10.0, 10.0]), np.array([2.0, 10.0, 10.0]) + 28.0 * u], axis=1)
    assert _pair_err(op, per, x) > 0.05


def test_isolation_factor_limits():
    n, b = 32, 6.0
    g_per = oracle.green_table(n, b, np.inf, 2, 2)
    g_far = oracle.green_table(n, b, np.inf, 2, 2, iso_L=1e7)
    assert np.abs(g_far - g_per).max() <= 1e-6 * np.abs(g_per).max()
    g_iso = oracle.green_table(n, b, np.inf, 2, 2, iso_L=n / 2)
    assert np.abs(g_iso - g_per).max() > 1e-3 * np.abs(g_per).max()
    # a truncated level (b_prev finite) is what it is with or without isolation:
    # the oracle applies the factor to the untruncated level only
    p = oracle.Params(n_fine=64, coarse_ratio=4, isolated=True)
    o, o0 = oracle.Oracle(p), oracle.Oracle(oracle.Params(n_fine=64, coarse_ratio=4))
    assert np.array_equal(o.green(1), o0.green(1))
    assert not np.array_equal(o.green(0), o0.green(0))


def _pairwise_residuals(p, seed, per_bin=8, nbins=15):
    """F/R - 1 of random single pairs, log-spaced in r from 0.05 to L/2
    (the experiment of section 3.1), unquantised positions."""
    o = oracle.Oracle(p, quant=False)
    L = p.n_fine / 2
    edges = np.exp(np.linspace(np.log(0.05), np.log(L / 2), nbins + 1))
    rng = np.random.default_rng(seed)
    res = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        for _ in range(per_bin):
            r = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            # both particles inside [2, L - 2] on every axis
            a0 = 2.0 + np.maximum(-r * u, 0.0) + rng.random(3) * (L - 4.0 - r * np.abs(u))
            F = o.accel(np.stack([a0, a0 + r * u], axis=1))[:, 0]
            res.append(np.linalg.norm(F) / oracle.refforce(r, p.b_pp) - 1.0)
    return np.array(res)


def test_pairwise_accuracy_at_the_papers_softenings():
    """With TSC, b_PP = 0.06 and every PM softening 3.5 cells of its own mesh
    (the defaults of section 2.2), the pair force over all separations is
    within the paper's accuracy figures for its pairwise test (section 3.1,
    Fig. 1 and the summary in section 4: worst case 7%, rms 2%)."""
    p = oracle.Params(n_fine=64, coarse_ratio=4, b_coarse=14.0, b_fine=3.5, b_pp=0.06,
                      assign=3, isolated=True)
    res = _pairwise_residuals(p, 1203)
    assert np.abs(res).max() < 0.07
    assert np.sqrt(np.mean(res ** 2)) < 0.02
