"""CPU pins of the FP32 forward pair law (eqs. 2 and 4d) as the PP kernel
evaluates it: h = g / (b_f^2 - s)^5 tabulated by s = r^2 with one cubic per
1/16 of an octave, g = h max(b_f^2 - s, 0)^5, evaluated on the host with the
kernel's own FP32 operations (cube2_pair_law_f32).  It is compared with

* the exact rational pair law of oracle.exact on separations that are
  multiples of 2^-15 fine cells (the only separations the IOS positions
  produce), and
* the extended-precision oracle pair law on a dense random sweep of r,
  including the neighbourhoods of the breakpoints b_pp/2, b_pp, b_f/2 and the
  cutoff b_f,

relative to g itself: |g32 - g| <= (2e-6 + 1e-6 / q) |g| with q = 1 - r/b_f.
The 1/q part is the FP32 rounding of s, which b_f^2 - s amplifies near the
cutoff (g vanishes like q^5 there); the table alone is within 8e-7.  The
sweep stops at q = 1e-3, below which the extended-precision oracle itself
loses digits to the cancellation R(r, b_pp) - R(r, b_f); the exact rational
check has no such limit.  Beyond the cutoff the law is exactly 0, and a
coincident pair gets a finite g."""
import ctypes
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from oracle import exact

CONFIGS = [(2.0, 0.2), (1.5, 0.1), (1.0, 0.3), (3.5, 0.0625)]


def _ctx(b_f, b_pp):
    import paper_2512_12629_amd as m
    cfg = m.cube2_config(n_fine=64, coarse_ratio=0, b_coarse=14.0, b_fine=b_f, b_pp=b_pp,
                         m_p=1.0, g_newton=1.0, alias_nmax=2, flags=0)
    return m, m.cube2_create(cfg)


@pytest.mark.parametrize("b_f,b_pp", CONFIGS)
def test_pair_law_f32_against_exact_rational(b_f, b_pp):
    m, h = _ctx(b_f, b_pp)
    try:
        rng = np.random.default_rng(7)
        # integer separations (units of 2^-15 fine cells) with r spread over
        # [2^-15, 1.2 b_f), log-uniform, plus r close below the cutoff
        r = np.concatenate([np.exp(rng.uniform(np.log(2.0 ** -14), np.log(1.2 * b_f), 300)),
                            b_f * (1 - 10 ** rng.uniform(-5, -1, 60))])
        u = rng.standard_normal((3, r.size))
        u /= np.linalg.norm(u, axis=0)
        n = np.rint(u * r * 2 ** 15).astype(np.int64)
        n[:, 0] = (1, 0, 0)                      # the smallest separation
        d = (n * 2.0 ** -15).astype(np.float32)
        assert np.array_equal(d.astype(np.float64) * 2 ** 15, n)     # exact floats
        g32 = m.cube2_pair_law_f32(h, d).astype(np.float64)
        bpp, bf = Fr(b_pp).limit_denominator(10 ** 12), Fr(b_f).limit_denominator(10 ** 12)
        for i in range(n.shape[1]):
            n2 = int((n[:, i] ** 2).sum())
            g = float(exact.pair_g(n2, bpp, bf))
            q = 1.0 - (n2 * 2.0 ** -30) ** 0.5 / b_f
            if q <= 0:
                assert g32[i] == 0.0
            else:
                assert abs(g32[i] - g) <= (2e-6 + 1e-6 / q) * abs(g), (i, n[:, i], g32[i], g)
    finally:
        m.cube2_destroy(h)


@pytest.mark.parametrize("b_f,b_pp", CONFIGS)
def test_pair_law_f32_sweep_against_oracle(b_f, b_pp):
    m, h = _ctx(b_f, b_pp)
    try:
        rng = np.random.default_rng(11)
        edges = [b_pp / 2, b_pp, b_f / 2]
        r = np.concatenate([np.exp(rng.uniform(np.log(3e-5), np.log(b_f), 6000)),
                            b_f * (1 - 10 ** rng.uniform(-3, -1, 1500)),
                            b_f * (1 + rng.uniform(0, 0.02, 500))] +
                           [e * (1 + rng.uniform(-0.02, 0.02, 1500)) for e in edges])
        u = rng.standard_normal((3, r.size))
        u /= np.linalg.norm(u, axis=0)
        d = (u * r).astype(np.float32)
        g32 = m.cube2_pair_law_f32(h, d).astype(np.float64)
        dd = d.astype(np.float64)
        rr = np.sqrt((dd * dd).sum(axis=0))
        ref = np.array([oracle.pp_g(x, b_pp, b_f) for x in rr])
        q = 1.0 - rr / b_f
        inside = q >= 1e-3
        err = np.abs(g32 - ref)[inside] / ((2e-6 + 1e-6 / q[inside]) * np.abs(ref[inside]))
        assert err.max() <= 1.0, (err.max(), rr[inside][np.argmax(err)])
        assert np.all(g32[q <= 0] == 0.0)
    finally:
        m.cube2_destroy(h)


def test_pair_law_f32_coincident_and_range():
    m, h = _ctx(2.0, 0.2)
    try:
        g = m.cube2_pair_law_f32(h, np.zeros((3, 1), np.float32))
        assert np.isfinite(g[0])
        # the largest separation of the staged box is below 4 cells per axis
        far = np.full((3, 1), 3.9999, np.float32)
        assert m.cube2_pair_law_f32(h, far)[0] == 0.0
        with pytest.raises(m.Cube2Error):
            m.cube2_pair_law_f32(h, np.full((3, 1), 4.0, np.float32))
    finally:
        m.cube2_destroy(h)


@pytest.mark.parametrize("b_f,b_pp", CONFIGS)
def test_pair_jacobian_f32_against_oracle(b_f, b_pp):
    """The adjoint kernel's (g, g_s = dg/ds) against the extended-precision
    oracle (g_s = (dg/dr) / 2r): g as above; the term 2 g_s D D^T of the pair
    Jacobian g I + 2 g_s D D^T within (1e-4 + 5e-7/q) of the Jacobian's size
    |g| + 2 |g_s| s (g_s comes from the derivative of the forward table's
    cubic, good to a few 1e-5 of the Jacobian, worst next to the breakpoints
    of eq. 2 inside a row; g_s vanishes like q^4 at the cutoff)."""
    m, h = _ctx(b_f, b_pp)
    try:
        rng = np.random.default_rng(13)
        edges = [b_pp / 2, b_pp, b_f / 2]
        r = np.concatenate([np.exp(rng.uniform(np.log(3e-5), np.log(b_f), 6000)),
                            b_f * (1 - 10 ** rng.uniform(-3, -1, 1500)),
                            b_f * (1 + rng.uniform(0, 0.02, 500))] +
                           [e * (1 + rng.uniform(-0.02, 0.02, 1500)) for e in edges])
        u = rng.standard_normal((3, r.size))
        u /= np.linalg.norm(u, axis=0)
        d = (u * r).astype(np.float32)
        g, gs = m.cube2_pair_jacobian_f32(h, d)
        dd = d.astype(np.float64)
        rr = np.sqrt((dd * dd).sum(axis=0))
        q = 1.0 - rr / b_f
        gref = np.array([oracle.pp_g(x, b_pp, b_f) for x in rr])
        gsref = np.array([oracle.pp_dg(x, b_pp, b_f) for x in rr]) / (2 * rr)
        inside = q >= 1e-3
        eg = np.abs(g - gref)[inside] / ((2e-6 + 1e-6 / q[inside]) * np.abs(gref[inside]))
        s2 = 2 * rr[inside] ** 2
        jac = np.abs(gref[inside]) + np.abs(gsref[inside]) * s2
        es = np.abs(gs - gsref)[inside] * s2 / ((1e-4 + 5e-7 / q[inside]) * jac)
        assert eg.max() <= 1.0, (eg.max(), rr[inside][np.argmax(eg)])
        assert es.max() <= 1.0, (es.max(), rr[inside][np.argmax(es)])
        assert np.all(g[q <= 0] == 0.0) and np.all(gs[q <= 0] == 0.0)
    finally:
        m.cube2_destroy(h)
