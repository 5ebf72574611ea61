"""Pins of the oracle's TSC assignment (eq. 5) and of the TSC force pipeline
(the G of eq. 11 with W = sinc^3, eq. 9), none of which re-types the
oracle's formulas:

* the fixed-point weights (16 bits, centre weight takes the remainder) sum to
  exactly one particle mass and lie within 2^-16 of eq. 5 evaluated here as
  a function of the node distance, for every node within reach (brute force
  over nodes, independent of the oracle's nearest-node decomposition);
* special positions (on a node, half way between nodes), translation,
  integer/float agreement;
* the first moment is exact: TSC interpolation of a linear field returns the
  field at the (quantised) particle position;
* forces: no self force, equal and opposite pairs, and against the exact
  periodic (Ewald) force of softened particles TSC is several times more
  accurate than CIC at the same softening, while TSC assignment with the
  CIC Green's function is not."""
import numpy as np
import pytest

import oracle
import synthetic


def _fine(x_box, n_f):
    return oracle.q_to_fine(oracle.quantize(x_box, n_f))


def _w_eq5(x):
    """eq. (5) as a function of the distance x to a node (level cells)."""
    x = np.abs(x)
    return np.where(x <= 0.5, 0.75 - x * x, np.where(x <= 1.5, 0.5 * (1.5 - x) ** 2, 0.0))


def test_tsc_deposit_conserves_mass_exactly():
    xf = _fine(synthetic.uniform(5000, 21), 32)
    acc = oracle.deposit_fx(xf, 32, 1.0, p=3)
    assert int(acc.sum(dtype=np.uint64)) == 5000 * 2 ** 48


@pytest.mark.parametrize("H", [1.0, 4.0])
def test_tsc_weights_within_rounding_of_eq5(H):
    n = 16
    rng = np.random.default_rng(22)
    for _ in range(200):
        x = rng.random(3) * n * H
        xq = _fine(x[:, None] / (n * H), int(n * H))[:, 0]     # 15-bit fine position
        acc = oracle.deposit_fx(xq[:, None], n, H, p=3).astype(np.float64) / 2.0 ** 48
        y = xq / H
        if H > 1:   # level fraction truncated to 15 bits, as the deposit does
            y = np.floor(y) + np.floor((y - np.floor(y)) * 32768) / 32768
        nodes = np.arange(n)
        ref = np.ones((n, n, n))
        for d, ax in ((0, (None, None, slice(None))), (1, (None, slice(None), None)),
                      (2, (slice(None), None, None))):
            dist = (y[d] - nodes + n / 2) % n - n / 2               # periodic distance
            ref = ref * _w_eq5(dist)[ax]
        # per-axis weights within 2^-16 of eq. 5: products within 3 * 2^-16
        assert np.abs(acc - ref).max() <= 3 * 2.0 ** -16 + 1e-15
        assert abs(acc.sum() - 1.0) < 1e-15


def test_tsc_special_positions():
    # on a node: 1/8, 3/4, 1/8 per axis; half way between nodes: 1/2, 1/2
    acc = oracle.deposit_fx(np.array([[5.0], [5.0], [5.0]]), 16, 1.0, p=3).astype(np.float64)
    w = acc[4:7, 5, 5] / (0.75 * 0.75 * 2.0 ** 48)
    assert np.array_equal(w, [0.125, 0.75, 0.125])
    acc = oracle.deposit_fx(np.array([[5.5], [5.0], [5.0]]), 16, 1.0, p=3).astype(np.float64)
    w = acc[5, 5, 4:8] / (0.75 * 0.75 * 2.0 ** 48)
    assert np.array_equal(w, [0.0, 0.5, 0.5, 0.0])


def test_tsc_deposit_translation_permutes_mesh():
    xf = _fine(synthetic.uniform(300, 23), 16)
    a0 = oracle.deposit_fx(xf, 16, 1.0, p=3)
    a1 = oracle.deposit_fx(np.mod(xf + np.array([[3.0], [1.0], [5.0]]), 16), 16, 1.0, p=3)
    assert np.array_equal(np.roll(a0, (5, 1, 3), axis=(0, 1, 2)), a1)


def test_tsc_integer_and_float_deposit_agree():
    xf = _fine(synthetic.uniform(2000, 24), 32)
    for H, n in ((1.0, 32), (4.0, 8)):
        a = oracle.deposit_fx(xf, n, H, p=3).astype(np.float64) * 2.0 ** -48
        b = oracle.deposit(xf, n, H, True, p=3)
        assert np.abs(a - b).max() < 1e-12


def test_tsc_interpolation_first_moment_is_exact():
    # E_x(n) = n, E_y(n) = 2n_y, E_z(n) = -n_z, particles away from the wrap
    n = 32
    g = np.arange(n, dtype=np.float64)
    E = np.stack([np.broadcast_to(g[None, None, :], (n, n, n)),
                  np.broadcast_to(2 * g[None, :, None], (n, n, n)),
                  np.broadcast_to(-g[:, None, None], (n, n, n))]).copy()
    rng = np.random.default_rng(25)
    xf = _fine(rng.uniform(4, 28, (3, 500)) / n, n)
    a = oracle.interp(xf, E, 1.0, True, p=3)
    assert np.abs(a[0] - xf[0]).max() < 1e-12
    assert np.abs(a[1] - 2 * xf[1]).max() < 1e-12
    assert np.abs(a[2] + xf[2]).max() < 1e-12


@pytest.fixture(scope="module")
def tsc64():
    return oracle.Oracle(oracle.Params(n_fine=64, assign=3))


def test_tsc_no_self_force_and_equal_opposite_pairs(tsc64):
    rng = np.random.default_rng(26)
    for _ in range(4):
        a = tsc64.pm_accel(rng.random((3, 1)) * 64)
        assert np.abs(a).max() < 1e-12
        a = tsc64.accel(rng.random((3, 2)) * 64)
        assert np.abs(a[:, 0] + a[:, 1]).max() < 1e-12 * max(1.0, np.abs(a).max())


def test_tsc_force_more_accurate_than_cic_against_ewald():
    xf = _fine(synthetic.uniform(256, 16), 32)
    med = {}
    for assign in (2, 3):
        p = oracle.Params(n_fine=32, b_fine=6.0, b_pp=0.6, assign=assign)
        ref = oracle.reference_accel(xf, p)
        a = oracle.Oracle(p).accel(xf)
        med[assign] = np.median(np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0))
    assert med[3] < 0.004 and med[3] < 0.4 * med[2], med
    # TSC assignment with the CIC window in G (eq. 9 exponent 2) is worse
    p = oracle.Params(n_fine=32, b_fine=6.0, b_pp=0.6, assign=3)
    o = oracle.Oracle(p)
    H, n, ba, bp = p.levels()[0]
    o._G[0] = oracle.green_table(n, ba / H, bp / H, p.alias_nmax, 2)
    ref = oracle.reference_accel(xf, p)
    bad = np.median(np.linalg.norm(o.accel(xf) - ref, axis=0) / np.linalg.norm(ref, axis=0))
    assert bad > 2 * med[3]


# ------------------------------------------------------------ TSC adjoints --

def _away_from_midpoints(xf, Hs, margin):
    """Positions whose level coordinates stay clear of the half-integers,
    where the nearest TSC node changes (eq. 5 is C1 there, but its second
    derivative jumps)."""
    ok = np.ones(xf.shape[1], dtype=bool)
    for H in Hs:
        fr = np.mod(xf / H, 1.0)
        ok &= np.all(np.abs(fr - 0.5) > margin, axis=0)
    return ok


@pytest.mark.parametrize("two_level", [False, True])
def test_tsc_force_adjoint_matches_finite_differences(two_level):
    # <xbar, v> = d/de sum(abar . a(x + e v)), FP64 central differences of
    # the continuous-position TSC forward
    p = oracle.Params(n_fine=32, coarse_ratio=4 if two_level else 0, b_coarse=14.0, assign=3)
    o = oracle.Oracle(p, quant=False)
    rng = np.random.default_rng(61)
    xf = rng.random((3, 200)) * 32
    xf = np.ascontiguousarray(xf[:, _away_from_midpoints(xf, [1, 4], 0.02)])
    N = xf.shape[1]
    abar = rng.standard_normal((3, N))
    xbar = o.accel_adjoint(xf, abar)
    for _ in range(3):
        v = rng.standard_normal((3, N))
        h = 1e-5
        fd = (np.sum(abar * o.accel(xf + h * v)) - np.sum(abar * o.accel(xf - h * v))) / (2 * h)
        assert np.sum(xbar * v) == pytest.approx(fd, rel=2e-6)


def test_tsc_deposit_adjoint_matches_finite_differences():
    o = oracle.Oracle(oracle.Params(n_fine=16, assign=3), quant=False)
    rng = np.random.default_rng(62)
    xf = rng.random((3, 100)) * 16
    xf = np.ascontiguousarray(xf[:, _away_from_midpoints(xf, [1], 0.02)])
    rhobar = rng.standard_normal((16, 16, 16))
    xbar = o.deposit_adjoint(xf, rhobar)
    v = rng.standard_normal(xf.shape)
    h = 1e-6
    f = lambda y: np.sum(rhobar * oracle.deposit(y, 16, 1, quant=False, p=3))
    fd = (f(xf + h * v) - f(xf - h * v)) / (2 * h)
    assert np.sum(xbar * v) == pytest.approx(fd, rel=1e-7)


def test_tsc_weight_derivatives_are_those_of_eq5():
    """The per-axis derivative used by the adjoints, checked through the
    deposit adjoint of a single particle against the slope of eq. 5 written
    out as a function of the node distance."""
    o = oracle.Oracle(oracle.Params(n_fine=16, assign=3), quant=False)
    W = lambda t: np.where(np.abs(t) <= 0.5, 0.75 - t * t,
                           np.where(np.abs(t) <= 1.5, 0.5 * (1.5 - np.abs(t)) ** 2, 0.0))
    dW = lambda t: np.where(np.abs(t) <= 0.5, -2 * t,
                            np.where(np.abs(t) <= 1.5, -np.sign(t) * (1.5 - np.abs(t)), 0.0))
    for y in (5.1, 5.3, 5.49, 5.51, 5.9):
        x = np.array([[y], [7.2], [8.6]])
        for node in (4, 5, 6, 7):
            rhobar = np.zeros((16, 16, 16))
            rhobar[8, 7, node] = 1.0        # [z][y][x]: only the x node varies
            xb = o.deposit_adjoint(x, rhobar)
            expect = dW(y - node) * W(7.2 - 7) * W(8.6 - 8)
            assert xb[0, 0] == pytest.approx(expect, abs=1e-14)
