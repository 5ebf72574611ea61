"""Pin of the optimized Green's function (section 2.1.2, eq. 11) at every
wave number, Nyquist planes included, without re-typing eq. 11.

G of eq. 11 is, by its construction, the influence function that minimises
the mean-square difference between the mesh force of the whole PM pipeline
(assignment, FFT x G, inverse FFT, the eq. 7 stencil, interpolation) and the
level's target force, averaged over the source particle's position in a cell
and over every test position (the alias sums of eq. 11 are that average in
Fourier space; the paper truncates them at |n_d| <= 2).  Here that average is
done by brute force instead: sources and test particles at Gauss-Legendre
points (4 per cell and axis for CIC, whose weights are linear in a cell; 3
per half cell for TSC, eq. 5, whose weights break at the cell centre), the
mesh force from the oracle's own deposit, potential, stencil and
interpolation, the target force R(r, b_a) - R(r, b_prev) of eq. 2 (a
truncated level, so the target has finite range and no periodic sum), and
for one octant entry m of the table at a time the scale factor 1 + eps of
that entry that minimises the functional (the functional is quadratic in it):

    eps* = -<(F - R) . F_m> / <F_m . F_m>,

F_m the mesh force of the table holding only the entry m.  At the optimum
eps* = 0.  The measured eps* shrinks with the alias range of eq. 11 as its
truncation error does (CIC: about 3e-2, 6e-3, 2e-3, 9e-4 for |n_d| <= 1..4 at
the highest wave numbers and below 1e-5 at the lowest; TSC, whose W^2 falls
faster: about 2e-4 at |n_d| <= 2 and 1e-5 at 4, measured with a finer
quadrature than the test's), so a mistake in any term
of eq. 11 (W for W^2, a dropped alias image, a wrong D or R component, a
wrong sign) shows up as an eps* far outside these bounds.  The source cell's
reflection symmetry lets one octant of it stand for the whole cell.
"""
import numpy as np
import pytest

import oracle

N = 16
B_A, B_PREV = 2.0, 5.0
MODES = [(7, 3, 1), (2, 1, 0), (1, 0, 0), (8, 4, 2), (4, 4, 4), (8, 1, 0), (8, 8, 1), (3, 8, 5)]


def _quad(u, w):
    """Sources in one octant of a cell and test particles in every cell at the
    points u (weights w) of [0, 1) per axis, with the target force of every
    (source, test) pair."""
    GQ = len(u)
    c1 = (np.arange(N)[:, None] + u[None, :]).ravel()
    w1 = np.tile(w, N)
    Z, Y, X = np.meshgrid(c1, c1, c1, indexing="ij")
    WZ, WY, WX = np.meshgrid(w1, w1, w1, indexing="ij")
    xt = np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()]))
    wt = (WZ * WY * WX).ravel()
    half = [i for i in range(GQ) if u[i] < 0.5]
    srcs = [(np.array([[u[a]], [u[b]], [u[c]]]) + 3.0, w[a] * w[b] * w[c])
            for a in half for b in half for c in half]
    refs = []
    for xs, _ in srcs:
        d = xs - xt                                   # towards the source
        d -= N * np.round(d / N)
        r = np.sqrt((d * d).sum(0))
        f = np.where(r < B_PREV, oracle.refforce_many(r, B_A) - oracle.refforce_many(r, B_PREV), 0.0)
        refs.append(f * d / np.maximum(r, 1e-300))
    return xt, wt, srcs, refs


def _gauss_cell(g):
    """g Gauss-Legendre points of the whole cell (CIC weights are linear in
    a cell)."""
    v, wv = np.polynomial.legendre.leggauss(g)
    return 0.5 * (v + 1.0), 0.5 * wv


def _gauss_half_cells(g):
    """g Gauss-Legendre points of each half cell (TSC weights break at the
    cell centre)."""
    v, wv = np.polynomial.legendre.leggauss(g)
    return (np.concatenate([0.25 * (v + 1.0), 0.5 + 0.25 * (v + 1.0)]),
            np.concatenate([0.25 * wv, 0.25 * wv]))


def _mesh_force(table, xs, xt, p):
    rho = oracle.deposit(np.ascontiguousarray(xs), N, 1.0, quant=False, p=p)
    E = oracle.fd_force(oracle.potential(rho, table))
    return oracle.interp(xt, E, 1.0, quant=False, p=p)


def _eps_star(quad, table, p, modes, scale=None):
    xt, wt, srcs, refs = quad
    t = table.copy()
    if scale is not None:
        t = t * scale
    f0 = [_mesh_force(t, xs, xt, p) for xs, _ in srcs]
    out = {}
    for m in modes:
        tm = np.zeros_like(t)
        tm[m[2], m[1], m[0]] = t[m[2], m[1], m[0]]
        num = den = 0.0
        for (xs, ws), f, r in zip(srcs, f0, refs):
            fm = _mesh_force(tm, xs, xt, p)
            num += ws * float(np.sum(wt * ((f - r) * fm).sum(0)))
            den += ws * float(np.sum(wt * (fm * fm).sum(0)))
        out[m] = -num / den
    return out


MODES_TSC = [(7, 3, 1), (8, 8, 1), (2, 1, 0), (8, 4, 2)]


def test_green_minimises_the_force_error():
    """CIC (the hot path's assignment): |eps*| < 1e-2 with the paper's alias
    range |n_d| <= 2 and < 1.5e-3 with |n_d| <= 4, falling by more than 3x
    between the two, and below 1e-5 on the longest waves."""
    quad = _quad(*_gauss_cell(4))
    e2 = _eps_star(quad, oracle.green_table(N, B_A, B_PREV, 2, 2), 2, MODES)
    e4 = _eps_star(quad, oracle.green_table(N, B_A, B_PREV, 4, 2), 2, MODES)
    for m in MODES:
        assert abs(e2[m]) < 1e-2, (m, e2[m])
        assert abs(e4[m]) < 1.5e-3, (m, e4[m])
    # the residual is the alias truncation: it falls with the alias range
    assert max(abs(v) for v in e4.values()) < 0.35 * max(abs(v) for v in e2.values())
    # the longest waves are optimal to far better than the truncation
    assert abs(e4[(1, 0, 0)]) < 1e-5 and abs(e4[(2, 1, 0)]) < 1e-4


def test_tsc_green_minimises_the_force_error():
    """TSC (eq. 5, W = sinc^3 in eq. 9): with 3 Gauss points per half cell
    the quadrature itself errs by up to ~4e-4 here, so the bound is 1e-3 at
    the paper's alias range (measured with 4 points per half cell: about
    2e-4 at |n_d| <= 2 and 1e-5 at 4); a dropped alias image or W for W^2
    would give eps* of several 1e-3 to O(1) at the highest wave numbers."""
    quad = _quad(*_gauss_half_cells(3))
    e2 = _eps_star(quad, oracle.green_table(N, B_A, B_PREV, 2, 3), 3, MODES_TSC)
    for m in MODES_TSC:
        assert abs(e2[m]) < 1e-3, (m, e2[m])
    assert abs(e2[(2, 1, 0)]) < 1e-6


def test_pin_resolves_a_one_percent_error():
    """The same measurement on a table scaled by 1.01 asks for the scale
    1/1.01 back at every entry: the pin resolves errors of a percent."""
    quad = _quad(*_gauss_cell(4))
    g = oracle.green_table(N, B_A, B_PREV, 4, 2)
    base = _eps_star(quad, g, 2, MODES)
    off = _eps_star(quad, g, 2, MODES, scale=1.01)
    for m in MODES:
        want = (1.0 + base[m]) / 1.01 - 1.0
        assert abs(off[m] - want) < 2e-4, (m, off[m], want)
