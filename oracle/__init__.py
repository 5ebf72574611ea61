"""FP64 CPU oracle of the CUBE2 force computation (arXiv 2512.12629).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP path (``paper_2512_12629_amd``) and neither imports the
other; the two meet only through the seeded inputs of ``synthetic``.

The oracle follows the paper's steps in order, in FP64:

* quantise positions to in-cell integer offsets (IOS, section 2.3);
* per PM level: CIC mass assignment (section 2.1.2, the CIC kernel in place
  of the paper's TSC), FFT, multiply by the optimized Green's function
  (eq. 11 with eqs. 9, 10, 12, 13), inverse FFT, the 4-point finite
  difference (eq. 7) and CIC interpolation with the same weights;
* the PP sum of eq. (4d) with the short-range softening handed over by the
  finest PM level;
* leapfrog kick and drift (sections 2.2.3 and 2.3);
* the adjoints of all of the above (not in the paper; derived in the module
  docstrings and pinned by finite differences in the tests).

The loops live in ``cube2_oracle.c`` (plain C, built with gcc); the FFT is
numpy's (a library primitive used as one step).  One step departs from FP64:
the PP pair law subtracts two eq. (2) forces that cancel near the cutoff, so
eq. (2) and the difference are evaluated in x87 extended precision and
rounded once.  ``oracle.exact`` evaluates the PP sum in exact rational
arithmetic for small particle sets.

Parity pins: see tests/test_oracle_*.py.  The IOS velocity codec follows a
linear reading of section 2.3 (the paper defers its formula to an earlier
paper): pinned by its own definition (round trip, cell means, invariances),
parity unpinned in the paper's terms.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cube2_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

FRAC_BITS = 15           # in-cell fraction of a fine cell: 2^-15
IOS_RATIO = 2            # IOS cell = 2 fine cells (= H_p in every workload)
TILE_CELLS = 8           # IOS cells per tile side in the particle order


def build(force: bool = False) -> str:
    """Compile the oracle's C part with gcc (no fast-math, no contraction)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        d, i, i64, p = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        sig = {
            "orc_profile": (d, [d, d]),
            "orc_refforce": (d, [d, d]),
            "orc_refforce_many": (None, [i64, p, d, p]),
            "orc_refforce_dr": (d, [d, d]),
            "orc_profile_k": (d, [d, d]),
            "orc_green_point": (d, [i, i, i, i, d, d, i, i, d]),
            "orc_green_table": (None, [i, d, d, i, i, d, p]),
            "orc_alias_w2_1d": (d, [d, i, i]),
            "orc_deposit_fx": (None, [i64, p, i, d, p]),
            "orc_deposit": (None, [i64, p, i, d, i, p]),
            "orc_fd_force": (None, [i, p, p]),
            "orc_fd_force_adjoint": (None, [i, p, p]),
            "orc_interp": (None, [i64, p, i, d, i, p, p]),
            "orc_deposit_tsc_fx": (None, [i64, p, i, d, p]),
            "orc_deposit_tsc": (None, [i64, p, i, d, i, p]),
            "orc_interp_tsc": (None, [i64, p, i, d, i, p, p]),
            "orc_interp_adjoint_mesh": (None, [i64, p, i, d, i, p, p]),
            "orc_interp_adjoint_pos": (None, [i64, p, i, d, i, p, p, p]),
            "orc_deposit_adjoint_pos": (None, [i64, p, i, d, i, p, p]),
            "orc_interp_adjoint_mesh_tsc": (None, [i64, p, i, d, i, p, p]),
            "orc_interp_adjoint_pos_tsc": (None, [i64, p, i, d, i, p, p, p]),
            "orc_deposit_adjoint_pos_tsc": (None, [i64, p, i, d, i, p, p]),
            "orc_pp_g": (d, [d, d, d]),
            "orc_pp_dg": (d, [d, d, d]),
            "orc_pp_brute": (None, [i64, p, d, d, d, p]),
            "orc_pp": (None, [i64, p, d, d, d, p]),
            "orc_pp_subset": (None, [i64, p, d, d, d, i64, p, p]),
            "orc_pp_count": (i64, [i64, p, d, d]),
            "orc_pp_adjoint": (None, [i64, p, d, d, d, p, p]),
            "orc_pp_adjoint_subset": (None, [i64, p, d, d, d, p, i64, p, p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------

@dataclass
class Params:
    """Force parameters in fine-cell units (section 2.1.1, 2.2).

    coarse_ratio = 0: one PM level with softening b_fine (b_0 = infinity).
    coarse_ratio = H: a coarse level of spacing H fine cells with softening
    b_coarse (untruncated) and a fine level with softening b_fine truncated
    at b_coarse (eq. 4a, 4b); PP softening b_pp, cutoff b_fine (eq. 4d).
    """
    n_fine: int
    coarse_ratio: int = 0
    b_coarse: float = 14.0
    b_fine: float = 2.0
    b_pp: float = 0.2
    m_p: float = 1.0
    G_N: float = 1.0
    alias_nmax: int = 2
    assign: int = 2          # 2 = CIC, 3 = TSC (eq. 5)
    isolated: bool = False   # isolated boundaries (appendix A): particles in the
                             # first half of the box, the untruncated level's
                             # target force truncated at half the box length

    def levels(self):
        """[(H, n, b_alpha, b_prev)] in fine-cell units; b_prev=inf for PM1."""
        if self.coarse_ratio:
            H = self.coarse_ratio
            return [(H, self.n_fine // H, self.b_coarse, math.inf),
                    (1, self.n_fine, self.b_fine, self.b_coarse)]
        return [(1, self.n_fine, self.b_fine, math.inf)]


# ---------------------------------------------------------------------------
# Closed forms (eqs. 1, 2, 13) and the Green's function (eq. 11)
# ---------------------------------------------------------------------------

def profile(r, b):
    return lib().orc_profile(float(r), float(b))


def refforce(r, b):
    return lib().orc_refforce(float(r), float(b))


def refforce_many(r, b):
    """R(r, b) of eq. (2) for an array of r (same evaluation as refforce)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.empty_like(r)
    lib().orc_refforce_many(r.size, _p(r), float(b), _p(out))
    return out


def refforce_dr(r, b):
    return lib().orc_refforce_dr(float(r), float(b))


def profile_k(k, b):
    return lib().orc_profile_k(float(k), -1.0 if math.isinf(b) else float(b))


def pp_g(r, b_pp, b_f):
    return lib().orc_pp_g(float(r), float(b_pp), float(b_f))


def pp_dg(r, b_pp, b_f):
    return lib().orc_pp_dg(float(r), float(b_pp), float(b_f))


def alias_w2_1d(k, nmax, p):
    return lib().orc_alias_w2_1d(float(k), int(nmax), int(p))


def _b(b):
    return -1.0 if math.isinf(b) else float(b)


def green_point(n, m, b_a, b_prev, nmax=2, p=2, iso_L=0.0):
    """G at integer wave vector m (level units: b in level cells); iso_L > 0:
    isolated boundaries, target force truncated at r = iso_L (appendix A)."""
    return lib().orc_green_point(int(n), int(m[0]), int(m[1]), int(m[2]),
                                 float(b_a), _b(b_prev), int(nmax), int(p), float(iso_L))


def green_table(n, b_a, b_prev, nmax=2, p=2, iso_L=0.0):
    """Octant table G[m3][m2][m1], m_d in [0, n/2], level units."""
    h = n // 2 + 1
    out = np.zeros((h, h, h))
    lib().orc_green_table(int(n), float(b_a), _b(b_prev), int(nmax), int(p), float(iso_L),
                          _p(out))
    return out


def green_full(table, n):
    """Expand the octant table to numpy's rfftn layout [kz, ky, kx]."""
    m = np.minimum(np.arange(n), n - np.arange(n))
    h = n // 2 + 1
    return table[m[:, None, None], m[None, :, None], np.arange(h)[None, None, :]]


# ---------------------------------------------------------------------------
# Positions: quantisation and the IOS particle order (section 2.3)
# ---------------------------------------------------------------------------

def quantize(x_box: np.ndarray, n_fine: int) -> np.ndarray:
    """Box-unit positions -> integer positions q in units of 2^-15 fine cells.

    q = floor(x * n_fine * 2^15) mod (n_fine * 2^15), exact in FP64.
    """
    span = n_fine << FRAC_BITS
    q = np.floor(np.asarray(x_box, dtype=np.float64) * span).astype(np.int64)
    return np.mod(q, span)


def q_to_fine(q: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(q.astype(np.float64) / float(1 << FRAC_BITS))


def ios_cell_key(q: np.ndarray, n_fine: int) -> np.ndarray:
    """Tile-major IOS cell index of each particle.

    IOS cell c_d = q_d >> 16 (2 fine cells); tiles of 8^3 IOS cells are laid
    out x-fastest, and so are the cells inside a tile.
    """
    n_ios = n_fine // IOS_RATIO
    nt = n_ios // TILE_CELLS
    c = q >> (FRAC_BITS + 1)
    t = c // TILE_CELLS
    u = c % TILE_CELLS
    tile = (t[2] * nt + t[1]) * nt + t[0]
    inner = (u[2] * TILE_CELLS + u[1]) * TILE_CELLS + u[0]
    return tile * TILE_CELLS ** 3 + inner


def ios_order(q: np.ndarray, n_fine: int):
    """Stable sort by IOS cell: returns (perm, cell_start, offsets uint16).

    perm[i] is the input index of the i-th sorted particle; cell_start has
    n_ios^3 + 1 entries; offsets = q & 0xFFFF in sorted order.
    """
    key = ios_cell_key(q, n_fine)
    perm = np.argsort(key, kind="stable")
    n_cells = (n_fine // IOS_RATIO) ** 3
    counts = np.bincount(key, minlength=n_cells)
    cell_start = np.zeros(n_cells + 1, dtype=np.int64)
    np.cumsum(counts, out=cell_start[1:])
    off = (q[:, perm] & 0xFFFF).astype(np.uint16)
    return perm, cell_start.astype(np.uint32), off


# ---------------------------------------------------------------------------
# PM steps
# ---------------------------------------------------------------------------

def deposit_fx(xf: np.ndarray, n: int, H: float, p: int = 2) -> np.ndarray:
    """Exact integer deposit (uint64): CIC (p = 2) with weights in units of
    2^-45, or TSC (p = 3, eq. 5) with 16-bit weights, units of 2^-48."""
    xf = np.ascontiguousarray(xf, dtype=np.float64)
    out = np.zeros((n, n, n), dtype=np.uint64)
    f = lib().orc_deposit_tsc_fx if p == 3 else lib().orc_deposit_fx
    f(xf.shape[1], _p(xf), int(n), float(H), _p(out))
    return out


def fx_scale(p: int = 2) -> float:
    """Value of one unit of the integer deposit accumulator (a particle mass)."""
    return 2.0 ** -48 if p == 3 else 2.0 ** -45


def density_f32(acc: np.ndarray, p: int = 2) -> np.ndarray:
    """FP32 density: the integer accumulator rounded to nearest, times its unit."""
    return (acc.astype(np.float32) * np.float32(fx_scale(p))).astype(np.float32)


def deposit(xf: np.ndarray, n: int, H: float, quant: bool = True, p: int = 2) -> np.ndarray:
    xf = np.ascontiguousarray(xf, dtype=np.float64)
    out = np.zeros((n, n, n))
    f = lib().orc_deposit_tsc if p == 3 else lib().orc_deposit
    f(xf.shape[1], _p(xf), int(n), float(H), int(quant), _p(out))
    return out


def potential(rho: np.ndarray, G_table: np.ndarray, workers: int = 1) -> np.ndarray:
    """phi = IFFT(G * FFT(rho)), forward unnormalised, inverse 1/n^3.

    workers > 1 uses scipy's multi-threaded FFT (the same transform, for the
    large meshes); otherwise numpy's."""
    n = rho.shape[0]
    if workers > 1:
        import scipy.fft
        spec = scipy.fft.rfftn(rho, workers=workers)
        spec *= green_full(G_table, n)
        return scipy.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2), workers=workers)
    return np.fft.irfftn(np.fft.rfftn(rho) * green_full(G_table, n), s=(n, n, n), axes=(0, 1, 2))


def fd_force(phi: np.ndarray) -> np.ndarray:
    n = phi.shape[0]
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    E = np.zeros((3, n, n, n))
    lib().orc_fd_force(int(n), _p(phi), _p(E))
    return E


def fd_force_adjoint(Eb: np.ndarray) -> np.ndarray:
    n = Eb.shape[1]
    Eb = np.ascontiguousarray(Eb, dtype=np.float64)
    out = np.zeros((n, n, n))
    lib().orc_fd_force_adjoint(int(n), _p(Eb), _p(out))
    return out


def interp(xf: np.ndarray, E: np.ndarray, H: float, quant: bool = True, p: int = 2) -> np.ndarray:
    xf = np.ascontiguousarray(xf, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    n = E.shape[1]
    acc = np.zeros((3, xf.shape[1]))
    f = lib().orc_interp_tsc if p == 3 else lib().orc_interp
    f(xf.shape[1], _p(xf), int(n), float(H), int(quant), _p(E), _p(acc))
    return acc


class Oracle:
    """The force computation for one parameter set, with cached G tables."""

    def __init__(self, params: Params, quant: bool = True, workers: int = 1):
        self.p = params
        self.quant = quant
        self.workers = workers       # threads of the library FFT (see potential)
        self._G = {}

    def green(self, level: int) -> np.ndarray:
        if level not in self._G:
            H, n, b_a, b_prev = self.p.levels()[level]
            iso_L = n / 2 if (self.p.isolated and math.isinf(b_prev)) else 0.0
            self._G[level] = green_table(n, b_a / H, b_prev / H, self.p.alias_nmax, self.p.assign,
                                         iso_L)
        return self._G[level]

    # -- forward ------------------------------------------------------------
    def level_mesh(self, xf, level):
        """(rho, phi, E) of one level, unit particle mass."""
        H, n, _, _ = self.p.levels()[level]
        rho = deposit(xf, n, H, self.quant, self.p.assign)
        phi = potential(rho, self.green(level), self.workers)
        return rho, phi, fd_force(phi)

    def pm_level_accel(self, xf, level):
        """Acceleration of one PM level in fine-cell units (G m included)."""
        H = self.p.levels()[level][0]
        _, _, E = self.level_mesh(xf, level)
        return interp(xf, E, H, self.quant, self.p.assign) * (self.p.G_N * self.p.m_p / H ** 2)

    def pm_accel(self, xf):
        return sum(self.pm_level_accel(xf, l) for l in range(len(self.p.levels())))

    def pp_accel(self, xf, brute: bool = False):
        xf = np.ascontiguousarray(xf, dtype=np.float64)
        acc = np.zeros((3, xf.shape[1]))
        f = lib().orc_pp_brute if brute else lib().orc_pp
        f(xf.shape[1], _p(xf), float(self.p.n_fine), float(self.p.b_pp),
          float(self.p.b_fine), _p(acc))
        return acc * (self.p.G_N * self.p.m_p)

    def pp_accel_subset(self, xf, idx):
        xf = np.ascontiguousarray(xf, dtype=np.float64)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        acc = np.zeros((3, len(idx)))
        lib().orc_pp_subset(xf.shape[1], _p(xf), float(self.p.n_fine), float(self.p.b_pp),
                            float(self.p.b_fine), len(idx), _p(idx), _p(acc))
        return acc * (self.p.G_N * self.p.m_p)

    def pp_pair_count(self, xf):
        xf = np.ascontiguousarray(xf, dtype=np.float64)
        return int(lib().orc_pp_count(xf.shape[1], _p(xf), float(self.p.n_fine),
                                      float(self.p.b_fine)))

    def accel(self, xf, pp: bool = True):
        a = self.pm_accel(xf)
        if pp:
            a = a + self.pp_accel(xf)
        return a

    # -- adjoints -------------------------------------------------------------
    def pm_level_adjoint(self, xf, level, abar):
        """x-bar of one PM level for the acceleration cotangent abar (3, N).

        With a_i = c sum_n W(y_i - n) E(n), E = -D phi, phi = K rho and
        rho(n) = sum_j W(y_j - n), c = G m / H^2:
          Abar = c * sum_i W(y_i - n) abar_i          (scatter)
          phibar = +D . Abar                          (FD transpose, D^T = -D)
          rhobar = K phibar                           (G real, even: K^T = K)
          xbar_i = c grad_x W . (abar_i . E) + grad_x W . rhobar
        """
        tsc = self.p.assign == 3
        H = self.p.levels()[level][0]
        n = self.p.levels()[level][1]
        c = self.p.G_N * self.p.m_p / H ** 2
        xf = np.ascontiguousarray(xf, dtype=np.float64)
        N = xf.shape[1]
        abar = np.ascontiguousarray(abar, dtype=np.float64)
        _, _, E = self.level_mesh(xf, level)
        xbar = np.zeros((3, N))
        ab_c = np.ascontiguousarray(abar * c)
        L = lib()
        adj_pos = L.orc_interp_adjoint_pos_tsc if tsc else L.orc_interp_adjoint_pos
        adj_mesh = L.orc_interp_adjoint_mesh_tsc if tsc else L.orc_interp_adjoint_mesh
        dep_pos = L.orc_deposit_adjoint_pos_tsc if tsc else L.orc_deposit_adjoint_pos
        adj_pos(N, _p(xf), int(n), float(H), int(self.quant),
                _p(np.ascontiguousarray(E)), _p(ab_c), _p(xbar))
        Eb = np.zeros((3, n, n, n))
        adj_mesh(N, _p(xf), int(n), float(H), int(self.quant), _p(ab_c), _p(Eb))
        phibar = fd_force_adjoint(Eb)
        rhobar = np.ascontiguousarray(potential(phibar, self.green(level)))
        dep_pos(N, _p(xf), int(n), float(H), int(self.quant), _p(rhobar), _p(xbar))
        return xbar

    def pm_adjoint(self, xf, abar):
        return sum(self.pm_level_adjoint(xf, l, abar) for l in range(len(self.p.levels())))

    def pp_adjoint(self, xf, abar):
        """xbar_k = G m sum_j J(D_kj) (abar_j - abar_k), J = g I + g' D D^T / r."""
        xf = np.ascontiguousarray(xf, dtype=np.float64)
        ab = np.ascontiguousarray(abar, dtype=np.float64)
        xbar = np.zeros((3, xf.shape[1]))
        lib().orc_pp_adjoint(xf.shape[1], _p(xf), float(self.p.n_fine), float(self.p.b_pp),
                             float(self.p.b_fine), _p(ab), _p(xbar))
        return xbar * (self.p.G_N * self.p.m_p)

    def pp_adjoint_subset(self, xf, abar, idx):
        """The PP adjoint of the target particles idx only (3, len(idx))."""
        xf = np.ascontiguousarray(xf, dtype=np.float64)
        ab = np.ascontiguousarray(abar, dtype=np.float64)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.zeros((3, len(idx)))
        lib().orc_pp_adjoint_subset(xf.shape[1], _p(xf), float(self.p.n_fine), float(self.p.b_pp),
                                    float(self.p.b_fine), _p(ab), len(idx), _p(idx), _p(out))
        return out * (self.p.G_N * self.p.m_p)

    def accel_adjoint(self, xf, abar, pp: bool = True):
        xb = self.pm_adjoint(xf, abar)
        if pp:
            xb = xb + self.pp_adjoint(xf, abar)
        return xb

    def deposit_adjoint(self, xf, rhobar, level=None):
        """x-bar of the unit-mass density of the finest level for rhobar."""
        if level is None:
            level = len(self.p.levels()) - 1
        H, n, _, _ = self.p.levels()[level]
        xf = np.ascontiguousarray(xf, dtype=np.float64)
        xbar = np.zeros((3, xf.shape[1]))
        dep_pos = lib().orc_deposit_adjoint_pos_tsc if self.p.assign == 3 else \
            lib().orc_deposit_adjoint_pos
        dep_pos(xf.shape[1], _p(xf), int(n), float(H), int(self.quant),
                _p(np.ascontiguousarray(rhobar, dtype=np.float64)), _p(xbar))
        return xbar


# ---------------------------------------------------------------------------
# Tile+buffer mode (section 2.2.3, PM2 paragraph)
# ---------------------------------------------------------------------------

def tile_local_accel(params: Params, xf: np.ndarray, origin, tile: int, buffer: int,
                     workers: int = 1):
    """Fine-level + PP acceleration of the particles of one tile computed on
    the local periodic box of the tile and a buffer zone around it.

    The box of fine cells [origin - buffer, origin + tile + buffer) (periodic
    in the global box) holds the local particles; in their local coordinates
    (shifted by origin - buffer) the finer level of the two-level split, whose
    target force R(r, b_fine) - R(r, b_coarse) is truncated at b_coarse, and
    the PP sum are evaluated with periodic boundaries on the local box of
    tile + 2 buffer cells.  Returns (indices of the tile's own particles in
    xf, their acceleration (3, k)); the coarse level is the global one."""
    xf = np.asarray(xf, dtype=np.float64)
    L = float(params.n_fine)
    o = np.asarray(origin, dtype=np.float64).reshape(3, 1)
    rel = np.mod(xf - (o - buffer), L)
    n_local = tile + 2 * buffer
    inb = np.all(rel < n_local, axis=0)
    own = np.all((rel >= buffer) & (rel < buffer + tile), axis=0)
    xl = np.ascontiguousarray(rel[:, inb])
    pl = Params(n_fine=n_local, coarse_ratio=params.coarse_ratio, b_coarse=params.b_coarse,
                b_fine=params.b_fine, b_pp=params.b_pp, m_p=params.m_p, G_N=params.G_N,
                alias_nmax=params.alias_nmax, assign=params.assign)
    ol = Oracle(pl, workers=workers)
    a = ol.pm_level_accel(xl, 1) + ol.pp_accel(xl)
    return np.nonzero(own)[0], a[:, own[inb]]


def pm3_local_accel(params: Params, xf: np.ndarray, origin, tile: int, buffer: int, h3: float,
                    beta3: float = 3.5, workers: int = 1):
    """PM3 level and its PP of the particles of one subtile (section 2.2.3,
    PM3 paragraph; eqs. 4c and 4d with three levels).

    On the local periodic box of the subtile and a buffer, a mesh of spacing
    H3 = h3 fine cells carries the level whose target force is R(r, b3) -
    R(r, b2), softening b3 = beta3 H3 truncated at the fine level's softening
    b2 = params.b_fine, and the PP sum with softening b_pp is cut at b3.  It
    is the tile computation of tile_local_accel in units of H3 cells (eq. 2
    is homogeneous of degree -2: R(r / H, b / H) = H^2 R(r, b)), scaled back
    to fine-cell units.  Returns (indices of the subtile's own particles,
    their PM3 + PP acceleration)."""
    scaled = Params(n_fine=int(round(params.n_fine / h3)), coarse_ratio=params.coarse_ratio,
                    b_coarse=params.b_fine / h3, b_fine=beta3, b_pp=params.b_pp / h3,
                    m_p=params.m_p, G_N=params.G_N, alias_nmax=params.alias_nmax,
                    assign=params.assign)
    o = [int(round(v / h3)) for v in origin]
    idx, a = tile_local_accel(scaled, np.asarray(xf, dtype=np.float64) / h3, o,
                              int(round(tile / h3)), int(round(buffer / h3)), workers)
    return idx, a / (h3 * h3)


# ---------------------------------------------------------------------------
# IOS velocities (section 2.3)
# ---------------------------------------------------------------------------
#
# The paper stores each velocity component as a short integer relative to a
# bulk velocity field on a mesh and defers the conversion formula to an
# earlier paper.  Reading used here (linear), written out plainly in FP64:
# the bulk velocity of a cell is the mean velocity of its particles (0 for an
# empty cell), one global step s = max |v - v_bulk| / 32767, the code is
# q = rint((v - v_bulk) / s) clamped to +-32767 as int16, and the decoded
# velocity is v_bulk + s q.  Parity of this step is defined by this reading
# only (no formula in the paper to pin it to); its pins are the round-trip
# bound, the cell means and the invariances.

def _bulk_key(q: np.ndarray, n_fine: int, shift: int) -> np.ndarray:
    nb = n_fine >> shift
    cell = (np.asarray(q, dtype=np.int64) >> 15) >> shift
    return (cell[2] * nb + cell[1]) * nb + cell[0]


def vel_encode(q: np.ndarray, v: np.ndarray, n_fine: int, shift: int):
    """(vq int16 (3, N), v_bulk float64 (3, nb, nb, nb), s float64, r float64
    (3, N)) for IOS positions q (int64, units of 2^-15 fine cells) and
    velocities v, bulk cells of 2^shift fine cells (nb = n_fine >> shift);
    r = (v - v_bulk) / s is the unrounded code."""
    v = np.asarray(v, dtype=np.float64)
    nb = n_fine >> shift
    key = _bulk_key(q, n_fine, shift)
    N = v.shape[1]
    cnt = np.bincount(key, minlength=nb ** 3)
    has = cnt > 0
    vb = np.zeros((3, nb ** 3))
    for d in range(3):
        sums = np.bincount(key, weights=v[d], minlength=nb ** 3)
        vb[d, has] = sums[has] / cnt[has]
    dev = v - vb[:, key]
    m = float(np.abs(dev).max()) if N else 0.0
    s = m / 32767.0 if m > 0 else 1.0
    r = dev / s
    vq = np.clip(np.rint(r), -32767, 32767).astype(np.int16)
    return vq, vb.reshape(3, nb, nb, nb), s, r


def vel_decode(q: np.ndarray, vq: np.ndarray, v_bulk: np.ndarray, s, n_fine: int, shift: int):
    """v = v_bulk(cell) + s q (FP64)."""
    key = _bulk_key(q, n_fine, shift)
    vb = np.asarray(v_bulk, dtype=np.float64).reshape(3, -1)[:, key]
    return vb + float(s) * np.asarray(vq, dtype=np.int16).astype(np.float64)


# ---------------------------------------------------------------------------
# Time stepping (leapfrog kick-drift, sections 2.2.3 and 2.3)
# ---------------------------------------------------------------------------

def kick_drift_q(q: np.ndarray, v: np.ndarray, a: np.ndarray, kick: float, drift: float,
                 n_fine: int):
    """One kick-drift step on integer positions.

    v' = v + kick * a (FP64, stored FP32); q' = q + rint(drift * v' * 2^15)
    (round half to even), wrapped into [0, n_fine * 2^15).
    Velocities are in fine cells per unit time.
    """
    v64 = v.astype(np.float64) + float(kick) * a.astype(np.float64)
    v32 = v64.astype(np.float32)
    dq = np.rint(float(drift) * v64 * float(1 << FRAC_BITS)).astype(np.int64)
    span = n_fine << FRAC_BITS
    return np.mod(q + dq, span), v32


def ewald_accel(xf: np.ndarray, L: float, alpha: float | None = None, n_real: int = 2,
                n_k: int = 12) -> np.ndarray:
    """Periodic 1/r^2 acceleration of unit point masses by Ewald summation.

    Textbook Ewald split with a neutralising background (no k = 0 term):
      a_i = sum_j sum_n [erfc(a r)/r^2 + 2a/sqrt(pi) exp(-a^2 r^2)/r] r_hat
          + (4 pi / V) sum_{k != 0} k/k^2 exp(-k^2/4a^2) sin(k . (x_j - x_i)),
    with r = x_j - x_i + n L.  For small N (it is O(N^2)).
    """
    from scipy.special import erfc
    xf = np.asarray(xf, dtype=np.float64)
    N = xf.shape[1]
    if alpha is None:
        alpha = 4.0 / L
    acc = np.zeros((3, N))
    D = xf[:, None, :] - xf[:, :, None]           # D[:, i, j] = x_j - x_i
    rng_ = range(-n_real, n_real + 1)
    for a0 in rng_:
        for a1 in rng_:
            for a2 in rng_:
                s = np.array([a0, a1, a2], dtype=np.float64)[:, None, None] * L
                R = D + s
                r = np.sqrt(np.sum(R * R, axis=0))
                with np.errstate(divide="ignore", invalid="ignore"):
                    f = (erfc(alpha * r) / r ** 2
                         + 2 * alpha / math.sqrt(math.pi) * np.exp(-(alpha * r) ** 2) / r) / r
                f[r == 0.0] = 0.0
                acc += np.sum(f[None] * R, axis=2)
    V = L ** 3
    ks = np.arange(-n_k, n_k + 1)
    kz, ky, kx = np.meshgrid(ks, ks, ks, indexing="ij")
    kv = np.stack([kx.ravel(), ky.ravel(), kz.ravel()]).astype(np.float64) * (2 * math.pi / L)
    k2 = np.sum(kv * kv, axis=0)
    keep = k2 > 0
    kv, k2 = kv[:, keep], k2[keep]
    coef = 4 * math.pi / V * np.exp(-k2 / (4 * alpha ** 2)) / k2
    phase = kv.T @ xf                              # (K, N)
    c, s = np.cos(phase), np.sin(phase)
    Sc, Ss = c.sum(axis=1), s.sum(axis=1)          # structure factor
    # sum_j sin(k.(x_j - x_i)) = Ss cos(k.x_i) - Sc sin(k.x_i)
    t = coef[:, None] * (Ss[:, None] * c - Sc[:, None] * s)   # (K, N)
    acc += kv @ t
    return acc


def reference_accel(xf: np.ndarray, params: Params) -> np.ndarray:
    """Exact periodic force of softened particles R(r, b_pp) (eq. 3 total).

    Ewald sum of point masses plus the softening correction
    [R(r, b_pp) - 1/r^2] r_hat for the (minimum-image) pairs with r < b_pp.
    """
    L = float(params.n_fine)
    acc = ewald_accel(xf, L)
    xf = np.asarray(xf, dtype=np.float64)
    D = xf[:, None, :] - xf[:, :, None]
    D = D - L * np.round(D / L)
    r = np.sqrt(np.sum(D * D, axis=0))
    N = xf.shape[1]
    for i in range(N):
        for j in range(N):
            if i != j and 0 < r[i, j] < params.b_pp:
                rr = r[i, j]
                acc[:, i] += (refforce(rr, params.b_pp) - 1.0 / rr ** 2) * D[:, i, j] / rr
    return acc * (params.G_N * params.m_p)


# ---------------------------------------------------------------------------
# Multi-step leapfrog and its gradient (continuous FP64 positions)
# ---------------------------------------------------------------------------

def leapfrog_states(o: "Oracle", x0f: np.ndarray, v0: np.ndarray, kick: float, drift: float,
                    steps: int):
    """States of `steps` kick-drift steps: x_{k+1} = x_k + drift v_{k+1},
    v_{k+1} = v_k + kick a(x_k); positions wrap into [0, n_fine)."""
    L = float(o.p.n_fine)
    xs, vs = [np.array(x0f, dtype=np.float64)], [np.array(v0, dtype=np.float64)]
    for _ in range(steps):
        a = o.accel(xs[-1])
        v = vs[-1] + kick * a
        xs.append(np.mod(xs[-1] + drift * v, L))
        vs.append(v)
    return xs, vs


def leapfrog_loss(o: "Oracle", x0f, v0, kick, drift, steps, rho_target):
    """Loss sum (rho_final - rho_target)^2 on the finest level, unit masses."""
    xs, _ = leapfrog_states(o, x0f, v0, kick, drift, steps)
    H, n, _, _ = o.p.levels()[-1]
    rho = deposit(xs[-1], n, H, o.quant)
    return float(np.sum((rho - rho_target) ** 2))


def leapfrog_loss_grad(o: "Oracle", x0f, v0, kick, drift, steps, rho_target):
    """(loss, d loss/d x0, d loss/d v0) by reverse mode through the steps:
    given (xbar, vbar) after step k+1:  vbar += drift * xbar,
    xbar_k = xbar + (da/dx)^T (kick * vbar), vbar_k = vbar."""
    xs, vs = leapfrog_states(o, x0f, v0, kick, drift, steps)
    H, n, _, _ = o.p.levels()[-1]
    rho = deposit(xs[-1], n, H, o.quant)
    loss = float(np.sum((rho - rho_target) ** 2))
    rhobar = 2.0 * (rho - rho_target)
    xbar = o.deposit_adjoint(xs[-1], rhobar)
    vbar = np.zeros_like(xbar)
    for k in range(steps - 1, -1, -1):
        vbar = vbar + drift * xbar
        xbar = xbar + o.accel_adjoint(xs[k], kick * vbar)
    return loss, xbar, vbar


def leapfrog_grad_on_states(o: "Oracle", xs, kick: float, drift: float, rho_target):
    """Reverse mode of the same loss along a given trajectory xs[0..K]
    (positions in one consistent particle order, fine cells); the map is
    linear in the velocities, so only positions are needed."""
    H, n, _, _ = o.p.levels()[-1]
    rho = deposit(xs[-1], n, H, o.quant)
    xbar = o.deposit_adjoint(xs[-1], 2.0 * (rho - rho_target))
    vbar = np.zeros_like(xbar)
    for k in range(len(xs) - 2, -1, -1):
        vbar = vbar + drift * xbar
        xbar = xbar + o.accel_adjoint(xs[k], kick * vbar)
    return xbar, vbar
