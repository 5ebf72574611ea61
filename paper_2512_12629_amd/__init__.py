"""MI355X (gfx950) implementation of the CUBE2 force computation.

Two-level particle-mesh + particle-particle gravity of Yu et al.,
arXiv 2512.12629 (section 2.1), with leapfrog kick-drift on integer in-cell
positions (section 2.3) and hand-written adjoints, as a C-ABI HIP library
(include/cube2.h, built into _build/libcube2.so).  This module is the thin
Python binding: the ``cube2_*`` functions take torch tensors and pass their
device pointers and the current HIP stream through; all arithmetic runs in
the library's kernels.  There is no CPU fallback: importing raises if the
library has not been built (``python -m paper_2512_12629_amd.build``).

Tensor conventions (device tensors, SoA over particles):
  x      float32 (3, N) box units in [0, 1)      (cube2_pack input)
  pos    int16   (3, N) in-cell offsets (uint16 bits)
  cs     int32   ((n_fine/2)^3 + 1,) cell_start (uint32 bits)
  perm   int32   (N,)
  vel, acc, x_bar, acc_bar  float32 (3, N), fine cells per time unit(s)
  meshes float32 (n, n, n) [z][y][x]
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libcube2.so")

CUBE2_PP_OFF = 1
CUBE2_FP64_FORM = 2
CUBE2_ASSIGN_TSC = 4
CUBE2_ISOLATED = 8
_ERRORS = {0: "ok", -1: "invalid argument", -2: "unsupported configuration",
           -3: "tables or work buffer too small", -4: "deposit overflow guard",
           -5: "HIP runtime error", -6: "tables not initialised",
           -7: "non-finite kick-drift"}


class Cube2Error(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_ERRORS.get(code, code)} ({code})")
        self.code = code


class cube2_config(ctypes.Structure):
    _fields_ = [("n_fine", ctypes.c_int32), ("coarse_ratio", ctypes.c_int32),
                ("b_coarse", ctypes.c_double), ("b_fine", ctypes.c_double),
                ("b_pp", ctypes.c_double), ("m_p", ctypes.c_double),
                ("g_newton", ctypes.c_double), ("alias_nmax", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libcube2.so not built ({LIB_PATH}); run `python -m paper_2512_12629_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sigs = {
        "cube2_create": [ctypes.POINTER(cube2_config), ctypes.POINTER(P)],
        "cube2_destroy": [P],
        "cube2_sizes": [P, I64, ctypes.POINTER(S), ctypes.POINTER(S)],
        "cube2_level_shape": [P, I, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
        "cube2_self_check": [P, I64],
        "cube2_init_tables": [P, P, S, P],
        "cube2_green_table": [P, I, P, P],
        "cube2_pack": [P, P, I64, P, P, P, P, S, P],
        "cube2_deposit": [P, P, P, I64, I, P, P, P, S, P],
        "cube2_fft_r2c": [P, I, P, P, P, S, P],
        "cube2_potential": [P, I, P, P, P, S, P],
        "cube2_interp": [P, P, P, I64, P, P, P, I, P],
        "cube2_pm_force": [P, P, P, I64, P, I, P, S, P],
        "cube2_pp_force": [P, P, P, I64, P, I, P, S, P],
        "cube2_pm_level_force": [P, P, P, I64, I, P, I, P, S, P],
        "cube2_pp_force_noalloc": [P, P, P, I64, P, I, P],
        "cube2_tile_gather": [P, P, P, I64, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                              ctypes.c_int32, ctypes.c_int32, P, P, I64, ctypes.POINTER(I64), P,
                              S, P],
        "cube2_tile_scatter_add": [I64, P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_float, P, P, I64, P],
        "cube2_pp_force_skip": [P, P, P, I64, P, P, I, P, S, P],
        "cube2_force": [P, P, P, I64, P, P, S, P],
        "cube2_force_backward": [P, P, P, I64, P, P, I, P, S, P],
        "cube2_kick_drift": [P, P, P, P, P, I64, D, D, P, P, P, P, P, S, P],
        "cube2_reduce": [P, P, P, I64, ctypes.POINTER(D), P, S, P],
        "cube2_status": [P, P],
        "cube2_vel_bulk_side": [P, ctypes.POINTER(I)],
        "cube2_vel_encode": [P, P, P, I64, P, P, P, P, P, S, P],
        "cube2_vel_decode": [P, P, P, I64, P, P, P, P, P],
        "cube2_deposit_backward": [P, P, P, I64, I, P, P, I, P, S, P],
        "cube2_pm_force_backward": [P, P, P, I64, P, P, I, P, S, P],
        "cube2_pp_force_backward": [P, P, P, I64, P, P, I, P, S, P],
        "cube2_kick_drift_backward": [P, I64, P, P, P, D, D, P, P, P, P],
        "cube2_potential_f64": [P, I, P, P, P, S, P],
        "cube2_pm_force_f64": [P, P, P, I64, P, I, P, S, P],
        "cube2_pp_force_f64": [P, P, P, I64, P, I, P, S, P],
        "cube2_pair_law_f32": [P, P, P, I64],
        "cube2_pair_jacobian_f32": [P, P, P, P, I64],
        "cube2_strerror": [I],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = None if name == "cube2_destroy" else (
            ctypes.c_char_p if name == "cube2_strerror" else ctypes.c_int)
    return L


_lib = _load()


def lib():
    return _lib


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(code, what):
    if code != 0:
        raise Cube2Error(code, what)


# ---------------------------------------------------------------------------
# Same-name wrappers of the C ABI (argument marshalling only)
# ---------------------------------------------------------------------------

def cube2_create(cfg: cube2_config):
    h = ctypes.c_void_p()
    _check(_lib.cube2_create(ctypes.byref(cfg), ctypes.byref(h)), "cube2_create")
    return h


def cube2_destroy(ctx):
    _lib.cube2_destroy(ctx)


def cube2_sizes(ctx, n_max: int):
    tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.cube2_sizes(ctx, int(n_max), ctypes.byref(tb), ctypes.byref(wb)), "cube2_sizes")
    return tb.value, wb.value


def cube2_self_check(ctx, n_max: int) -> int:
    """Host-only layout/index check of the context (returns the status code)."""
    return _lib.cube2_self_check(ctx, int(n_max))


def cube2_level_shape(ctx, level: int):
    n, p = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.cube2_level_shape(ctx, int(level), ctypes.byref(n), ctypes.byref(p)),
           "cube2_level_shape")
    return n.value, p.value


def cube2_init_tables(ctx, tables, stream=None):
    _check(_lib.cube2_init_tables(ctx, _ptr(tables), tables.numel() * tables.element_size(),
                                  _stream(stream)), "cube2_init_tables")


def cube2_green_table(ctx, level, out, stream=None):
    _check(_lib.cube2_green_table(ctx, int(level), _ptr(out), _stream(stream)), "cube2_green_table")


def cube2_pack(ctx, x, pos, cell_start, perm, work, stream=None):
    _check(_lib.cube2_pack(ctx, _ptr(x), x.shape[1], _ptr(pos), _ptr(cell_start), _ptr(perm),
                           _ptr(work), work.numel(), _stream(stream)), "cube2_pack")


def cube2_deposit(ctx, pos, cell_start, level, rho, rho_fx, work, stream=None):
    _check(_lib.cube2_deposit(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], int(level),
                              _ptr(rho), _ptr(rho_fx), _ptr(work), work.numel(), _stream(stream)),
           "cube2_deposit")


def cube2_fft_r2c(ctx, level, mesh, spec, work, stream=None):
    _check(_lib.cube2_fft_r2c(ctx, int(level), _ptr(mesh), _ptr(spec), _ptr(work), work.numel(),
                              _stream(stream)), "cube2_fft_r2c")


def cube2_potential(ctx, level, rho, phi, work, stream=None):
    _check(_lib.cube2_potential(ctx, int(level), _ptr(rho), _ptr(phi), _ptr(work), work.numel(),
                                _stream(stream)), "cube2_potential")


def cube2_interp(ctx, pos, cell_start, phi_fine, phi_coarse, acc, accumulate=False, stream=None):
    _check(_lib.cube2_interp(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], _ptr(phi_fine),
                             _ptr(phi_coarse), _ptr(acc), int(bool(accumulate)), _stream(stream)),
           "cube2_interp")


def cube2_pm_force(ctx, pos, cell_start, acc, work, accumulate=False, stream=None):
    _check(_lib.cube2_pm_force(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], _ptr(acc),
                               int(bool(accumulate)), _ptr(work), work.numel(), _stream(stream)),
           "cube2_pm_force")


def cube2_pm_level_force(ctx, pos, cell_start, level, acc, work, accumulate=False, stream=None):
    _check(_lib.cube2_pm_level_force(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], int(level),
                                     _ptr(acc), int(bool(accumulate)), _ptr(work), work.numel(),
                                     _stream(stream)), "cube2_pm_level_force")


def cube2_tile_gather(ctx, pos, cell_start, origins, tile, buffer, x_local, idx, work,
                      stream=None):
    """Gathers the particles of the tiles at `origins` (a list of (x, y, z)
    fine-cell origins) with their buffers into one packed box; returns their
    number m.  x_local holds (3, m) at its front and idx m entries, unless
    m > idx.numel(), when nothing is written (the caller grows its buffers
    and calls again)."""
    flat = [int(v) for o in origins for v in o]
    o = (ctypes.c_int32 * len(flat))(*flat)
    m = ctypes.c_int64()
    code = _lib.cube2_tile_gather(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], o,
                                  len(flat) // 3, int(tile), int(buffer), _ptr(x_local),
                                  _ptr(idx), idx.numel(), ctypes.byref(m), _ptr(work),
                                  work.numel(), _stream(stream))
    if code != -3:
        _check(code, "cube2_tile_gather")
    return m.value


def cube2_tile_scatter_add(perm_local, x_local, idx, n_tiles, tile, buffer, acc_local, acc,
                           scale=1.0, stream=None):
    m = perm_local.shape[0]
    _check(_lib.cube2_tile_scatter_add(m, _ptr(perm_local), _ptr(x_local), _ptr(idx),
                                       int(n_tiles), int(tile), int(buffer), float(scale),
                                       _ptr(acc_local), _ptr(acc), acc.shape[1],
                                       _stream(stream)), "cube2_tile_scatter_add")


def cube2_pp_force_skip(ctx, pos, cell_start, skip_tiles, acc, work, accumulate=False,
                        stream=None):
    _check(_lib.cube2_pp_force_skip(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1],
                                    _ptr(skip_tiles), _ptr(acc), int(bool(accumulate)),
                                    _ptr(work), work.numel(), _stream(stream)),
           "cube2_pp_force_skip")


def cube2_force(ctx, pos, cell_start, acc, work, stream=None):
    _check(_lib.cube2_force(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], _ptr(acc),
                            _ptr(work), work.numel(), _stream(stream)), "cube2_force")


def cube2_force_backward(ctx, pos, cell_start, acc_bar, x_bar, work, accumulate=False,
                         stream=None):
    _check(_lib.cube2_force_backward(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1],
                                     _ptr(acc_bar), _ptr(x_bar), int(bool(accumulate)),
                                     _ptr(work), work.numel(), _stream(stream)),
           "cube2_force_backward")


def cube2_pp_force(ctx, pos, cell_start, acc, work, accumulate=False, stream=None):
    _check(_lib.cube2_pp_force(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], _ptr(acc),
                               int(bool(accumulate)), _ptr(work), work.numel(), _stream(stream)),
           "cube2_pp_force")


def cube2_pp_force_noalloc(ctx, pos, cell_start, acc, accumulate=False, stream=None):
    _check(_lib.cube2_pp_force_noalloc(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], _ptr(acc),
                                       int(bool(accumulate)), _stream(stream)),
           "cube2_pp_force_noalloc")


def cube2_kick_drift(ctx, pos_in, cs_in, vel_in, acc, kick, drift, pos_out, cs_out, vel_out,
                     perm_out, work, stream=None):
    _check(_lib.cube2_kick_drift(ctx, _ptr(pos_in), _ptr(cs_in), _ptr(vel_in), _ptr(acc),
                                 pos_in.shape[1], float(kick), float(drift), _ptr(pos_out),
                                 _ptr(cs_out), _ptr(vel_out), _ptr(perm_out), _ptr(work),
                                 work.numel(), _stream(stream)), "cube2_kick_drift")


def cube2_reduce(ctx, vel, acc, work, stream=None):
    out = (ctypes.c_double * 8)()
    _check(_lib.cube2_reduce(ctx, _ptr(vel), _ptr(acc), acc.shape[1], out, _ptr(work),
                             work.numel(), _stream(stream)), "cube2_reduce")
    return list(out)


def cube2_vel_bulk_side(ctx):
    side = ctypes.c_int()
    _check(_lib.cube2_vel_bulk_side(ctx, ctypes.byref(side)), "cube2_vel_bulk_side")
    return side.value


def cube2_vel_encode(ctx, pos, cs, vel, vq, v_bulk, v_scale, work, stream=None):
    _check(_lib.cube2_vel_encode(ctx, _ptr(pos), _ptr(cs), pos.shape[1], _ptr(vel), _ptr(vq),
                                 _ptr(v_bulk), _ptr(v_scale), _ptr(work), work.numel(),
                                 _stream(stream)), "cube2_vel_encode")


def cube2_vel_decode(ctx, pos, cs, vq, v_bulk, v_scale, vel, stream=None):
    _check(_lib.cube2_vel_decode(ctx, _ptr(pos), _ptr(cs), pos.shape[1], _ptr(vq), _ptr(v_bulk),
                                 _ptr(v_scale), _ptr(vel), _stream(stream)), "cube2_vel_decode")


def cube2_status(ctx, stream=None):
    return _lib.cube2_status(ctx, _stream(stream))


def cube2_deposit_backward(ctx, pos, cell_start, level, rho_bar, x_bar, work, accumulate=False,
                           stream=None):
    _check(_lib.cube2_deposit_backward(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], int(level),
                                       _ptr(rho_bar), _ptr(x_bar), int(bool(accumulate)),
                                       _ptr(work), work.numel(), _stream(stream)),
           "cube2_deposit_backward")


def cube2_pm_force_backward(ctx, pos, cell_start, acc_bar, x_bar, work, accumulate=False,
                            stream=None):
    _check(_lib.cube2_pm_force_backward(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1],
                                        _ptr(acc_bar), _ptr(x_bar), int(bool(accumulate)),
                                        _ptr(work), work.numel(), _stream(stream)),
           "cube2_pm_force_backward")


def cube2_pp_force_backward(ctx, pos, cell_start, acc_bar, x_bar, work, accumulate=False,
                            stream=None):
    _check(_lib.cube2_pp_force_backward(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1],
                                        _ptr(acc_bar), _ptr(x_bar), int(bool(accumulate)),
                                        _ptr(work), work.numel(), _stream(stream)),
           "cube2_pp_force_backward")


def cube2_kick_drift_backward(ctx, perm, xbar_out, vbar_out, kick, drift, xbar_in, vbar_in,
                              acc_bar, stream=None):
    _check(_lib.cube2_kick_drift_backward(ctx, perm.shape[0], _ptr(perm), _ptr(xbar_out),
                                          _ptr(vbar_out), float(kick), float(drift),
                                          _ptr(xbar_in), _ptr(vbar_in), _ptr(acc_bar),
                                          _stream(stream)), "cube2_kick_drift_backward")


def cube2_potential_f64(ctx, level, rho, phi, work, stream=None):
    _check(_lib.cube2_potential_f64(ctx, int(level), _ptr(rho), _ptr(phi), _ptr(work),
                                    work.numel(), _stream(stream)), "cube2_potential_f64")


def cube2_pm_force_f64(ctx, pos, cell_start, acc, work, accumulate=False, stream=None):
    _check(_lib.cube2_pm_force_f64(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], _ptr(acc),
                                   int(bool(accumulate)), _ptr(work), work.numel(),
                                   _stream(stream)), "cube2_pm_force_f64")


def cube2_pp_force_f64(ctx, pos, cell_start, acc, work, accumulate=False, stream=None):
    _check(_lib.cube2_pp_force_f64(ctx, _ptr(pos), _ptr(cell_start), pos.shape[1], _ptr(acc),
                                   int(bool(accumulate)), _ptr(work), work.numel(),
                                   _stream(stream)), "cube2_pp_force_f64")


def cube2_pair_law_f32(ctx, d):
    """g for the separations d (numpy float32 (3, n), fine cells), evaluated
    on the host exactly as the FP32 forward PP kernel does."""
    import numpy as np
    d = np.ascontiguousarray(d, dtype=np.float32)
    n = d.shape[1]
    g = np.empty(n, dtype=np.float32)
    _check(_lib.cube2_pair_law_f32(ctx, d.ctypes.data_as(ctypes.c_void_p),
                                   g.ctypes.data_as(ctypes.c_void_p), n), "cube2_pair_law_f32")
    return g


def cube2_pair_jacobian_f32(ctx, d):
    """(g, dg/ds) for the separations d (numpy float32 (3, n)), evaluated on
    the host exactly as the FP32 PP adjoint kernel does."""
    import numpy as np
    d = np.ascontiguousarray(d, dtype=np.float32)
    n = d.shape[1]
    g = np.empty(n, dtype=np.float32)
    gs = np.empty(n, dtype=np.float32)
    _check(_lib.cube2_pair_jacobian_f32(ctx, d.ctypes.data_as(ctypes.c_void_p),
                                        g.ctypes.data_as(ctypes.c_void_p),
                                        gs.ctypes.data_as(ctypes.c_void_p), n),
           "cube2_pair_jacobian_f32")
    return g, gs


def cube2_strerror(code: int) -> str:
    return _lib.cube2_strerror(int(code)).decode()


# ---------------------------------------------------------------------------
# Convenience object: owns the context, the tables and a work buffer
# ---------------------------------------------------------------------------

@dataclass
class Config:
    """Force parameters, lengths in fine cells (see include/cube2.h)."""
    n_fine: int
    coarse_ratio: int = 0
    b_coarse: float = 14.0
    b_fine: float = 2.0
    b_pp: float = 0.2
    m_p: float = 1.0
    g_newton: float = 1.0
    alias_nmax: int = 2
    flags: int = 0

    def c(self) -> cube2_config:
        return cube2_config(self.n_fine, self.coarse_ratio, self.b_coarse, self.b_fine, self.b_pp,
                            self.m_p, self.g_newton, self.alias_nmax, self.flags)


class Cube2:
    """Context + device tables + work buffer on one GPU."""

    def __init__(self, cfg: Config, n_max: int, device="cuda"):
        self.cfg = cfg
        self.device = torch.device(device)
        self.ctx = cube2_create(cfg.c())
        tb, wb = cube2_sizes(self.ctx, n_max)
        self.n_max = n_max
        self.tables = torch.empty(tb, dtype=torch.uint8, device=self.device)
        self.work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        cube2_init_tables(self.ctx, self.tables)
        self.n_cells = (cfg.n_fine // 2) ** 3
        self.levels = 2 if cfg.coarse_ratio else 1

    def __del__(self):
        try:
            if getattr(self, "ctx", None) is not None:
                cube2_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def level_shape(self, level):
        return cube2_level_shape(self.ctx, level)

    def _need(self, n):
        if n > self.n_max:
            raise ValueError(f"{n} particles > n_max {self.n_max}")

    # -- forward -------------------------------------------------------------
    def pack(self, x):
        n = x.shape[1]
        self._need(n)
        pos = torch.empty((3, n), dtype=torch.int16, device=self.device)
        cs = torch.empty(self.n_cells + 1, dtype=torch.int32, device=self.device)
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        cube2_pack(self.ctx, x.contiguous(), pos, cs, perm, self.work)
        return pos, cs, perm

    def deposit(self, pos, cs, level=0, fx=False):
        n, _ = self.level_shape(level)
        rho = torch.empty((n, n, n), dtype=torch.float32, device=self.device)
        rfx = torch.empty((n, n, n), dtype=torch.int64, device=self.device) if fx else None
        cube2_deposit(self.ctx, pos, cs, level, rho, rfx, self.work)
        return (rho, rfx) if fx else rho

    def fft_r2c(self, mesh, level=0):
        n, pitch = self.level_shape(level)
        spec = torch.empty((n, n, pitch, 2), dtype=torch.float32, device=self.device)
        cube2_fft_r2c(self.ctx, level, mesh.contiguous(), spec, self.work)
        return torch.view_as_complex(spec)[:, :, : n // 2 + 1]

    def potential(self, rho, level=0):
        phi = torch.empty_like(rho)
        cube2_potential(self.ctx, level, rho.contiguous(), phi, self.work)
        return phi

    def green_table(self, level=0):
        n, _ = self.level_shape(level)
        h = n // 2 + 1
        out = torch.empty((h, h, h), dtype=torch.float32, device=self.device)
        cube2_green_table(self.ctx, level, out)
        return out

    def interp(self, pos, cs, phi_f, phi_c=None, acc=None):
        acc_out = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_interp(self.ctx, pos, cs, phi_f, phi_c, acc_out)
        return acc_out

    def pm_force(self, pos, cs, acc=None):
        accumulate = acc is not None
        if acc is None:
            acc = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_pm_force(self.ctx, pos, cs, acc, self.work, accumulate)
        return acc

    def pp_force(self, pos, cs, acc=None):
        accumulate = acc is not None
        if acc is None:
            acc = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_pp_force(self.ctx, pos, cs, acc, self.work, accumulate)
        return acc

    def force(self, pos, cs):
        acc = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_force(self.ctx, pos, cs, acc, self.work)
        return acc

    def pm_level_force(self, pos, cs, level, acc=None):
        accumulate = acc is not None
        if acc is None:
            acc = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_pm_level_force(self.ctx, pos, cs, level, acc, self.work, accumulate)
        return acc

    def kick_drift(self, pos, cs, vel, acc, kick, drift):
        n = pos.shape[1]
        pos2 = torch.empty_like(pos)
        cs2 = torch.empty_like(cs)
        vel2 = torch.empty_like(vel)
        perm = torch.empty(n, dtype=torch.int32, device=self.device)
        cube2_kick_drift(self.ctx, pos, cs, vel.contiguous(), acc.contiguous(), kick, drift, pos2,
                         cs2, vel2, perm, self.work)
        return pos2, cs2, vel2, perm

    def reduce(self, vel, acc):
        return cube2_reduce(self.ctx, vel, acc, self.work)

    def status(self):
        return cube2_status(self.ctx)

    # -- IOS velocities ---------------------------------------------------------
    def vel_encode(self, pos, cs, vel):
        """(vq int16 (3, n), v_bulk (3, nb, nb, nb), v_scale (1,)) of FP32 velocities."""
        nb = cube2_vel_bulk_side(self.ctx)
        vq = torch.empty((3, pos.shape[1]), dtype=torch.int16, device=self.device)
        vb = torch.empty((3, nb, nb, nb), dtype=torch.float32, device=self.device)
        sc = torch.empty(1, dtype=torch.float32, device=self.device)
        cube2_vel_encode(self.ctx, pos, cs, vel.contiguous(), vq, vb, sc, self.work)
        return vq, vb, sc

    def vel_decode(self, pos, cs, vq, v_bulk, v_scale):
        vel = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_vel_decode(self.ctx, pos, cs, vq.contiguous(), v_bulk.contiguous(), v_scale, vel)
        return vel

    # -- adjoints -------------------------------------------------------------
    def deposit_backward(self, pos, cs, rho_bar, level=0):
        xb = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_deposit_backward(self.ctx, pos, cs, level, rho_bar.contiguous(), xb, self.work)
        return xb

    def pm_force_backward(self, pos, cs, acc_bar, x_bar=None):
        accumulate = x_bar is not None
        if x_bar is None:
            x_bar = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_pm_force_backward(self.ctx, pos, cs, acc_bar.contiguous(), x_bar, self.work,
                                accumulate)
        return x_bar

    def force_backward(self, pos, cs, acc_bar, x_bar=None):
        """PM + PP adjoint (cube2_force_backward); adds to x_bar if given."""
        accumulate = x_bar is not None
        if x_bar is None:
            x_bar = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_force_backward(self.ctx, pos, cs, acc_bar.contiguous(), x_bar, self.work, accumulate)
        return x_bar

    def pp_force_backward(self, pos, cs, acc_bar, x_bar=None):
        accumulate = x_bar is not None
        if x_bar is None:
            x_bar = torch.empty((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        cube2_pp_force_backward(self.ctx, pos, cs, acc_bar.contiguous(), x_bar, self.work,
                                accumulate)
        return x_bar

    # -- FP64 plain form (context created with CUBE2_FP64_FORM) ---------------
    def potential_f64(self, rho, level=0):
        phi = torch.empty_like(rho, dtype=torch.float64)
        cube2_potential_f64(self.ctx, level, rho.to(torch.float64).contiguous(), phi, self.work)
        return phi

    def pm_force_f64(self, pos, cs, acc=None):
        accumulate = acc is not None
        if acc is None:
            acc = torch.empty((3, pos.shape[1]), dtype=torch.float64, device=self.device)
        cube2_pm_force_f64(self.ctx, pos, cs, acc, self.work, accumulate)
        return acc

    def pp_force_f64(self, pos, cs, acc=None):
        accumulate = acc is not None
        if acc is None:
            acc = torch.empty((3, pos.shape[1]), dtype=torch.float64, device=self.device)
        cube2_pp_force_f64(self.ctx, pos, cs, acc, self.work, accumulate)
        return acc

    def force_f64(self, pos, cs):
        acc = self.pm_force_f64(pos, cs)
        return self.pp_force_f64(pos, cs, acc)

    def kick_drift_backward(self, perm, xbar_out, vbar_out, kick, drift):
        xb = torch.empty_like(xbar_out)
        vb = torch.empty_like(vbar_out)
        ab = torch.empty_like(vbar_out)
        cube2_kick_drift_backward(self.ctx, perm, xbar_out.contiguous(), vbar_out.contiguous(),
                                  kick, drift, xb, vb, ab)
        return xb, vb, ab


class Cube2Tiled:
    """Tile+buffer force of a two-level configuration (section 2.2.3, PM2
    paragraph): the coarse level on the whole periodic box, the fine level and
    PP of each tile on a local periodic box of the tile plus a buffer, the
    results of the tile's own particles added in.  Every step is a C-ABI call;
    this class only owns the two contexts and loops over the tiles.

    tile, buffer: fine cells, even; tile divides n_fine and tile + 2 buffer is
    a power of two in [32, 512].  The buffer should be at least b_coarse + 3
    fine cells (the truncation plus the assignment and stencil reach)."""

    def __init__(self, cfg: Config, tile: int, buffer: int, n_max: int, device="cuda"):
        import dataclasses
        if not cfg.coarse_ratio:
            raise ValueError("the tile+buffer mode splits a two-level configuration")
        if cfg.n_fine % tile:
            raise ValueError("tiles must tile the box")
        self.tile, self.buffer = int(tile), int(buffer)
        self.n_local = self.tile + 2 * self.buffer
        self.g = Cube2(cfg, n_max, device)
        self.cfg_local = dataclasses.replace(cfg, n_fine=self.n_local)
        self.device = self.g.device
        self.local = None
        self.m_cap = 0

    def _local(self, m):
        if self.local is None or m > self.m_cap:
            self.m_cap = max(m, 1024)
            self.local = Cube2(self.cfg_local, self.m_cap, self.device)
            self.x_buf = torch.empty(3 * self.m_cap, dtype=torch.float32, device=self.device)
            self.i_buf = torch.empty(self.m_cap, dtype=torch.int32, device=self.device)
        return self.local

    def origins(self):
        k = self.g.cfg.n_fine // self.tile
        return [(x * self.tile, y * self.tile, z * self.tile)
                for z in range(k) for y in range(k) for x in range(k)]

    def tile_force(self, pos, cs, origin, acc):
        """Adds the fine-level + PP force of the particles of one tile to acc."""
        loc = self._local(1024)
        m = cube2_tile_gather(self.g.ctx, pos, cs, [origin], self.tile, self.buffer, self.x_buf,
                              self.i_buf, self.g.work)
        if m > self.m_cap:
            loc = self._local(m)
            m = cube2_tile_gather(self.g.ctx, pos, cs, [origin], self.tile, self.buffer,
                                  self.x_buf, self.i_buf, self.g.work)
        if m == 0:
            return
        xl = self.x_buf[:3 * m].view(3, m)
        pos_l, cs_l, perm_l = loc.pack(xl)
        a_l = loc.pm_level_force(pos_l, cs_l, 0)
        loc.pp_force(pos_l, cs_l, a_l)
        cube2_tile_scatter_add(perm_l, xl, self.i_buf[:m], 1, self.tile, self.buffer, a_l, acc)

    def force(self, pos, cs, origins=None):
        """Coarse level for every particle plus, for the tiles at `origins`
        (default: all), the fine level and PP of their own particles."""
        acc = self.g.pm_level_force(pos, cs, 1)
        for o in (self.origins() if origins is None else origins):
            self.tile_force(pos, cs, o, acc)
        return acc


class Cube2PM3:
    """Three-level force with an adaptive PM3 level on subtiles (section
    2.2.3, PM3 paragraph; eq. 4 with three levels): the coarse and fine PM
    levels on the whole box; for the selected tiles (the PP kernel's 16^3
    fine-cell tiles) a PM3 level of spacing H3 = h3 fine cells with softening
    b3 = beta3 H3, truncated at the fine softening b2, plus a PP sum cut at
    b3, computed on local boxes of the tile and a buffer (several tiles packed
    into one box); for the other tiles the PP sum cut at b2.  Every step is a
    C-ABI call (cube2_pm_force, cube2_pp_force_skip, cube2_tile_gather,
    cube2_pack / cube2_pm_level_force / cube2_pp_force on the PM3 context,
    cube2_tile_scatter_add with scale 1/H3^2).

    Which tiles get a PM3 level follows the paper's rule: the one that
    minimises t_PM3 + t_PP, from a cost model measured on the device
    (calibrate): the PP time per candidate pair of the b2 range, and the PM3
    time per particle of a packed box."""

    TILE = 16

    def __init__(self, cfg: Config, n_max: int, h3: float = 0.5, beta3: float = 3.5,
                 device="cuda", max_batch: int | None = None):
        import dataclasses
        self.max_batch = max_batch
        if not cfg.coarse_ratio:
            raise ValueError("the PM3 level sits below a two-level configuration")
        self.g = Cube2(cfg, n_max, device)
        self.device = self.g.device
        self.h3, self.beta3 = float(h3), float(beta3)
        self.scale = 1.0 / (self.h3 * self.h3)
        b2 = cfg.b_fine
        # buffer: at least b2 + 3 H3 (truncation plus assignment and stencil
        # reach), even, with a power-of-two slot of 32 fine cells or more
        self.buffer = 8
        while self.buffer < b2 + 3 * self.h3 or (self.TILE + 2 * self.buffer) & (
                self.TILE + 2 * self.buffer - 1):
            self.buffer += 2
        self.n_slot = self.TILE + 2 * self.buffer
        self.cfg3 = dataclasses.replace(cfg, n_fine=0, b_coarse=b2 / self.h3, b_fine=self.beta3,
                                        b_pp=cfg.b_pp / self.h3)
        self.nt = cfg.n_fine // self.TILE
        self._ctx3 = {}
        self.model = None

    def _pm3_ctx(self, k, m):
        key = k
        c, cap = self._ctx3.get(key, (None, 0))
        if c is None or m > cap:
            import dataclasses
            cap = max(m, 4096)
            n3 = int(round(k * self.n_slot / self.h3))
            c = Cube2(dataclasses.replace(self.cfg3, n_fine=n3), cap, self.device)
            self._ctx3[key] = (c, cap)
        return c

    def origins(self, tiles):
        nt = self.nt
        return [((t % nt) * self.TILE, (t // nt % nt) * self.TILE, (t // (nt * nt)) * self.TILE)
                for t in tiles]

    @staticmethod
    def _box_sum(grid, reach):
        """Sum over the (2 reach + 1)^3 box around every cell (periodic)."""
        for ax in range(3):
            acc = grid.clone()
            for r in range(1, reach + 1):
                acc += grid.roll(r, ax) + grid.roll(-r, ax)
            grid = acc
        return grid

    def tile_stats(self, pos, cs):
        """Per tile (index (tz nt + ty) nt + tx): particle count, candidate
        pairs of the PP sum at the b2 range (particles of each IOS cell times
        those of the IOS cells within its reach), and candidate pairs of the
        PM3 boxes' PP sum at the b3 range (the same on cells of 2 H3 fine
        cells, the PM3 box's IOS cells)."""
        nt, n_ios = self.nt, 8 * self.nt
        counts = cs[1:].long() - cs[:-1].long()
        cnt = counts.view(nt, nt, nt, 8, 8, 8)
        grid = cnt.permute(0, 3, 1, 4, 2, 5).reshape(n_ios, n_ios, n_ios).float()
        r2 = 1 if self.g.cfg.b_fine <= 2.0 else 2
        cand2 = (grid * self._box_sum(grid, r2)).view(nt, 8, nt, 8, nt, 8).sum((1, 3, 5))
        # cells of 2 H3 fine cells: the particle's fine position from its IOS
        # cell (tile-major key) and its offset, in units of 2 H3
        per = int(round(1.0 / (2.0 * self.h3)))          # PM3 IOS cells per fine cell
        nc3 = self.g.cfg.n_fine * per
        key = torch.repeat_interleave(torch.arange(counts.numel(), device=cs.device), counts)
        t, u = key // 512, key % 512
        cx = (t % nt) * 8 + u % 8
        cy = (t // nt % nt) * 8 + u // 8 % 8
        cz = (t // (nt * nt)) * 8 + u // 64
        off = pos.long() & 0xFFFF
        f = [((2 * c + (off[d] >> 15)) * per + ((off[d] & 0x7FFF) * per >> 15))
             for d, c in enumerate((cx, cy, cz))]
        g3 = torch.bincount((f[2] * nc3 + f[1]) * nc3 + f[0], minlength=nc3 ** 3).float()
        g3 = g3.view(nc3, nc3, nc3)
        r3 = 1 if self.beta3 <= 2.0 else 2
        c3 = 16 * per
        cand3 = (g3 * self._box_sum(g3, r3)).view(nt, c3, nt, c3, nt, c3).sum((1, 3, 5))
        return cnt.sum((3, 4, 5)).reshape(-1), cand2.reshape(-1), cand3.reshape(-1)

    def pm3_tiles(self, pos, cs, tiles, acc):
        """Adds the PM3 level + PP of the given tiles' particles to acc."""
        tiles = list(tiles)
        n = pos.shape[1]
        kmax = 1
        while kmax * 2 * self.n_slot <= 512 and (kmax * 2) ** 3 * (self.n_slot // 2) ** 3 <= \
                (self.nt * 8) ** 3:
            kmax *= 2
        per = kmax ** 3 if self.max_batch is None else max(1, min(kmax ** 3, self.max_batch))
        for b in range(0, len(tiles), per):
            batch = tiles[b:b + per]
            k = 1
            while k ** 3 < len(batch):
                k *= 2
            cap = max(4096, int(n))
            while True:   # buffers overlap, so a batch can hold more than n particles
                x_buf = torch.empty(3 * cap, dtype=torch.float32, device=self.device)
                i_buf = torch.empty(cap, dtype=torch.int32, device=self.device)
                m = cube2_tile_gather(self.g.ctx, pos, cs, self.origins(batch), self.TILE,
                                      self.buffer, x_buf, i_buf, self.g.work)
                if m <= cap:
                    break
                cap = m
            if m == 0:
                continue
            c3 = self._pm3_ctx(k, m)
            xl = x_buf[:3 * m].view(3, m)
            p3, cs3, perm3 = c3.pack(xl)
            a3 = c3.pm_level_force(p3, cs3, 0)
            c3.pp_force(p3, cs3, a3)
            cube2_tile_scatter_add(perm3, xl, i_buf[:m], len(batch), self.TILE, self.buffer, a3,
                                   acc, self.scale)

    def force(self, pos, cs, tiles=None):
        """Coarse + fine PM of every particle; PP cut at b2 for the tiles not
        in `tiles`; PM3 + PP cut at b3 for those in it (default: the model's
        choice, none before calibrate())."""
        if tiles is None:
            tiles = self.select(pos, cs) if self.model else []
        acc = self.g.pm_force(pos, cs)
        skip = torch.zeros(self.nt ** 3, dtype=torch.uint8, device=self.device)
        if len(tiles):
            skip[torch.as_tensor(list(tiles), dtype=torch.long, device=self.device)] = 1
        cube2_pp_force_skip(self.g.ctx, pos, cs, skip, acc, self.g.work, accumulate=True)
        if len(tiles):
            self.pm3_tiles(pos, cs, tiles, acc)
        return acc

    def calibrate(self, pos, cs, trial=64, reps=3):
        """Measures the cost model on the device: the b2-range PP time per
        candidate pair (the whole PP sum), and the PM3 time of two packed
        batches of `trial` tiles each (the heaviest tiles, and tiles from the
        middle of the occupied ones), fitted as t = c_tile n_tiles + c_pp3
        (their b3-range candidates): the mesh time per tile and the PM3 box's
        PP time per candidate.  Kept for select()."""
        import numpy as np
        count, cand2, cand3 = self.tile_stats(pos, cs)
        stream = torch.cuda.current_stream()

        def timed(fn):
            ts = []
            for _ in range(reps + 1):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                a.record(stream)
                fn()
                b.record(stream)
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b))
            return float(np.median(ts[1:])) * 1e-3

        acc = torch.zeros((3, pos.shape[1]), dtype=torch.float32, device=self.device)
        t_pp = timed(lambda: self.g.pp_force(pos, cs, acc))
        c_pp = t_pp / max(float(cand2.sum()), 1.0)
        order = torch.argsort(count, descending=True)
        occupied = int((count > 0).sum())
        sets = [order[:trial], order[max(0, occupied // 2 - trial // 2):][:trial]]
        rows, ts = [], []
        for sset in sets:
            tl = sset.tolist()
            ts.append(timed(lambda: self.pm3_tiles(pos, cs, tl, acc)))
            rows.append([float(len(tl)), float(cand3[sset].sum())])
        A, t = np.array(rows), np.array(ts)
        try:
            c_tile, c_pp3 = np.linalg.solve(A, t)
        except np.linalg.LinAlgError:
            c_tile, c_pp3 = -1.0, -1.0
        if not (c_tile > 0 and c_pp3 > 0):       # ill-conditioned: the PP rate of the sum
            c_pp3 = c_pp
            c_tile = max((t[0] - c_pp3 * A[0, 1]) / A[0, 0], t[1] / A[1, 0], 1e-9)
        self.model = {"pp_s_per_candidate": c_pp, "pm3_pp_s_per_candidate": float(c_pp3),
                      "pm3_s_per_tile": float(c_tile), "t_pp_s": t_pp,
                      "t_pm3_trials_s": ts, "trial_tiles": trial}
        return self.model

    def predicted_change(self, pos, cs, tiles):
        """The model's change of the force time (s) when `tiles` get PM3."""
        _, cand2, cand3 = self.tile_stats(pos, cs)
        t = torch.as_tensor(list(tiles), dtype=torch.long, device=cand2.device)
        md = self.model
        return (md["pm3_s_per_tile"] * len(tiles) + md["pm3_pp_s_per_candidate"] * float(
            cand3[t].sum()) - md["pp_s_per_candidate"] * float(cand2[t].sum()))

    def select(self, pos, cs):
        """Tiles whose predicted b2-range PP time exceeds their predicted
        PM3 time (mesh time per tile plus the PP at the b3 range): the rule
        of the paper (minimal t_PM3 + t_PP per subtile), with the costs
        measured by calibrate()."""
        _, cand2, cand3 = self.tile_stats(pos, cs)
        md = self.model
        gain = (md["pp_s_per_candidate"] * cand2 - md["pm3_pp_s_per_candidate"] * cand3
                - md["pm3_s_per_tile"])
        return torch.nonzero(gain > 0).flatten().tolist()
