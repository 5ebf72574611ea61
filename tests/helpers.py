"""Shared test helpers: parameter sets, error statistics, IOS decoding."""
from __future__ import annotations

import numpy as np

TILE = 8


def ios_decode(pos: np.ndarray, cs: np.ndarray, n_fine: int) -> np.ndarray:
    """Integer positions q (int64, (3, N)) from IOS offsets + cell_start."""
    N = pos.shape[1]
    n_ios = n_fine // 2
    nt = n_ios // TILE
    cs = cs.astype(np.int64)
    key = np.searchsorted(cs, np.arange(N), side="right") - 1
    tile, inner = key // TILE ** 3, key % TILE ** 3
    t = np.stack([tile % nt, (tile // nt) % nt, tile // (nt * nt)])
    u = np.stack([inner % TILE, (inner // TILE) % TILE, inner // (TILE * TILE)])
    c = t * TILE + u
    off = pos.astype(np.int64) & 0xFFFF
    return (c << 16) + off


def rel_err(a: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-particle |a - ref| / |ref| for (3, N) arrays."""
    num = np.linalg.norm(a - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return num / np.maximum(den, 1e-300)


def force_stats(a, ref):
    e = rel_err(np.asarray(a, dtype=np.float64), np.asarray(ref, dtype=np.float64))
    return float(np.median(e)), float(np.percentile(e, 99)), float(e.max())


def ulp32(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float32)
    return np.spacing(np.abs(x)).astype(np.float64)


def exact_sum_u64(a: np.ndarray) -> int:
    """Exact sum of a uint64 array as a Python int (split into 32-bit halves,
    each summed in int64 without overflow for up to 2^31 entries)."""
    a = np.asarray(a, dtype=np.uint64).ravel()
    hi = int((a >> np.uint64(32)).astype(np.int64).sum())
    lo = int((a & np.uint64(0xFFFFFFFF)).astype(np.int64).sum())
    return (hi << 32) + lo


def zero_force_ok(acc: np.ndarray, has: np.ndarray, floor: float) -> bool:
    """Particles with no pair inside the cutoff in exact arithmetic get an
    exactly zero oracle force; in FP32 the squared separation of a pair
    within a rounding of the cutoff may fall just inside it, where the pair
    law is ~1e-30 of a typical force: such particles must stay below the
    error floor."""
    return bool(np.all(np.abs(acc[:, ~has]) <= floor))
