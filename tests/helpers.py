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
