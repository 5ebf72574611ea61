"""Seeded synthetic particle inputs shared by the HIP path and the oracle.

This module only draws inputs.  It holds none of the force method's
arithmetic: no deposit, no Green's function, no pair force.  Both the tests
of the GPU path and the oracle take their particles from here, so that the
two sides see bit-identical inputs.

Positions are returned in box units, float32, shape (3, N) (SoA), each
component in [0, 1).  The box is periodic with side 1.

Workload recipes (stand-ins for the paper's 1LPT initial conditions of a
LambdaCDM spectrum at z=200, whose transfer function and dataset are not
available here):

* ``uniform``: x ~ U[0,1)^3.
* ``zeldovich``: particles on an n_p^3 Lagrangian lattice at cell centres,
  displaced by a Zel'dovich (1LPT) field of a Gaussian random field with
  P(k) ~ k^-2; the rms of the 3D displacement is ``rms_disp`` lattice
  spacings (H_p).
* ``clustered``: a Zel'dovich lattice in which a seeded random subset of
  ``n_spheres * per_sphere`` particles is moved into Plummer spheres with
  uniformly random centres, to load the short-range pair sum the way halos do.
"""
from __future__ import annotations

import numpy as np

try:  # multi-threaded FFT for the large lattices; numpy fallback otherwise
    import scipy.fft as _sfft

    def _rfftn(a):
        return _sfft.rfftn(a, workers=-1)

    def _irfftn(a, s):
        return _sfft.irfftn(a, s=s, workers=-1)
except Exception:  # pragma: no cover
    def _rfftn(a):
        return np.fft.rfftn(a)

    def _irfftn(a, s):
        return np.fft.irfftn(a, s=s)


def _wrap01(x: np.ndarray) -> np.ndarray:
    """Wrap into [0,1) in float32 without producing 1.0 by rounding."""
    x = np.mod(x, 1.0).astype(np.float32)
    x[x >= np.float32(1.0)] = np.float32(0.0)
    x[x < np.float32(0.0)] = np.float32(0.0)
    return x


def uniform(n_part: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return _wrap01(rng.random((3, n_part), dtype=np.float64))


def zeldovich_displacement(n_p: int, seed: int) -> np.ndarray:
    """Unit-rms (3D magnitude) 1LPT displacement of a k^-2 Gaussian field.

    Returns float64 (3, n_p, n_p, n_p) in lattice spacings, indexed
    [d, z, y, x] on the Lagrangian lattice.
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n_p, n_p, n_p))
    nk = _rfftn(noise)
    kz = np.fft.fftfreq(n_p)[:, None, None] * n_p
    ky = np.fft.fftfreq(n_p)[None, :, None] * n_p
    kx = np.fft.rfftfreq(n_p)[None, None, :] * n_p
    k2 = kz * kz + ky * ky + kx * kx
    k2[0, 0, 0] = 1.0
    delta = nk / np.sqrt(k2)            # sqrt(P) with P ~ k^-2
    delta[0, 0, 0] = 0.0
    psi = np.empty((3, n_p, n_p, n_p))
    for d, kd in enumerate((kx, ky, kz)):
        psi[d] = _irfftn(1j * kd * delta / k2, s=(n_p, n_p, n_p))
    rms = np.sqrt(np.mean(np.sum(psi * psi, axis=0)))
    return psi / rms


def zeldovich(n_p: int, rms_disp: float, seed: int, return_psi: bool = False):
    """Lattice of n_p^3 particles displaced by a k^-2 Zel'dovich field.

    ``rms_disp`` is the rms of the 3D displacement in lattice spacings H_p.
    Particle order is the lattice order (x fastest).
    """
    psi = zeldovich_displacement(n_p, seed) * rms_disp
    g = (np.arange(n_p, dtype=np.float64) + 0.5)
    qz, qy, qx = np.meshgrid(g, g, g, indexing="ij")
    lag = np.stack([qx, qy, qz]).reshape(3, -1)
    disp = psi.reshape(3, -1)
    x = _wrap01((lag + disp) / n_p)
    if return_psi:
        return x, (disp / n_p)
    return x


def plummer_offsets(n: int, a: float, rng: np.random.Generator) -> np.ndarray:
    """Plummer sphere of scale radius a, truncated at 10a (inverse CDF).

    Returns float64 (3, n) offsets from the centre.
    """
    r = np.empty(n)
    filled = 0
    while filled < n:
        m = n - filled
        X = rng.random(m)
        X = np.clip(X, 1e-300, 1.0)
        rr = a / np.sqrt(np.maximum(X ** (-2.0 / 3.0) - 1.0, 1e-300))
        rr = rr[rr < 10.0 * a]
        take = min(len(rr), m)
        r[filled:filled + take] = rr[:take]
        filled += take
    u = rng.standard_normal((3, n))
    u /= np.linalg.norm(u, axis=0, keepdims=True)
    return u * r


def clustered(n_p: int, rms_disp: float, n_spheres: int, per_sphere: int,
              scale_radius: float, seed: int) -> np.ndarray:
    """Zel'dovich lattice with a subset moved into Plummer spheres.

    ``scale_radius`` is in box units.  The total particle number stays n_p^3.
    """
    x = zeldovich(n_p, rms_disp, seed).astype(np.float64)
    rng = np.random.default_rng(seed + 7919)
    n = x.shape[1]
    k = n_spheres * per_sphere
    if k > n:
        raise ValueError("more sphere particles than particles")
    idx = rng.choice(n, size=k, replace=False)
    centres = rng.random((3, n_spheres))
    off = plummer_offsets(k, scale_radius, rng)
    x[:, idx] = np.repeat(centres, per_sphere, axis=1) + off
    return _wrap01(x)


# Named workloads, sizes as in the method's test matrix.  "n_fine" is the fine
# mesh (cells per side); "coarse_ratio" 0 means a single PM level.
WORKLOADS = {
    "uniform32": dict(n_p=32, n_fine=64, coarse_ratio=0, kind="uniform"),
    "zel128": dict(n_p=128, n_fine=256, coarse_ratio=0, kind="zeldovich", rms=0.25),
    "clu256": dict(n_p=256, n_fine=512, coarse_ratio=4, kind="clustered", rms=0.25,
                   n_spheres=1000, per_sphere=2048),
    "zel128_grad": dict(n_p=128, n_fine=256, coarse_ratio=0, kind="zeldovich", rms=0.1),
    "clu512": dict(n_p=512, n_fine=1024, coarse_ratio=4, kind="clustered", rms=0.25,
                   n_spheres=8000, per_sphere=2048),
    # the same sphere mass fraction in 8x heavier spheres (denser halos, the
    # regime where the paper's adaptive PM3 level pays)
    "clu256_halos": dict(n_p=256, n_fine=512, coarse_ratio=4, kind="clustered", rms=0.25,
                         n_spheres=125, per_sphere=16384),
}

SEED_BASE = 12629


def make(name: str, seed: int | None = None, n_p: int | None = None) -> np.ndarray:
    """Positions (3, N) float32 for a named workload (optionally resized)."""
    w = dict(WORKLOADS[name])
    if n_p is not None:
        scale = (n_p / w["n_p"]) ** 3
        w["n_p"] = n_p
        if "n_spheres" in w:
            w["n_spheres"] = max(1, int(round(w["n_spheres"] * scale)))
    if seed is None:
        seed = SEED_BASE + list(WORKLOADS).index(name) + 1
    if w["kind"] == "uniform":
        return uniform(w["n_p"] ** 3, seed)
    if w["kind"] == "zeldovich":
        return zeldovich(w["n_p"], w["rms"], seed)
    n_fine = w["n_fine"] * (w["n_p"] / WORKLOADS[name]["n_p"])
    return clustered(w["n_p"], w["rms"], w["n_spheres"], w["per_sphere"],
                     0.5 / n_fine, seed)


def unit_directions(shape, count: int, seed: int) -> np.ndarray:
    """`count` seeded directions of the given shape, each of unit Euclidean
    norm (Gaussian, normalised): perturbation directions for directional
    finite differences."""
    rng = np.random.default_rng(seed)
    out = np.empty((count,) + tuple(shape))
    for k in range(count):
        v = rng.standard_normal(shape)
        out[k] = v / np.linalg.norm(v)
    return out
