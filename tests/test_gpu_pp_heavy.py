"""PP parity (eq. 4d) on tiles loaded like the Plummer-sphere tiles of the
benchmark workloads: IOS cells of hundreds of particles, tiles of thousands,
spheres that straddle tile faces, and a tile whose box needs several z-chunks.

Workload: 64^3 mesh (4^3 tiles of 8^3 IOS cells), 24000 uniform background
particles and six Plummer spheres (a = 0.6 fine cell): one of 3000 inside a
tile, one of 5000 centred on a tile face (two dense tiles whose pairs cross
the face), two of 2600 in one tile (more particles than one staged box
holds: z-chunks), one of 400 (a light tile with a dense cell) and one of
1500.  Checked:
* the workload has the intended shape (tiles over 1024 particles with dense
  cells, one over the staging capacity, a light tile with a dense cell);
* the PP force against the oracle's FP64 pair sum (median <= 1e-4,
  p99 <= 1e-3 relative to max(|F|, 1e-6 median |F|));
* the PP force bit for bit equal on two calls, and cube2_force bit for bit
  equal to the separate PM and PP calls;
* momentum: the pair forces sum to zero to FP32 rounding of the sums.
"""
import numpy as np
import pytest

import oracle
from helpers import ios_decode

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_FINE = 64
SPHERES = [((8.3, 9.1, 7.7), 3000), ((16.0, 20.0, 27.0), 5000), ((40.5, 42.0, 36.0), 2600),
           ((43.0, 41.0, 44.0), 2600), ((56.0, 8.0, 24.0), 400), ((24.0, 56.0, 52.0), 1500)]


def _plummer(rng, n, a):
    # radius from the Plummer mass profile M(<r) = r^3 / (r^2 + a^2)^1.5,
    # truncated at 3 a, isotropic directions
    u = rng.random(n) * (27.0 / 10.0 ** 1.5)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    d = rng.standard_normal((3, n))
    return r * d / np.linalg.norm(d, axis=0)


def _positions(seed):
    rng = np.random.default_rng(seed)
    parts = [rng.random((3, 24000)) * N_FINE]
    for (cx, cy, cz), n in SPHERES:
        parts.append(np.array([[cx], [cy], [cz]]) + _plummer(rng, n, 0.6))
    x = np.concatenate(parts, axis=1) % N_FINE / N_FINE
    return np.ascontiguousarray(rng.permutation(x.T).T).astype(np.float32)


@pytest.fixture(scope="module")
def heavy():
    import paper_2512_12629_amd as m
    x = _positions(12629)
    c = m.Cube2(m.Config(n_fine=N_FINE, coarse_ratio=4), n_max=x.shape[1])
    pos, cs, _ = c.pack(torch.from_numpy(x).cuda())
    q = ios_decode(pos.cpu().numpy().view(np.uint16), cs.cpu().numpy().view(np.uint32), N_FINE)
    cell = q >> 16
    counts = np.zeros((32, 32, 32), dtype=np.int64)
    np.add.at(counts, (cell[2], cell[1], cell[0]), 1)
    return dict(c=c, pos=pos, cs=cs, xf=q / 2.0 ** 15, counts=counts,
                p=oracle.Params(n_fine=N_FINE, coarse_ratio=4))


def test_workload_shape(heavy):
    counts = heavy["counts"]
    tiles = counts.reshape(4, 8, 4, 8, 4, 8)
    per_tile = tiles.sum(axis=(1, 3, 5))
    dense = (tiles >= 32).any(axis=(1, 3, 5))
    heavy_t = per_tile >= 1024
    assert (heavy_t & dense).sum() >= 4
    assert (~heavy_t & dense).any()                 # a light tile with a dense cell
    # a tile whose staged box exceeds the staging capacity (3840)
    assert per_tile.max() > 3840


def test_heavy_pp_force_against_oracle(heavy):
    got = heavy["c"].pp_force(heavy["pos"], heavy["cs"]).cpu().numpy().astype(np.float64)
    ref = oracle.Oracle(heavy["p"]).pp_accel(heavy["xf"])
    fr = np.linalg.norm(ref, axis=0)
    has = fr > 0
    floor = 1e-6 * np.median(fr[has])
    e = np.linalg.norm(got - ref, axis=0)[has] / np.maximum(fr[has], floor)
    med, p99 = float(np.median(e)), float(np.percentile(e, 99))
    assert med < 1e-4 and p99 < 1e-3, (med, p99)


def test_heavy_pp_force_is_reproducible(heavy):
    import paper_2512_12629_amd as m
    c, pos, cs = heavy["c"], heavy["pos"], heavy["cs"]
    a = c.pp_force(pos, cs)
    assert torch.equal(c.pp_force(pos, cs), a)
    ref = c.pp_force(pos, cs, c.pm_force(pos, cs))
    assert torch.equal(c.force(pos, cs), ref)
    del m


def test_heavy_pp_momentum(heavy):
    a = heavy["c"].pp_force(heavy["pos"], heavy["cs"]).double()
    total = torch.linalg.vector_norm(a.sum(dim=1)).item()
    scale = torch.linalg.vector_norm(a, dim=0).sum().item()
    assert total <= 1e-6 * scale, (total, scale)
