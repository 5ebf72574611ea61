"""GPU tile+buffer mode (section 2.2.3, PM2 paragraph) through the C ABI:
cube2_pm_level_force (the global coarse level), cube2_tile_gather (the
particles of a tile and its buffer as a local box), a local context's
cube2_pack, cube2_pm_level_force (fine level, truncated at b_coarse) and
cube2_pp_force, and cube2_tile_scatter_add (the tile's own particles back).

* parity: for a sample of tiles, the forces of their particles against the
  oracle's tile mode (oracle.tile_local_accel plus the oracle's global
  coarse level) at the force bar (median 1e-4, p99 1e-3);
* the whole tiling (every particle in exactly one tile) against the
  periodic two-level force of the same particles on the GPU, within the
  mesh-tail bound that the oracle's own tile mode shows (median 5e-3, p99
  2e-2 for a 64^3 local box), and the PP part of a tile equal to the
  periodic PP part to FP32 summation order;
* a local box as large as the whole box reproduces the periodic force.
Workload: 48^3 particles (Zel'dovich + 20 Plummer spheres) in a 128^3 box,
coarse ratio 4; tiles of 16 fine cells with a buffer of 24 (>= b_coarse + 3
= 17 fine cells), local boxes of 64^3.
"""
import numpy as np
import pytest

import oracle
import synthetic
from helpers import force_stats

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NG, TILE, BUF = 128, 16, 24


@pytest.fixture(scope="module")
def setup():
    import paper_2512_12629_amd as m
    x = synthetic.clustered(48, 0.25, 20, 256, 0.5 / NG, 882)
    cfg = m.Config(n_fine=NG, coarse_ratio=4)
    t = m.Cube2Tiled(cfg, TILE, BUF, n_max=x.shape[1])
    pos, cs, perm = t.g.pack(torch.from_numpy(x).cuda())
    q = oracle.quantize(x, NG)
    xf = oracle.q_to_fine(q[:, perm.cpu().numpy().astype(np.int64)])   # GPU particle order
    p = oracle.Params(n_fine=NG, coarse_ratio=4)
    return dict(m=m, t=t, pos=pos, cs=cs, xf=xf, p=p, cfg=cfg)


def test_tile_mode_against_oracle_tile_mode(setup):
    t, xf, p = setup["t"], setup["xf"], setup["p"]
    a_c = oracle.Oracle(p).pm_level_accel(xf, 0)
    origins = [(0, 0, 0), (48, 16, 112), (64, 64, 64), (112, 96, 32), (16, 112, 80)]
    got = t.force(setup["pos"], setup["cs"], origins).cpu().numpy().astype(np.float64)
    for o in origins:
        print(f"[tile] oracle tile {o}", flush=True)
        idx, a = oracle.tile_local_accel(p, xf, o, TILE, BUF)
        if idx.size == 0:
            continue
        med, p99, _ = force_stats(got[:, idx], a_c[:, idx] + a)
        assert med < 1e-4 and p99 < 1e-3, (o, med, p99)


def test_whole_tiling_against_periodic_force(setup):
    t, pos, cs = setup["t"], setup["pos"], setup["cs"]
    a_tile = t.force(pos, cs).cpu().numpy().astype(np.float64)
    a_per = t.g.force(pos, cs).cpu().numpy().astype(np.float64)
    med, p99, _ = force_stats(a_tile, a_per)
    assert med < 5e-3 and p99 < 2e-2, (med, p99)
    # every particle received its tile's fine + PP part exactly once: the
    # coarse part alone is far from the periodic total
    a_c = t.g.pm_level_force(pos, cs, 1).cpu().numpy().astype(np.float64)
    assert force_stats(a_c, a_per)[0] > 20 * med


def test_tile_pp_part_is_the_periodic_pp(setup):
    m, t, pos, cs = setup["m"], setup["t"], setup["pos"], setup["cs"]
    n = pos.shape[1]
    o = (48, 16, 112)
    loc = t._local(1024)
    mcount = m.cube2_tile_gather(t.g.ctx, pos, cs, [o], TILE, BUF, t.x_buf, t.i_buf, t.g.work)
    if mcount > t.m_cap:
        loc = t._local(mcount)
        mcount = m.cube2_tile_gather(t.g.ctx, pos, cs, [o], TILE, BUF, t.x_buf, t.i_buf, t.g.work)
    xl = t.x_buf[:3 * mcount].view(3, mcount)
    pos_l, cs_l, perm_l = loc.pack(xl)
    a_l = loc.pp_force(pos_l, cs_l)
    acc = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    m.cube2_tile_scatter_add(perm_l, xl, t.i_buf[:mcount], 1, TILE, BUF, a_l, acc)
    ref = t.g.pp_force(pos, cs).cpu().numpy().astype(np.float64)
    got = acc.cpu().numpy().astype(np.float64)
    idx, _ = oracle.tile_local_accel(setup["p"], setup["xf"], o, TILE, BUF)
    own = np.zeros(n, dtype=bool)
    own[idx] = True
    assert np.all(got[:, ~own] == 0.0)
    scale = np.abs(ref[:, own]).max()
    assert np.allclose(got[:, own], ref[:, own], rtol=1e-5, atol=1e-6 * scale)


def test_local_box_of_the_whole_box(setup):
    m = setup["m"]
    t2 = m.Cube2Tiled(setup["cfg"], 64, 32, n_max=setup["pos"].shape[1])
    pos, cs = setup["pos"], setup["cs"]
    a = t2.force(pos, cs, [(0, 0, 0), (64, 0, 0), (0, 64, 0), (64, 64, 0), (0, 0, 64),
                           (64, 0, 64), (0, 64, 64), (64, 64, 64)])
    ref = t2.g.force(pos, cs)
    med, p99, _ = force_stats(a.cpu().numpy().astype(np.float64),
                              ref.cpu().numpy().astype(np.float64))
    assert med < 1e-5 and p99 < 1e-4, (med, p99)
