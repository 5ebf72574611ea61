"""Pins of the oracle's tile+buffer mode (section 2.2.3, PM2 paragraph;
oracle.tile_local_accel): the coarse level on the whole periodic box, the
fine level and PP of a tile on a local periodic box of the tile and a buffer.

* with a buffer beyond the PP cutoff the tile's PP forces are the global
  ones (the same pair set);
* a local box as large as the whole box is the whole box shifted by whole
  cells: the tile forces are the periodic ones to FP64 rounding;
* the fine level of a smaller local box differs from the periodic one only
  by the mesh force's tail beyond the truncation (the mesh force of the
  optimised G is not zero there), which shrinks as the local box grows:
  measured here (64^3 particles, 256^3 box, a Plummer-loaded Zel'dovich
  field; buffers of at least b_coarse + 3 fine cells, the paper's depth) at
  median 3.7e-3 / p99 1.1e-2 of the total force for a 64^3 local box and
  8e-4 / 5.5e-3 for 128^3 (the paper accepts per-pair errors of 2 % rms)."""
import numpy as np
import pytest

import oracle
import synthetic
from helpers import force_stats


@pytest.fixture(scope="module")
def box():
    ng = 256
    x = synthetic.clustered(64, 0.25, 40, 256, 0.5 / ng, 881)
    xf = oracle.q_to_fine(oracle.quantize(x, ng))
    p = oracle.Params(n_fine=ng, coarse_ratio=4)
    o = oracle.Oracle(p, workers=4)
    parts = (o.pm_level_accel(xf, 0), o.pm_level_accel(xf, 1), o.pp_accel(xf))
    return dict(xf=xf, p=p, parts=parts, ng=ng)


def _tile(box, origin, tile, buffer):
    idx, a = oracle.tile_local_accel(box["p"], box["xf"], origin, tile, buffer, workers=4)
    a_c, a_f, a_pp = box["parts"]
    return idx, a_c[:, idx] + a, (a_c + a_f + a_pp)[:, idx]


def test_tile_pp_is_the_global_pp(box):
    o = oracle.Oracle(oracle.Params(n_fine=64, coarse_ratio=4))
    rel = np.mod(box["xf"] - (np.array([[32], [0], [224]]) - 24), box["ng"])
    inb = np.all(rel < 64, axis=0)
    own = np.all((rel >= 24) & (rel < 40), axis=0)
    pp_l = o.pp_accel(np.ascontiguousarray(rel[:, inb]))[:, own[inb]]
    assert np.allclose(pp_l, box["parts"][2][:, own], rtol=1e-12, atol=1e-12 * np.abs(pp_l).max())


def test_local_box_of_the_whole_box_is_the_periodic_force(box):
    idx, a, ref = _tile(box, (32, 64, 224), 128, 64)
    assert idx.size > 0
    assert np.allclose(a, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_buffer_error_is_the_mesh_tail(box):
    stats = {}
    for tile, buffer in ((16, 24), (64, 32)):   # buffers >= b_coarse + 3 = 17
        idx, a, ref = _tile(box, (96, 64, 224), tile, buffer)
        stats[tile + 2 * buffer] = force_stats(a, ref)
    med64, p99_64, _ = stats[64]
    assert med64 < 5e-3 and p99_64 < 2e-2, stats
    assert stats[128][0] < 0.5 * med64 and stats[128][1] < 0.6 * p99_64, stats
