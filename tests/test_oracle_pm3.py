"""Pins of the oracle's PM3 level (section 2.2.3, PM3 paragraph;
oracle.pm3_local_accel): on a subtile's local box, a mesh of spacing H3
carries the target R(r, b3) - R(r, b2) (b3 = beta3 H3, truncated at the fine
level's softening b2) and the PP sum is cut at b3.

* With b3 = b2 the PM3 level's target vanishes (its Green's function is
  zero) and PP cut at b3 is PP cut at b2: the three-level force equals the
  two-level force to rounding, which pins the change of units (positions in
  H3 cells, softenings in H3 cells, accelerations scaled by 1/H3^2 from the
  homogeneity of eq. 2) and the subtile plumbing exactly.
* With b3 < b2 the three-level force differs from the two-level one by the
  PM3 mesh's own error on the short-range force (the paper's PM levels err
  by a few % per pair near their softening): measured at median 3.5e-3 /
  p99 1.3e-2 of the total force for H3 = 1/2 fine cell, beta3 = 3.5, on the
  densest subtiles of a Plummer-loaded field; the bound here is twice that.
"""
import numpy as np
import pytest

import oracle
import synthetic
from helpers import force_stats

NG = 64


@pytest.fixture(scope="module")
def field():
    x = synthetic.clustered(32, 0.25, 12, 512, 0.5 / NG, 883)
    xf = oracle.q_to_fine(oracle.quantize(x, NG))
    p = oracle.Params(n_fine=NG, coarse_ratio=4)
    o = oracle.Oracle(p, workers=4)
    key = np.floor(xf / 16).astype(int)
    tid = (key[2] * 4 + key[1]) * 4 + key[0]
    dense = np.argsort(-np.bincount(tid, minlength=64))[:3]
    origins = [(int(t % 4) * 16, int(t // 4 % 4) * 16, int(t // 16) * 16) for t in dense]
    return dict(xf=xf, p=p, pm=o.pm_accel(xf), pp=o.pp_accel(xf), origins=origins)


def test_pm3_with_b3_equal_b2_is_the_two_level_force(field):
    for o in field["origins"][:2]:
        idx, a3 = oracle.pm3_local_accel(field["p"], field["xf"], o, 16, 8, 0.5, 4.0)
        assert idx.size > 500
        ref = field["pp"][:, idx]
        assert np.allclose(a3, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())


def test_pm3_differs_by_its_mesh_error(field):
    for o in field["origins"]:
        idx, a3 = oracle.pm3_local_accel(field["p"], field["xf"], o, 16, 8, 0.5, 3.5)
        two = (field["pm"] + field["pp"])[:, idx]
        med, p99, _ = force_stats(field["pm"][:, idx] + a3, two)
        assert med < 7e-3 and p99 < 2.6e-2, (o, med, p99)
