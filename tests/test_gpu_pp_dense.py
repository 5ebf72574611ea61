"""PP parity (eq. 4d) and its adjoint where a tile's box of IOS cells holds
more particles than the kernels stage in LDS at once.

The PP kernels stage the particles of a tile's (8 + 2)^3 box of IOS cells in
LDS (at most 3840 for the forward, 4096 for the adjoint, which stages the
cotangents too).  A denser box is done in z-chunks of the tile's own cells
(2, 4 or 8 of them, each staging its slice of box layers), and a chunk whose
slice still does not fit reads its neighbours straight from HBM.  The
clustered workloads never reach these paths at test sizes, so the cases here
put one dense column into one tile of a 64^3 mesh:

* "chunked": 6000 particles in a 4 x 4 x 16 fine-cell column (the forward
  runs 4 chunks, the adjoint 2, every slice staged);
* "unstaged": 14000 particles in the same column (8 chunks; the inner
  slices exceed both capacities and read HBM, the outer ones are staged);
on a uniform background of 6000 particles.  The chunk counts are
recomputed here from the cell counts, to show that each case takes the
intended path.  Checked against the oracle: the PP force and the PP adjoint
(median <= 1e-4, p99 <= 1e-3 relative to max(|F|, 1e-6 median |F|), as in
the other PP tests), and cube2_force / cube2_force_backward bit for bit
against the separate PM and PP entry points.
"""
import numpy as np
import pytest

import oracle
from helpers import ios_decode

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_FINE = 64
CAP_FWD, CAP_ADJ = 3840, 4096
CASES = {"chunked": 6000, "unstaged": 14000}


def _positions(n_col, seed):
    rng = np.random.default_rng(seed)
    bg = rng.random((3, 6000))
    col = np.empty((3, n_col))
    col[0] = 20.0 + 4.0 * rng.random(n_col)
    col[1] = 20.0 + 4.0 * rng.random(n_col)
    col[2] = 16.0 + 16.0 * rng.random(n_col)
    x = np.concatenate([bg, col / N_FINE], axis=1)
    return np.ascontiguousarray(rng.permutation(x.T).T).astype(np.float32)


def _chunks(counts, cap):
    """(C, staged flags) the PP kernels choose for tile (1, 1, 1) of the
    IOS-cell counts (z, y, x): the smallest power-of-two number of z-chunks
    (at most 8) whose box slices fit `cap`, and which slices do."""
    box = counts[7:17, 7:17, 7:17]            # IOS cells [8-1, 16+1) per axis
    layer = box.sum(axis=(1, 2))
    C = 1
    while True:
        sl = [int(layer[c * 8 // C:(c + 1) * 8 // C + 2].sum()) for c in range(C)]
        if all(v <= cap for v in sl) or C == 8:
            return C, [v <= cap for v in sl]
        C *= 2


@pytest.fixture(scope="module", params=list(CASES))
def dense(request):
    import paper_2512_12629_amd as m
    x = _positions(CASES[request.param], 4242 + CASES[request.param])
    c = m.Cube2(m.Config(n_fine=N_FINE, coarse_ratio=4), n_max=x.shape[1])
    pos, cs, perm = c.pack(torch.from_numpy(x).cuda())
    q = ios_decode(pos.cpu().numpy().view(np.uint16), cs.cpu().numpy().view(np.uint32), N_FINE)
    xf = q / 2.0 ** 15                         # the GPU's particle order, fine cells
    cell = q >> 16
    counts = np.zeros((32, 32, 32), dtype=np.int64)
    np.add.at(counts, (cell[2], cell[1], cell[0]), 1)
    rng = np.random.default_rng(77)
    abar = rng.standard_normal((3, x.shape[1])).astype(np.float32)
    return dict(name=request.param, c=c, pos=pos, cs=cs, xf=xf, counts=counts, abar=abar,
                p=oracle.Params(n_fine=N_FINE, coarse_ratio=4))


def _rel(got, ref):
    fr = np.linalg.norm(ref, axis=0)
    has = fr > 0
    floor = 1e-6 * np.median(fr[has])
    e = np.linalg.norm(got - ref, axis=0)[has] / np.maximum(fr[has], floor)
    return float(np.median(e)), float(np.percentile(e, 99))


def test_cases_take_the_dense_paths(dense):
    cf, sf = _chunks(dense["counts"], CAP_FWD)
    ca, sa = _chunks(dense["counts"], CAP_ADJ)
    if dense["name"] == "chunked":
        assert cf > 1 and ca > 1 and all(sf) and all(sa), (cf, sf, ca, sa)
    else:
        assert cf == 8 and ca == 8 and not all(sf) and not all(sa) and any(sf) and any(sa)


def test_dense_pp_force_against_oracle(dense):
    got = dense["c"].pp_force(dense["pos"], dense["cs"]).cpu().numpy().astype(np.float64)
    ref = oracle.Oracle(dense["p"]).pp_accel(dense["xf"])
    med, p99 = _rel(got, ref)
    assert med < 1e-4 and p99 < 1e-3, (med, p99)


def test_dense_pp_adjoint_against_oracle(dense):
    ab = torch.from_numpy(dense["abar"]).cuda()
    got = dense["c"].pp_force_backward(dense["pos"], dense["cs"], ab).cpu().numpy()
    ref = oracle.Oracle(dense["p"]).pp_adjoint(dense["xf"], dense["abar"].astype(np.float64))
    med, p99 = _rel(got.astype(np.float64), ref)
    assert med < 1e-4 and p99 < 1e-3, (med, p99)


def test_dense_force_entries_equal_separate_calls(dense):
    import paper_2512_12629_amd as m
    c, pos, cs = dense["c"], dense["pos"], dense["cs"]
    ref = c.pp_force(pos, cs, c.pm_force(pos, cs))
    ab = torch.from_numpy(dense["abar"]).cuda()
    refb = torch.empty_like(ab)
    m.cube2_pm_force_backward(c.ctx, pos, cs, ab, refb, c.work)
    m.cube2_pp_force_backward(c.ctx, pos, cs, ab, refb, c.work, accumulate=True)
    for _ in range(2):
        assert torch.equal(c.force(pos, cs), ref)
        assert torch.equal(c.force_backward(pos, cs, ab), refb)
    # accumulate: x_bar = 1 + adjoint, the same adds as the separate calls
    acc_ref = torch.ones_like(ab)
    m.cube2_pm_force_backward(c.ctx, pos, cs, ab, acc_ref, c.work, accumulate=True)
    m.cube2_pp_force_backward(c.ctx, pos, cs, ab, acc_ref, c.work, accumulate=True)
    assert torch.equal(c.force_backward(pos, cs, ab, torch.ones_like(ab)), acc_ref)
