"""GPU adaptive PM3 level (section 2.2.3, PM3 paragraph) through the C ABI:
the two PM levels on the whole box, cube2_pp_force_skip for the tiles without
a PM3 level, and for the others the PM3 level (spacing H3 = 1/2 fine cell,
softening b3 = 3.5 H3, truncated at the fine softening b2) plus the PP sum
cut at b3 on packed subtile boxes (cube2_tile_gather of several tiles into
one box, a PM3 context's cube2_pack, cube2_pm_level_force and cube2_pp_force,
cube2_tile_scatter_add with scale 1/H3^2).

* cube2_pp_force_skip: the other tiles' particles bit for bit equal to
  cube2_pp_force, the skipped ones untouched;
* the packed gather: tile t's particles in slot t, at the single-tile
  gather's positions shifted by the slot origin, exactly;
* one subtile per box: the forces of the PM3 tiles' particles against the
  oracle's PM3 level (oracle.pm3_local_accel plus its two PM levels) at the
  force bar (median 1e-4, p99 1e-3);
* packed boxes: against one subtile per box, within the packing's
  crosstalk (the other slots are farther than the truncation; only the
  mesh's tail reaches them): median 1e-4, p99 1e-3 of the total force;
* the three-level force against the two-level one within the PM3 mesh's
  own error, the oracle's bound (median 7e-3, p99 2.6e-2);
* the cost model: calibrate() measures it, select() returns tiles, and the
  force of the selection is finite and within the same bound.
Workload: 32^3 particles (Zel'dovich + 12 Plummer spheres of 512) in a 64^3
box, coarse ratio 4, b_f = 2, b_pp = 0.2.
"""
import numpy as np
import pytest

import oracle
import synthetic
from helpers import force_stats

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NG = 64


@pytest.fixture(scope="module")
def field():
    import paper_2512_12629_amd as m
    x = synthetic.clustered(32, 0.25, 12, 512, 0.5 / NG, 883)
    cfg = m.Config(n_fine=NG, coarse_ratio=4)
    pm3 = m.Cube2PM3(cfg, x.shape[1])
    pos, cs, perm = pm3.g.pack(torch.from_numpy(x).cuda())
    q = oracle.quantize(x, NG)
    xf = oracle.q_to_fine(q[:, perm.cpu().numpy().astype(np.int64)])     # GPU order
    count, _, _ = pm3.tile_stats(pos, cs)
    dense = torch.argsort(count, descending=True)[:5].tolist()
    return dict(m=m, cfg=cfg, pm3=pm3, pos=pos, cs=cs, xf=xf, dense=dense,
                p=oracle.Params(n_fine=NG, coarse_ratio=4))


def test_pp_skip_leaves_skipped_tiles_alone(field):
    m, pm3, pos, cs = field["m"], field["pm3"], field["pos"], field["cs"]
    ref = pm3.g.pp_force(pos, cs)
    skip = torch.zeros(pm3.nt ** 3, dtype=torch.uint8, device="cuda")
    skip[torch.tensor(field["dense"][:3], device="cuda")] = 1
    acc = torch.full_like(ref, 7.0)
    m.cube2_pp_force_skip(pm3.g.ctx, pos, cs, skip, acc, pm3.g.work)
    torch.cuda.synchronize()
    cnt = (cs[1:].long() - cs[:-1].long()).view(pm3.nt ** 3, 512).sum(1)
    tile_of = torch.repeat_interleave(torch.arange(pm3.nt ** 3, device="cuda"), cnt)
    skipped = skip[tile_of].bool()
    assert torch.all(acc[:, skipped] == 7.0)
    assert torch.equal(acc[:, ~skipped], ref[:, ~skipped])


def test_packed_gather_places_tiles_in_slots(field):
    m, pm3, pos, cs = field["m"], field["pm3"], field["pos"], field["cs"]
    tiles = field["dense"][:3]
    origins = pm3.origins(tiles)
    n = pos.shape[1]
    xb = torch.empty(3 * 4 * n, device="cuda")
    ib = torch.empty(4 * n, dtype=torch.int32, device="cuda")
    mp = m.cube2_tile_gather(pm3.g.ctx, pos, cs, origins, 16, pm3.buffer, xb, ib, pm3.g.work)
    xp = xb[:3 * mp].view(3, mp).double().cpu().numpy() * (2 * pm3.n_slot)   # k = 2
    ip = ib[:mp].cpu().numpy()
    start = 0
    for t, o in enumerate(origins):
        xs = torch.empty(3 * n, device="cuda")
        isg = torch.empty(n, dtype=torch.int32, device="cuda")
        ms = m.cube2_tile_gather(pm3.g.ctx, pos, cs, [o], 16, pm3.buffer, xs, isg, pm3.g.work)
        x1 = xs[:3 * ms].view(3, ms).double().cpu().numpy() * pm3.n_slot
        slot = np.array([t % 2, t // 2 % 2, t // 4]).reshape(3, 1) * pm3.n_slot
        assert np.array_equal(ip[start:start + ms], isg[:ms].cpu().numpy())
        assert np.array_equal(xp[:, start:start + ms], x1 + slot)
        start += ms
    assert start == mp


def _oracle_pm3(field, tiles):
    o = oracle.Oracle(field["p"])
    pm = o.pm_accel(field["xf"])
    out = {}
    for t, org in zip(tiles, field["pm3"].origins(tiles)):
        idx, a3 = oracle.pm3_local_accel(field["p"], field["xf"], org, 16, field["pm3"].buffer,
                                         0.5, 3.5)
        out[t] = (idx, pm[:, idx] + a3)
    return out


def test_pm3_one_subtile_per_box_against_oracle(field):
    m = field["m"]
    tiles = field["dense"][:3]
    one = m.Cube2PM3(field["cfg"], field["pos"].shape[1], max_batch=1)
    got = one.force(field["pos"], field["cs"], tiles).double().cpu().numpy()
    for t, (idx, ref) in _oracle_pm3(field, tiles).items():
        med, p99, _ = force_stats(got[:, idx], ref)
        assert med < 1e-4 and p99 < 1e-3, (t, med, p99)


def test_pm3_packed_boxes_against_single(field):
    m = field["m"]
    tiles = field["dense"][:5]
    one = m.Cube2PM3(field["cfg"], field["pos"].shape[1], max_batch=1)
    a1 = one.force(field["pos"], field["cs"], tiles).double().cpu().numpy()
    ap = field["pm3"].force(field["pos"], field["cs"], tiles).double().cpu().numpy()
    med, p99, _ = force_stats(ap, a1)
    assert med < 1e-4 and p99 < 1e-3, (med, p99)


def test_pm3_against_two_level(field):
    pm3, pos, cs = field["pm3"], field["pos"], field["cs"]
    tiles = field["dense"][:5]
    a3 = pm3.force(pos, cs, tiles).double().cpu().numpy()
    a2 = pm3.g.force(pos, cs).double().cpu().numpy()
    cnt = (cs[1:].long() - cs[:-1].long()).view(pm3.nt ** 3, 512).sum(1)
    tile_of = torch.repeat_interleave(torch.arange(pm3.nt ** 3, device="cuda"), cnt).cpu().numpy()
    sel = np.isin(tile_of, tiles)
    med, p99, _ = force_stats(a3[:, sel], a2[:, sel])
    assert med < 7e-3 and p99 < 2.6e-2, (med, p99)
    assert np.array_equal(a3[:, ~sel], a2[:, ~sel]) or force_stats(a3[:, ~sel], a2[:, ~sel])[1] < 1e-6


def test_pm3_cost_model(field):
    pm3, pos, cs = field["pm3"], field["pos"], field["cs"]
    model = pm3.calibrate(pos, cs, trial=8, reps=2)
    assert model["pp_s_per_candidate"] > 0 and model["pm3_s_per_tile"] >= 0
    tiles = pm3.select(pos, cs)
    # the candidate counts: every particle of a tile is a candidate of
    # itself at least, and the b3 range (5 cells of 1 fine cell) sees fewer
    # than the b2 range (3 IOS cells of 2 fine cells) on average
    count, cand2, cand3 = pm3.tile_stats(pos, cs)
    assert torch.all(cand2 >= count) and torch.all(cand3 >= count)
    assert float(cand3.sum()) < float(cand2.sum())
    a = pm3.force(pos, cs)
    assert torch.isfinite(a).all()
    assert all(0 <= t < pm3.nt ** 3 for t in tiles)
