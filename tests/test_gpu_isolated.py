"""GPU parity of isolated boundary conditions (appendix A; context flag
CUBE2_ISOLATED) against the oracle: a two-level 64^3 mesh (coarse ratio 4,
and 8) whose coarse (untruncated) level carries the 1 - sinc(kL) factor,
particles in the first half of the box.  Green's tables within one FP32 ulp of the oracle's;
forces within the force bar, also for single pairs across the matching
scales (the experiment of section 3.1, run by bench.py --pairwise)."""
import numpy as np
import pytest

import oracle
import synthetic
from helpers import force_stats, ulp32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[4, 8], ids=["ratio4", "ratio8"])
def iso(request):
    import paper_2512_12629_amd as m
    n_f, cr = 64, request.param
    x = 0.5 * synthetic.clustered(12, 0.25, 4, 256, 0.5 / 32, 401)   # in [0, 1/2)^3
    c = m.Cube2(m.Config(n_fine=n_f, coarse_ratio=cr, flags=m.CUBE2_ISOLATED), n_max=x.shape[1])
    pos, cs, perm = c.pack(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    p = oracle.Params(n_fine=n_f, coarse_ratio=cr, isolated=True)
    q = oracle.quantize(x, n_f)
    perm_or, _, _ = oracle.ios_order(q, n_f)
    torch.cuda.synchronize()
    return dict(m=m, c=c, p=p, pos=pos, cs=cs, xf=oracle.q_to_fine(q[:, perm_or]))


def test_isolated_green_tables_within_one_ulp(iso):
    c, p = iso["c"], iso["p"]
    o = oracle.Oracle(p)
    for level in range(len(p.levels())):
        g_or = o.green(len(p.levels()) - 1 - level)
        g = iso["c"].green_table(level).cpu().numpy().astype(np.float64)
        assert np.all(np.abs(g - g_or.astype(np.float32)) <= ulp32(g_or) + 1e-30)


def test_isolated_forces_against_oracle(iso):
    o = oracle.Oracle(iso["p"])
    acc = iso["c"].force(iso["pos"], iso["cs"]).cpu().numpy()
    med, p99, _ = force_stats(acc, o.accel(iso["xf"]))
    assert med < 1e-4 and p99 < 1e-3, (med, p99)


def test_isolated_pairs_against_oracle(iso):
    """Single pairs across the matching scales and out to 3/4 of the
    isolation length: the GPU force on each particle within 1e-4 of the
    oracle's (both use the same quantised positions)."""
    m, c = iso["m"], iso["c"]
    o = oracle.Oracle(iso["p"])
    rng = np.random.default_rng(402)
    for r in (0.3, 1.5, 3.0, 10.0, 14.0, 20.0, 24.0):
        u = np.abs(rng.standard_normal(3))
        u /= np.linalg.norm(u)
        a0 = 2.0 + rng.random(3)
        xf = np.stack([a0, a0 + r * u], axis=1)
        x32 = (xf / 64.0).astype(np.float32)
        pos, cs, perm = c.pack(torch.from_numpy(x32).cuda())
        acc = np.empty((3, 2))
        acc[:, perm.cpu().numpy().astype(np.int64)] = c.force(pos, cs).double().cpu().numpy()
        ref = o.accel(oracle.q_to_fine(oracle.quantize(x32, 64)))
        assert np.linalg.norm(acc - ref) <= 1e-4 * np.linalg.norm(ref), r
