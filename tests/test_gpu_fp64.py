"""The FP64 plain form (contexts created with CUBE2_FP64_FORM), called through
the C ABI, against the FP64 oracle on the small seeded cases.

Both sides compute in FP64 from the same exact integer positions, so the
bars are set by FP64 rounding: the potential within 1e-11 (norm-relative;
two FFT orders and two G tables), forces within median 1e-10 and 99th
percentile 1e-8 per particle.  The PP term alone is compared with the exact
rational sum of oracle.exact (stored under tests/golden): the FP64 oracle's
difference R(r, b_pp) - R(r, b_f) cancels near the cutoff (its own error
reaches 7e-4 for some particles of the ragged case), the exact sum does not.
Errors there are relative to max(|F|, 1e-6 median |F|), as in the FP32 PP
test.
"""
import os

import numpy as np
import pytest

import oracle
import synthetic
from helpers import force_stats

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

CASES = {
    "uniform_64": (64, 0, lambda: synthetic.uniform(32 ** 3, 101)),
    "clustered_64_two_level": (64, 4, lambda: synthetic.clustered(24, 0.25, 6, 512, 0.5 / 64, 102)),
    # the largest coarse ratio the library takes (8: a coarse mesh of 8^3)
    "clustered_64_ratio8": (64, 8, lambda: synthetic.clustered(24, 0.25, 6, 512, 0.5 / 64, 105)),
    "zel_32_ragged": (32, 2, lambda: synthetic.zeldovich(13, 0.25, 103)),
    # the single-level Zel'dovich workload at its stated size: 128^3 particles
    # (k^-2 field, rms 0.25 H_p), 256^3 mesh
    "zel128": (256, 0, lambda: synthetic.make("zel128")),
}


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    import paper_2512_12629_amd as m
    n_fine, cr, gen = CASES[request.param]
    x = gen()
    c = m.Cube2(m.Config(n_fine=n_fine, coarse_ratio=cr, flags=m.CUBE2_FP64_FORM),
                n_max=x.shape[1])
    pos, cs, _ = c.pack(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    p = oracle.Params(n_fine=n_fine, coarse_ratio=cr)
    q = oracle.quantize(x, n_fine)
    perm_or, _, _ = oracle.ios_order(q, n_fine)
    xf = oracle.q_to_fine(q[:, perm_or])
    torch.cuda.synchronize()
    return dict(c=c, p=p, pos=pos, cs=cs, xf=xf)


def test_fp64_potential_against_oracle(case):
    c, p = case["c"], case["p"]
    o = oracle.Oracle(p)
    for level in range(len(p.levels())):
        lvl_or = len(p.levels()) - 1 - level
        _, fx = c.deposit(case["pos"], case["cs"], level, fx=True)
        rho = fx.to(torch.float64) * 2.0 ** -45
        phi = _np(c.potential_f64(rho, level))
        phi_or = oracle.potential(_np(rho), o.green(lvl_or))
        err = np.linalg.norm(phi - phi_or) / np.linalg.norm(phi_or)
        assert err < 1e-11, err


def test_fp64_pm_force_against_oracle(case):
    acc = _np(case["c"].pm_force_f64(case["pos"], case["cs"]))
    ref = oracle.Oracle(case["p"]).pm_accel(case["xf"])
    med, p99, _ = force_stats(acc, ref)
    assert med < 1e-10 and p99 < 1e-8, (med, p99)


EXACT = {
    "zel_32_ragged": (32, lambda: synthetic.zeldovich(13, 0.25, 103)),
    "clustered_32": (32, lambda: synthetic.clustered(12, 0.25, 1, 256, 0.5 / 32, 105)),
}


@pytest.mark.parametrize("name", list(EXACT))
def test_fp64_pp_force_against_exact(name):
    """PP against the exact rational sum (tests/golden, from oracle.exact):
    FP64 rounding only, so median 1e-12 and p99 1e-10 (floor as above)."""
    import paper_2512_12629_amd as m
    n_f, gen = EXACT[name]
    x = gen()
    ref = np.loadtxt(os.path.join(GOLDEN, f"pp_exact_{name}.txt")).T
    c = m.Cube2(m.Config(n_fine=n_f, flags=m.CUBE2_FP64_FORM), n_max=x.shape[1])
    pos, cs, perm = c.pack(torch.from_numpy(x).cuda())
    acc = np.empty_like(ref)
    acc[:, _np(perm).astype(np.int64)] = _np(c.pp_force_f64(pos, cs))
    fr = np.linalg.norm(ref, axis=0)
    has = fr > 0
    assert np.all(acc[:, ~has] == 0)
    floor = 1e-6 * np.median(fr[has])
    e = np.linalg.norm(acc - ref, axis=0)[has] / np.maximum(fr[has], floor)
    med, p99 = float(np.median(e)), float(np.percentile(e, 99))
    assert med < 1e-12 and p99 < 1e-10, (med, p99)


def test_fp64_total_force_against_oracle(case):
    acc = _np(case["c"].force_f64(case["pos"], case["cs"]))
    ref = oracle.Oracle(case["p"]).accel(case["xf"])
    med, p99, _ = force_stats(acc, ref)
    assert med < 1e-10 and p99 < 1e-8, (med, p99)


def test_fp32_path_against_fp64_form(case):
    a32 = _np(case["c"].force(case["pos"], case["cs"])).astype(np.float64)
    a64 = _np(case["c"].force_f64(case["pos"], case["cs"]))
    med, p99, _ = force_stats(a32, a64)
    assert med < 1e-4 and p99 < 1e-3, (med, p99)


def test_fp64_entry_points_need_the_flag():
    import paper_2512_12629_amd as m
    x = synthetic.uniform(512, 104)
    c = m.Cube2(m.Config(n_fine=16), n_max=x.shape[1])
    pos, cs, _ = c.pack(torch.from_numpy(x).cuda())
    with pytest.raises(m.Cube2Error) as e:
        c.pm_force_f64(pos, cs)
    assert e.value.code == -6
    with pytest.raises(m.Cube2Error) as e:
        c.pp_force_f64(pos, cs)
    assert e.value.code == -6
