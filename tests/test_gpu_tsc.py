"""GPU parity of the TSC assignment variant (eq. 5; context flag
CUBE2_ASSIGN_TSC) against the oracle's TSC pipeline on the seeded small
cases, through the C ABI.

Bars as for CIC: the fixed-point density bit-exact (16-bit weights, unit
2^-48) on both levels; the Green's table (W = sinc^3) within one FP32 ulp;
interpolation from the same potential within median 1e-5 / p99 1e-4; PM
and total forces within median 1e-4 / p99 1e-3 per particle.  The FP64
plain form with TSC matches the oracle within median 1e-10 / p99 1e-8.  The
PM and deposit adjoints (TSC weights, slopes of eq. 5) meet the force bar
and the deposit-adjoint bar of the CIC ones against the oracle's TSC
adjoints."""
import numpy as np
import pytest

import oracle
import synthetic
from helpers import exact_sum_u64, force_stats, ulp32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MED, P99 = 1e-4, 1e-3

CASES = {
    "uniform_64": (64, 0, lambda: synthetic.uniform(32 ** 3, 301)),
    "clustered_64_two_level": (64, 4, lambda: synthetic.clustered(24, 0.25, 6, 512, 0.5 / 64, 302)),
    "zel_32_ragged": (32, 2, lambda: synthetic.zeldovich(13, 0.25, 303)),
    # the largest coarse ratio the library takes (8: a coarse mesh of 8^3)
    "clustered_64_ratio8": (64, 8, lambda: synthetic.clustered(24, 0.25, 6, 512, 0.5 / 64, 304)),
}


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    import paper_2512_12629_amd as m
    n_fine, cr, gen = CASES[request.param]
    x = gen()
    flags = m.CUBE2_ASSIGN_TSC | m.CUBE2_FP64_FORM
    c = m.Cube2(m.Config(n_fine=n_fine, coarse_ratio=cr, flags=flags), n_max=x.shape[1])
    pos, cs, perm = c.pack(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    p = oracle.Params(n_fine=n_fine, coarse_ratio=cr, assign=3)
    q = oracle.quantize(x, n_fine)
    perm_or, _, _ = oracle.ios_order(q, n_fine)
    xf = oracle.q_to_fine(q[:, perm_or])
    torch.cuda.synchronize()
    return dict(c=c, p=p, pos=pos, cs=cs, xf=xf)


def test_tsc_green_table_within_one_ulp(case):
    c, p = case["c"], case["p"]
    for level, (H, n, b_a, b_prev) in enumerate(reversed(p.levels())):
        g_or = oracle.green_table(n, b_a / H, b_prev / H, p.alias_nmax, 3)
        g = _np(c.green_table(level)).astype(np.float64)
        assert np.all(np.abs(g - g_or.astype(np.float32)) <= ulp32(g_or) + 1e-30)


def test_tsc_deposit_bit_exact(case):
    c, p, xf = case["c"], case["p"], case["xf"]
    for level, (H, n, _, _) in enumerate(reversed(p.levels())):
        rho, fx = c.deposit(case["pos"], case["cs"], level, fx=True)
        acc_or = oracle.deposit_fx(xf, n, H, p=3)
        assert np.array_equal(_np(fx).view(np.uint64), acc_or)
        assert np.array_equal(_np(rho), oracle.density_f32(acc_or, p=3))
        assert exact_sum_u64(acc_or) == xf.shape[1] * 2 ** 48
    assert c.status() == 0


def test_tsc_interp_against_oracle(case):
    c, p, xf = case["c"], case["p"], case["xf"]
    lv = list(reversed(p.levels()))
    phis = [c.potential(c.deposit(case["pos"], case["cs"], l), l) for l in range(len(lv))]
    acc = _np(c.interp(case["pos"], case["cs"], phis[0], phis[1] if len(lv) > 1 else None))
    ref = np.zeros_like(acc, dtype=np.float64)
    for l, (H, n, _, _) in enumerate(lv):
        E = oracle.fd_force(_np(phis[l]).astype(np.float64))
        ref += oracle.interp(xf, E, H, True, p=3) / H ** 2
    med, p99, _ = force_stats(acc, ref)
    assert med < 1e-5 and p99 < 1e-4, (med, p99)


def test_tsc_pm_and_total_force_against_oracle(case):
    c, o = case["c"], oracle.Oracle(case["p"])
    acc = _np(c.pm_force(case["pos"], case["cs"]))
    med, p99, _ = force_stats(acc, o.pm_accel(case["xf"]))
    assert med < MED and p99 < P99, (med, p99)
    acc = _np(c.force(case["pos"], case["cs"]))
    med, p99, _ = force_stats(acc, o.accel(case["xf"]))
    assert med < MED and p99 < P99, (med, p99)


def test_tsc_fp64_form_against_oracle(case):
    acc = _np(case["c"].pm_force_f64(case["pos"], case["cs"]))
    med, p99, _ = force_stats(acc, oracle.Oracle(case["p"]).pm_accel(case["xf"]))
    assert med < 1e-10 and p99 < 1e-8, (med, p99)


def test_tsc_momentum_conservation(case):
    a = case["c"].pm_force(case["pos"], case["cs"]).double()
    total = torch.linalg.vector_norm(a.sum(dim=1)).item()
    assert total <= 1e-6 * torch.linalg.vector_norm(a, dim=0).sum().item()


def _stats(a, ref):
    fr = np.linalg.norm(ref, axis=0)
    floor = 1e-6 * np.median(fr[fr > 0]) if np.any(fr > 0) else 1e-30
    e = np.linalg.norm(a - ref, axis=0) / np.maximum(fr, floor)
    return float(np.median(e)), float(np.percentile(e, 99))


def test_tsc_pm_backward_against_oracle(case):
    """The PM adjoint with TSC weights and the slopes of eq. 5 against the
    oracle's TSC adjoint (pinned by finite differences on the CPU)."""
    c = case["c"]
    rng = np.random.default_rng(304)
    abar = rng.standard_normal(case["xf"].shape).astype(np.float32)
    xb = _np(c.pm_force_backward(case["pos"], case["cs"], torch.from_numpy(abar).cuda()))
    ref = oracle.Oracle(case["p"]).pm_adjoint(case["xf"], abar.astype(np.float64))
    med, p99 = _stats(xb, ref)
    assert med < MED and p99 < P99, (med, p99)


def test_tsc_deposit_backward_against_oracle(case):
    c = case["c"]
    o = oracle.Oracle(case["p"])
    levels = case["p"].levels()
    rng = np.random.default_rng(305)
    for lvl_gpu in range(len(levels)):
        H, n, _, _ = levels[len(levels) - 1 - lvl_gpu]
        rb = rng.standard_normal((n, n, n)).astype(np.float32)
        xb = _np(c.deposit_backward(case["pos"], case["cs"], torch.from_numpy(rb).cuda(), lvl_gpu))
        ref = o.deposit_adjoint(case["xf"], rb.astype(np.float64), level=len(levels) - 1 - lvl_gpu)
        med, p99 = _stats(xb, ref)
        assert med < 1e-5 and p99 < 1e-4, (lvl_gpu, med, p99)
