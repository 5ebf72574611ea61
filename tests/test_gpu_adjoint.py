"""GPU parity of the adjoint (backward) entry points against the oracle's
FP64 adjoints on the same seeded inputs and the same fixed-point weights.

The oracle's adjoints are pinned by finite differences of its forward
(tests/test_oracle_pipeline.py).  Bar: per-particle relative error of x_bar
with median <= 1e-4 and 99th percentile <= 1e-3, measured against
max(|x_bar_ref|, 1e-6 * median |x_bar_ref|) (cancellation floor).
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MED, P99 = 1e-4, 1e-3

CASES = {
    "uniform_64": (64, 0, lambda: synthetic.uniform(32 ** 3, 201)),
    "clustered_64_two_level": (64, 4, lambda: synthetic.clustered(24, 0.25, 6, 512, 0.5 / 64, 202)),
    # the largest coarse ratio the library takes (8: a coarse mesh of 8^3)
    "clustered_64_ratio8": (64, 8, lambda: synthetic.clustered(24, 0.25, 6, 512, 0.5 / 64, 204)),
    "zel_32_ragged": (32, 2, lambda: synthetic.zeldovich(13, 0.25, 203)),
}


def _np(t):
    return t.detach().cpu().numpy()


def _stats(a, ref):
    fr = np.linalg.norm(ref, axis=0)
    floor = 1e-6 * np.median(fr[fr > 0]) if np.any(fr > 0) else 1e-30
    e = np.linalg.norm(a - ref, axis=0) / np.maximum(fr, floor)
    return float(np.median(e)), float(np.percentile(e, 99))


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    import paper_2512_12629_amd as m
    n_fine, cr, gen = CASES[request.param]
    x = gen()
    c = m.Cube2(m.Config(n_fine=n_fine, coarse_ratio=cr), n_max=x.shape[1])
    pos, cs, _ = c.pack(torch.from_numpy(x).cuda())
    q = oracle.quantize(x, n_fine)
    perm, _, _ = oracle.ios_order(q, n_fine)
    xf = oracle.q_to_fine(q[:, perm])
    o = oracle.Oracle(oracle.Params(n_fine=n_fine, coarse_ratio=cr), quant=True)
    rng = np.random.default_rng(31)
    abar = rng.standard_normal(xf.shape).astype(np.float32)
    return dict(c=c, pos=pos, cs=cs, xf=xf, o=o, abar=abar, n_fine=n_fine, cr=cr)


def test_pp_backward(case):
    c = case["c"]
    xb = _np(c.pp_force_backward(case["pos"], case["cs"], torch.from_numpy(case["abar"]).cuda()))
    ref = case["o"].pp_adjoint(case["xf"], case["abar"].astype(np.float64))
    med, p99 = _stats(xb, ref)
    assert med < MED and p99 < P99, (med, p99)


def test_pm_backward(case):
    c = case["c"]
    xb = _np(c.pm_force_backward(case["pos"], case["cs"], torch.from_numpy(case["abar"]).cuda()))
    ref = case["o"].pm_adjoint(case["xf"], case["abar"].astype(np.float64))
    med, p99 = _stats(xb, ref)
    assert med < MED and p99 < P99, (med, p99)


def test_deposit_backward(case):
    c = case["c"]
    levels = case["o"].p.levels()
    rng = np.random.default_rng(32)
    for lvl_gpu in range(len(levels)):
        H, n, _, _ = levels[len(levels) - 1 - lvl_gpu]
        rb = rng.standard_normal((n, n, n)).astype(np.float32)
        xb = _np(c.deposit_backward(case["pos"], case["cs"], torch.from_numpy(rb).cuda(), lvl_gpu))
        ref = case["o"].deposit_adjoint(case["xf"], rb.astype(np.float64),
                                       level=len(levels) - 1 - lvl_gpu)
        med, p99 = _stats(xb, ref)
        assert med < 1e-5 and p99 < 1e-4, (lvl_gpu, med, p99)


def test_kick_drift_backward_is_the_transpose(case):
    c = case["c"]
    N = case["xf"].shape[1]
    rng = np.random.default_rng(33)
    vel = torch.from_numpy(rng.standard_normal((3, N)).astype(np.float32)).cuda()
    acc = c.force(case["pos"], case["cs"])
    kick, drift = 0.1, 0.2
    _, _, _, perm = c.kick_drift(case["pos"], case["cs"], vel, acc, kick, drift)
    xbo = rng.standard_normal((3, N)).astype(np.float32)
    vbo = rng.standard_normal((3, N)).astype(np.float32)
    xb, vb, ab = c.kick_drift_backward(perm, torch.from_numpy(xbo).cuda(),
                                       torch.from_numpy(vbo).cuda(), kick, drift)
    p = _np(perm)
    # forward (rint as identity): x' = x + drift (v + kick a), v' = v + kick a,
    # reordered by perm; transpose maps output cotangents back through perm.
    xb_ref = np.zeros_like(xbo)
    vb_ref = np.zeros_like(vbo)
    xb_ref[:, p] = xbo
    vb_ref[:, p] = vbo + np.float32(drift) * xbo
    assert np.allclose(_np(xb), xb_ref, rtol=0, atol=0)
    assert np.allclose(_np(vb), vb_ref, rtol=1e-6, atol=1e-6)
    assert np.allclose(_np(ab), np.float32(kick) * vb_ref, rtol=1e-6, atol=1e-6)
