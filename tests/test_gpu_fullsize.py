"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (one context per workload, the whole particle set resident):

* clu256: 256^3 particles, fine 512^3, coarse 128^3;
* clu512: 512^3 particles, fine 1024^3, coarse 256^3;
both Zel'dovich k^-2 plus Plummer spheres (the bench workloads).

What is checked, per workload:
* the fine and coarse fixed-point densities, bit-exact against the oracle's
  integer deposit of the same quantised positions (whole meshes);
* PP on a seeded sample of 4096 particles against the oracle's FP64 pair sum
  for exactly those particles (median <= 1e-4, p99 <= 1e-3, floor as in the
  small-case PP test);
* the PP adjoint of another 4096-particle sample (Gaussian cotangents on all
  particles) against the oracle's FP64 adjoint of those particles (same bars);
* the FP32 force of every particle against the FP64 plain form on the GPU
  (median <= 1e-4, p99 <= 1e-3), the FP64 form itself being pinned to the
  oracle on the small cases;
* momentum conservation of each part: the PM scheme (CIC deposit and
  interpolation, even G, antisymmetric stencil) and the pair sum (exactly
  antisymmetric pair forces) both sum to zero in exact arithmetic, so
  |sum F| <= 1e-6 sum |F| in FP32.
The oracle's inputs are its own quantisation of the generated positions;
the GPU outputs are mapped back to input order with the GPU's permutation.
"""
import numpy as np
import pytest

import oracle
import synthetic
from helpers import zero_force_ok

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WORKLOADS = {"clu256": (512, 4), "clu512": (1024, 4)}


@pytest.fixture(scope="module", params=list(WORKLOADS))
def big(request):
    import paper_2512_12629_amd as m
    name = request.param
    n_f, cr = WORKLOADS[name]
    print(f"[fullsize] {name}: generating", flush=True)
    x = synthetic.make(name)
    c = m.Cube2(m.Config(n_fine=n_f, coarse_ratio=cr, flags=m.CUBE2_FP64_FORM), n_max=x.shape[1])
    pos, cs, perm = c.pack(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    xf = oracle.q_to_fine(oracle.quantize(x, n_f))          # oracle input, input order
    inv = torch.empty_like(perm)
    inv[perm.long()] = torch.arange(perm.numel(), dtype=perm.dtype, device=perm.device)
    yield dict(name=name, c=c, pos=pos, cs=cs, perm=perm.long(), inv=inv.long(), xf=xf,
               p=oracle.Params(n_fine=n_f, coarse_ratio=cr), n_f=n_f, cr=cr)
    del c
    torch.cuda.empty_cache()


def _stats(a, ref):
    """median and 99th percentile of |a - ref| / |ref| per particle (GPU, FP64)."""
    num = torch.linalg.vector_norm(a.double() - ref, dim=0)
    den = torch.linalg.vector_norm(ref, dim=0).clamp_min(1e-300)
    e = (num / den).cpu().numpy()
    k99 = int(0.99 * (e.size - 1))
    part = np.partition(e, [e.size // 2, k99])
    return float(part[e.size // 2]), float(part[k99])


def test_fullsize_density_bit_exact(big):
    c = big["c"]
    for level, H in ((0, 1), (1, big["cr"])):
        n = big["n_f"] // H
        print(f"[fullsize] {big['name']}: deposit level {level}", flush=True)
        _, fx = c.deposit(big["pos"], big["cs"], level, fx=True)
        ref = oracle.deposit_fx(big["xf"], n, float(H))
        assert np.array_equal(fx.cpu().numpy().view(np.uint64), ref)
        del fx, ref


def test_fullsize_pp_sample_against_oracle(big):
    c = big["c"]
    n = big["xf"].shape[1]
    idx = np.sort(np.random.default_rng(12629).choice(n, 4096, replace=False))
    print(f"[fullsize] {big['name']}: PP sample", flush=True)
    acc = c.pp_force(big["pos"], big["cs"])
    got = acc[:, big["inv"][torch.from_numpy(idx).cuda()]].double().cpu().numpy()
    ref = oracle.Oracle(big["p"]).pp_accel_subset(big["xf"], idx)
    fr = np.linalg.norm(ref, axis=0)
    has = fr > 0
    floor = 1e-6 * np.median(fr[has])
    assert zero_force_ok(got, has, floor)
    e = np.linalg.norm(got - ref, axis=0)[has] / np.maximum(fr[has], floor)
    med, p99 = float(np.median(e)), float(np.percentile(e, 99))
    assert med < 1e-4 and p99 < 1e-3, (med, p99)


def test_fullsize_pp_adjoint_sample_against_oracle(big):
    """The PP adjoint (pair Jacobians applied to cotangent differences) of a
    seeded sample of 4096 particles against the oracle's FP64 adjoint for
    exactly those particles, with seeded Gaussian cotangents on all."""
    c = big["c"]
    n = big["xf"].shape[1]
    idx = np.sort(np.random.default_rng(12630).choice(n, 4096, replace=False))
    abar_in = np.random.default_rng(12631).standard_normal((3, n)).astype(np.float32)
    print(f"[fullsize] {big['name']}: PP adjoint sample", flush=True)
    ab_gpu = torch.from_numpy(abar_in).cuda()[:, big["perm"]].contiguous()   # IOS order
    xb = c.pp_force_backward(big["pos"], big["cs"], ab_gpu)
    got = xb[:, big["inv"][torch.from_numpy(idx).cuda()]].double().cpu().numpy()
    del xb, ab_gpu
    ref = oracle.Oracle(big["p"]).pp_adjoint_subset(big["xf"], abar_in.astype(np.float64), idx)
    fr = np.linalg.norm(ref, axis=0)
    has = fr > 0
    floor = 1e-6 * np.median(fr[has])
    assert zero_force_ok(got, has, floor)
    e = np.linalg.norm(got - ref, axis=0)[has] / np.maximum(fr[has], floor)
    med, p99 = float(np.median(e)), float(np.percentile(e, 99))
    assert med < 1e-4 and p99 < 1e-3, (med, p99)


def test_fullsize_fp32_against_fp64_form(big):
    c = big["c"]
    print(f"[fullsize] {big['name']}: FP32 vs FP64 forms", flush=True)
    a32 = c.force(big["pos"], big["cs"])
    a64 = c.force_f64(big["pos"], big["cs"])
    med, p99 = _stats(a32, a64)
    assert med < 1e-4 and p99 < 1e-3, (med, p99)


def test_fullsize_momentum_conservation(big):
    c = big["c"]
    for part in ("pm", "pp"):
        a = getattr(c, f"{part}_force")(big["pos"], big["cs"]).double()
        total = torch.linalg.vector_norm(a.sum(dim=1)).item()
        scale = torch.linalg.vector_norm(a, dim=0).sum().item()
        assert total <= 1e-6 * scale, (part, total, scale)
