"""GPU parity: every stage of the HIP path, called through the C ABI, against
the FP64 oracle on the same seeded inputs.

Bars: bit-exact for the integer work (IOS order, cell_start, the fixed-point
density, the drifted integer positions); FP32 results within the stated
tolerances of the FP64 oracle (forces: median relative error <= 1e-4 and
99th percentile <= 1e-3 per particle).
"""
import math

import numpy as np
import pytest

import oracle
import synthetic
from helpers import exact_sum_u64, force_stats, ios_decode, rel_err, ulp32, zero_force_ok

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MED, P99 = 1e-4, 1e-3


def _setup(n_fine, coarse_ratio, x_box, **kw):
    import paper_2512_12629_amd as m
    cfg = m.Config(n_fine=n_fine, coarse_ratio=coarse_ratio, **kw)
    c = m.Cube2(cfg, n_max=max(1, x_box.shape[1]))
    p = oracle.Params(n_fine=n_fine, coarse_ratio=coarse_ratio,
                      **{k: v for k, v in kw.items() if k in ("b_coarse", "b_fine", "b_pp", "m_p")})
    if "g_newton" in kw:
        p.G_N = kw["g_newton"]
    x = torch.from_numpy(np.ascontiguousarray(x_box)).cuda()
    pos, cs, perm = c.pack(x)
    return c, p, pos, cs, perm


def _np(t):
    return t.detach().cpu().numpy()


CASES = {
    # name: (n_fine, coarse_ratio, positions)
    "uniform_64": (64, 0, lambda: synthetic.uniform(32 ** 3, 101)),
    "clustered_64_two_level": (64, 4, lambda: synthetic.clustered(24, 0.25, 6, 512, 0.5 / 64, 102)),
    "zel_32_ragged": (32, 2, lambda: synthetic.zeldovich(13, 0.25, 103)),
    # the largest coarse ratio the library takes (8: a coarse mesh of 8^3)
    "clustered_64_ratio8": (64, 8, lambda: synthetic.clustered(24, 0.25, 6, 512, 0.5 / 64, 104)),
    # the single-level Zel'dovich workload at its stated size: 128^3 particles
    # (k^-2 field, rms 0.25 H_p), 256^3 mesh
    "zel128": (256, 0, lambda: synthetic.make("zel128")),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    n_fine, cr, gen = CASES[request.param]
    x = gen()
    c, p, pos, cs, perm = _setup(n_fine, cr, x)
    torch.cuda.synchronize()
    q_or = oracle.quantize(x, n_fine)
    return dict(name=request.param, x=x, c=c, p=p, pos=pos, cs=cs, perm=perm, q=q_or,
                n_fine=n_fine)


def _sorted_fine(case):
    perm_or, _, _ = oracle.ios_order(case["q"], case["n_fine"])
    return oracle.q_to_fine(case["q"][:, perm_or])


def test_pack_bit_exact(case):
    perm_or, cs_or, off_or = oracle.ios_order(case["q"], case["n_fine"])
    assert np.array_equal(_np(case["cs"]).view(np.uint32), cs_or)
    assert np.array_equal(_np(case["perm"]), perm_or.astype(np.int32))
    assert np.array_equal(_np(case["pos"]).view(np.uint16), off_or)
    q_gpu = ios_decode(_np(case["pos"]).view(np.uint16), _np(case["cs"]).view(np.uint32),
                       case["n_fine"])
    assert np.array_equal(q_gpu, case["q"][:, perm_or])


@pytest.mark.parametrize("n_fine,npart", [(256, 0), (256, 5), (128, 4097)])
def test_pack_sparse_bit_exact(n_fine, npart):
    """Few particles on a large mesh (stretches of thousands of empty cells
    between them), an empty input, and one key past a full 4096-key sort
    block: cell_start, order and offsets against the oracle."""
    rng = np.random.default_rng(110 + npart)
    x = rng.random((3, npart)).astype(np.float32)
    if npart >= 2:
        x[:, 1] = x[:, 0]                    # two particles in one cell
        x[:, -1] = np.float32(1.0 - 2.0 ** -24)  # the last cell of the box
    c, p, pos, cs, perm = _setup(n_fine, 0, x)
    torch.cuda.synchronize()
    q = oracle.quantize(x, n_fine)
    perm_or, cs_or, off_or = oracle.ios_order(q, n_fine)
    assert np.array_equal(_np(cs).view(np.uint32), cs_or)
    assert np.array_equal(_np(perm), perm_or.astype(np.int32))
    assert np.array_equal(_np(pos).view(np.uint16).reshape(3, -1), off_or.reshape(3, -1))


def test_green_table_within_one_ulp(case):
    c, p = case["c"], case["p"]
    for level, (H, n, b_a, b_prev) in enumerate(reversed(p.levels())):
        g_or = oracle.green_table(n, b_a / H, b_prev / H, p.alias_nmax)
        g = _np(c.green_table(level)).astype(np.float64)
        tol = ulp32(g_or) + 1e-30
        assert np.all(np.abs(g - g_or.astype(np.float32)) <= tol)


def test_deposit_bit_exact(case):
    c, p = case["c"], case["p"]
    xf = _sorted_fine(case)
    for level, (H, n, _, _) in enumerate(reversed(p.levels())):
        rho, fx = c.deposit(case["pos"], case["cs"], level, fx=True)
        acc_or = oracle.deposit_fx(xf, n, H)
        assert np.array_equal(_np(fx).view(np.uint64), acc_or)
        assert np.array_equal(_np(rho), oracle.density_f32(acc_or))
        assert exact_sum_u64(acc_or) == xf.shape[1] * 2 ** 45
    assert c.status() == 0


def test_fft_forward_matches_library_fft(case):
    c, p = case["c"], case["p"]
    for level, (H, n, _, _) in enumerate(reversed(p.levels())):
        rho = c.deposit(case["pos"], case["cs"], level)
        spec = _np(c.fft_r2c(rho, level)).astype(np.complex128)
        ref = np.fft.rfftn(_np(rho).astype(np.float64))
        err = np.linalg.norm(spec - ref) / np.linalg.norm(ref)
        assert err < 2e-6, err


def test_potential_against_oracle(case):
    c, p = case["c"], case["p"]
    o = oracle.Oracle(p)
    for level, (H, n, _, _) in enumerate(reversed(p.levels())):
        lvl_or = len(p.levels()) - 1 - level
        rho = c.deposit(case["pos"], case["cs"], level)
        phi = _np(c.potential(rho, level)).astype(np.float64)
        phi_or = oracle.potential(_np(rho).astype(np.float64), o.green(lvl_or))
        err = np.linalg.norm(phi - phi_or) / np.linalg.norm(phi_or)
        assert err < 2e-6, err


def test_interp_against_oracle(case):
    # same potential on both sides: isolates the stencil and the gather
    c, p = case["c"], case["p"]
    xf = _sorted_fine(case)
    lv = list(reversed(p.levels()))
    phis = [c.potential(c.deposit(case["pos"], case["cs"], l), l) for l in range(len(lv))]
    acc = _np(c.interp(case["pos"], case["cs"], phis[0], phis[1] if len(lv) > 1 else None))
    ref = np.zeros_like(acc, dtype=np.float64)
    for l, (H, n, _, _) in enumerate(lv):
        E = oracle.fd_force(_np(phis[l]).astype(np.float64))
        ref += oracle.interp(xf, E, H) / H ** 2
    med, p99, _ = force_stats(acc, ref)
    assert med < 1e-5 and p99 < 1e-4, (med, p99)


def test_pm_force_against_oracle(case):
    c, p = case["c"], case["p"]
    xf = _sorted_fine(case)
    acc = _np(c.pm_force(case["pos"], case["cs"]))
    ref = oracle.Oracle(p).pm_accel(xf)
    med, p99, _ = force_stats(acc, ref)
    assert med < MED and p99 < P99, (med, p99)


def test_pp_force_against_oracle(case):
    c, p = case["c"], case["p"]
    xf = _sorted_fine(case)
    acc = _np(c.pp_force(case["pos"], case["cs"]))
    ref = oracle.Oracle(p).pp_accel(xf)
    fr = np.linalg.norm(ref, axis=0)
    has = fr > 0
    # Particles whose only neighbours sit within ~1e-3 of the cutoff have
    # PP forces near 1e-16, where the oracle's FP64 difference
    # R(r, b_pp) - R(r, b_f) has lost every digit (the GPU evaluates the
    # exactly factored tail instead); errors are measured relative to
    # max(|F|, 1e-6 median |F|).
    floor = 1e-6 * np.median(fr[has])
    assert zero_force_ok(acc, has, floor)
    e = np.linalg.norm(acc - ref, axis=0)[has] / np.maximum(fr[has], floor)
    med, p99 = float(np.median(e)), float(np.percentile(e, 99))
    assert med < MED and p99 < P99, (med, p99)


EXACT = {
    "zel_32_ragged": (32, lambda: synthetic.zeldovich(13, 0.25, 103)),
    "clustered_32": (32, lambda: synthetic.clustered(12, 0.25, 1, 256, 0.5 / 32, 105)),
}


@pytest.mark.parametrize("name", list(EXACT))
def test_pp_force_against_exact(name):
    """FP32 PP against the exact rational PP sum of oracle.exact (stored in
    tests/golden/pp_exact_*.txt): median <= 1e-4, p99 <= 1e-3 with the
    floor of the oracle comparison above."""
    import os
    import paper_2512_12629_amd as m
    n_f, gen = EXACT[name]
    x = gen()
    ref = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                  f"pp_exact_{name}.txt")).T
    c = m.Cube2(m.Config(n_fine=n_f), n_max=x.shape[1])
    pos, cs, perm = c.pack(torch.from_numpy(x).cuda())
    acc = np.empty_like(ref)
    acc[:, _np(perm).astype(np.int64)] = _np(c.pp_force(pos, cs))
    fr = np.linalg.norm(ref, axis=0)
    has = fr > 0
    floor = 1e-6 * np.median(fr[has])
    assert zero_force_ok(acc, has, floor)
    e = np.linalg.norm(acc - ref, axis=0)[has] / np.maximum(fr[has], floor)
    med, p99 = float(np.median(e)), float(np.percentile(e, 99))
    assert med < MED and p99 < P99, (med, p99)


def test_pp_pair_law_bit_exact_two_particles():
    """Two particles: the PP kernel's force on each is g(D) D with g the FP32
    pair law that cube2_pair_law_f32 evaluates on the host with the same
    operations, so the device result is bit-exact against g * D rounded once
    (G m = 1; the Kahan sum of one term is that term).  Separations span the
    pair law's pieces, in both directions and across cell and tile edges."""
    import paper_2512_12629_amd as m
    n_f = 16
    c = m.Cube2(m.Config(n_fine=n_f), n_max=2)
    rng = np.random.default_rng(29)
    L = n_f << 15
    for k in range(24):
        r = float(np.exp(rng.uniform(np.log(2.0 ** -13), np.log(2.2))))
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        qi = rng.integers(0, L, 3)
        qj = (qi + np.rint(u * r * 2 ** 15).astype(np.int64)) % L
        x = (np.stack([qi, qj], axis=1).astype(np.float64) + 0.5) / L
        pos, cs, perm = c.pack(torch.from_numpy(x.astype(np.float32)).cuda())
        q = np.floor(x.astype(np.float32).astype(np.float64) * L).astype(np.int64)
        d = (q[:, 1] - q[:, 0] + L // 2) % L - L // 2           # j - i, minimum image
        dj = (d * 2.0 ** -15).astype(np.float32).reshape(3, 1)
        g = m.cube2_pair_law_f32(c.ctx, dj)[0]
        want = np.stack([np.float32(g) * dj[:, 0], -(np.float32(g) * dj[:, 0])], axis=1)
        acc = np.empty((3, 2), np.float32)
        acc[:, _np(perm).astype(np.int64)] = _np(c.pp_force(pos, cs))
        assert np.array_equal(acc, want), (k, r, acc, want)


def test_total_force_against_oracle(case):
    c, p = case["c"], case["p"]
    xf = _sorted_fine(case)
    acc = _np(c.force(case["pos"], case["cs"]))
    ref = oracle.Oracle(p).accel(xf)
    med, p99, _ = force_stats(acc, ref)
    assert med < MED and p99 < P99, (med, p99)


def test_force_entry_equals_pm_then_pp(case):
    """cube2_force (the PP on the context's side stream beside the PM force,
    its own tile queue, summed after the join) against cube2_pm_force then
    cube2_pp_force with accumulate: bit for bit, on two calls in a row."""
    c = case["c"]
    ref = c.pp_force(case["pos"], case["cs"], c.pm_force(case["pos"], case["cs"]))
    for _ in range(2):
        acc = c.force(case["pos"], case["cs"])
        torch.cuda.synchronize()
        assert torch.equal(acc, ref)


def test_force_entry_output_not_16_byte_aligned(case):
    """cube2_force into an output that starts 4 bytes into its buffer (the
    final PM + PP sum then takes its scalar path instead of 16-byte
    accesses): the same floats as the separate entry points."""
    import paper_2512_12629_amd as m
    c, pos, cs = case["c"], case["pos"], case["cs"]
    n = pos.shape[1]
    ref = c.pp_force(pos, cs, c.pm_force(pos, cs))
    buf = torch.full((3 * n + 1,), float("nan"), dtype=torch.float32, device="cuda")
    acc = buf[1:].view(3, n)
    assert acc.data_ptr() % 16 != 0
    m.cube2_force(c.ctx, pos, cs, acc, c.work)
    torch.cuda.synchronize()
    assert torch.equal(acc, ref)
    assert torch.isnan(buf[0])


def test_force_backward_entry_equals_pm_then_pp(case):
    """cube2_force_backward (PP adjoint on the side stream beside the PM
    adjoint) against the two adjoint entry points in sequence: bit for bit,
    on two calls in a row (every adjoint scatter sums in exact fixed point)."""
    import paper_2512_12629_amd as m
    c, pos, cs = case["c"], case["pos"], case["cs"]
    n = pos.shape[1]
    g = torch.Generator(device="cuda")
    g.manual_seed(211)
    abar = torch.randn((3, n), device="cuda", generator=g)
    ref = torch.empty_like(abar)
    m.cube2_pm_force_backward(c.ctx, pos, cs, abar, ref, c.work)
    m.cube2_pp_force_backward(c.ctx, pos, cs, abar, ref, c.work, accumulate=True)
    for _ in range(2):
        xb = torch.empty_like(abar)
        m.cube2_force_backward(c.ctx, pos, cs, abar, xb, c.work)
        torch.cuda.synchronize()
        assert torch.equal(xb, ref)


def test_kick_drift_bit_exact(case):
    c, p = case["c"], case["p"]
    N = case["x"].shape[1]
    rng = np.random.default_rng(7)
    vel = rng.standard_normal((3, N)).astype(np.float32)
    acc = _np(c.force(case["pos"], case["cs"]))
    kick, drift = 0.05, 0.3
    pos2, cs2, vel2, perm = c.kick_drift(case["pos"], case["cs"], torch.from_numpy(vel).cuda(),
                                        torch.from_numpy(acc).cuda(), kick, drift)
    perm_or0, _, _ = oracle.ios_order(case["q"], case["n_fine"])
    q0 = case["q"][:, perm_or0]
    q1, v1 = oracle.kick_drift_q(q0, vel, acc, kick, drift, case["n_fine"])
    perm1, cs1, off1 = oracle.ios_order(q1, case["n_fine"])
    assert np.array_equal(_np(cs2).view(np.uint32), cs1)
    assert np.array_equal(_np(perm), perm1.astype(np.int32))
    assert np.array_equal(_np(pos2).view(np.uint16), off1)
    vg, vo = _np(vel2), v1[:, perm1]
    bad = vg != vo
    assert not bad.any(), (int(bad.sum()), vg[bad][:5], vo[bad][:5])


def test_reduce_matches_fp64(case):
    c, p = case["c"], case["p"]
    N = case["x"].shape[1]
    rng = np.random.default_rng(8)
    vel = rng.standard_normal((3, N)).astype(np.float32)
    acc = _np(c.force(case["pos"], case["cs"]))
    out = c.reduce(torch.from_numpy(vel).cuda(), torch.from_numpy(acc).cuda())
    v, a = vel.astype(np.float64), acc.astype(np.float64)
    ref = list(v.sum(axis=1)) + [0.5 * np.sum(v * v)] + list(a.sum(axis=1)) + \
        [np.max(np.linalg.norm(a, axis=0))]
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-9 * np.abs(a).max())
    # momentum conservation of the whole force: sum of accelerations ~ 0
    assert max(abs(x) for x in out[4:7]) < 1e-4 * np.abs(a).sum() / N * N ** 0.5 + 1e-3


def test_deterministic_repeat(case):
    c = case["c"]
    a1 = _np(c.force(case["pos"], case["cs"]))
    a2 = _np(c.force(case["pos"], case["cs"]))
    assert np.array_equal(a1, a2)


def test_overflow_guard_sets_status():
    import paper_2512_12629_amd as m
    # 70000 particles inside one tile of a two-level mesh: the coarse guard
    # (2^16 own particles per tile) trips; the call itself still completes.
    rng = np.random.default_rng(9)
    x = (rng.random((3, 70000)) * (16 / 64)).astype(np.float32)
    c = m.Cube2(m.Config(n_fine=64, coarse_ratio=4), n_max=70000)
    pos, cs, _ = c.pack(torch.from_numpy(x).cuda())
    c.deposit(pos, cs, 0)
    assert c.status() == 0
    c.deposit(pos, cs, 1)
    assert c.status() == -4          # CUBE2_EOVERFLOW
    assert c.status() == 0           # cleared by the read


def test_nonfinite_kick_sets_status():
    import paper_2512_12629_amd as m
    # A NaN and an infinite acceleration, and a finite velocity whose drift
    # overflows the 64-bit position arithmetic: those three particles keep
    # their positions, every other particle moves exactly as in a run where
    # they stand still, and the status reports it once.
    rng = np.random.default_rng(11)
    n = 5000
    x = rng.random((3, n)).astype(np.float32)
    c = m.Cube2(m.Config(n_fine=32), n_max=n)
    pos, cs, _ = c.pack(torch.from_numpy(x).cuda())
    vel = (0.2 * rng.standard_normal((3, n))).astype(np.float32)
    acc = rng.standard_normal((3, n)).astype(np.float32)
    for i in (17, 300, 2500):
        acc[:, i] = 0.0
        vel[:, i] = 0.0
    ok = c.kick_drift(pos, cs, torch.from_numpy(vel).cuda(), torch.from_numpy(acc).cuda(), 0.05, 0.3)
    assert c.status() == 0
    acc[1, 17] = np.nan
    acc[2, 2500] = np.inf
    vel[0, 300] = 3.0e38                 # finite, but 0.3 * 3e38 * 2^15 passes 2^62
    bad = c.kick_drift(pos, cs, torch.from_numpy(vel).cuda(), torch.from_numpy(acc).cuda(), 0.05, 0.3)
    assert c.status() == -7          # CUBE2_ENONFINITE
    assert c.status() == 0           # cleared by the read
    for a, b in zip(ok[:2], bad[:2]):
        assert torch.equal(a, b)
    assert torch.equal(ok[3], bad[3])
    v_ok, v_bad, perm = _np(ok[2]), _np(bad[2]), _np(ok[3])
    keep = (perm != 17) & (perm != 2500) & (perm != 300)
    assert np.array_equal(v_ok[:, keep], v_bad[:, keep])
    assert not np.isfinite(v_bad[:, (perm == 17) | (perm == 2500)]).all()
    assert v_bad[0, perm == 300][0] == np.float32(3.0e38)


def test_empty_input():
    import paper_2512_12629_amd as m
    c = m.Cube2(m.Config(n_fine=32), n_max=1)
    x = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    pos, cs, perm = c.pack(x)
    assert int(cs.abs().sum()) == 0
    rho = c.deposit(pos, cs, 0)
    assert float(rho.abs().sum()) == 0.0
    acc = c.force(pos, cs)
    assert acc.shape == (3, 0)
