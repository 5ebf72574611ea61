"""Oracle parity of the production mesh path at the benchmark mesh sizes,
where the FP32 column transforms of 512 and 1024 points move their LDS
transposes as split real/imaginary halves and the z pass reads the z-ordered
copy of the Green's table (neither of which the 64^3 cases reach):

* clu256 (256^3 particles, fine 512^3, coarse 128^3) and clu512 (512^3
  particles, fine 1024^3, coarse 256^3), in the launch configuration the
  benchmark times (one context per workload, all particles resident);
* the forward R2C transform of the GPU's own FP32 density on both levels
  against scipy's FFT of the same values in FP64 (a library routine taken as
  the definition of the unnormalised DFT), relative L2 <= 2e-6;
* the Green's tables (eq. 11) at n = 1024, 512, 256 and 128 against the
  oracle's point evaluation on seeded octant points, every edge and Nyquist
  plane included: within one FP32 ulp;
* the potential (eqs. 9-13 through both FFTs and the z-ordered G) of a sum of
  plane waves on every level of both workloads: for rho = sum_j a_j cos(k_j.n
  + p_j) the exact potential is sum_j a_j G(k_j) cos(k_j.n + p_j) (G real and
  even), evaluated at sampled nodes with the oracle's G(k_j);
* clu256: the potential of the GPU density on both levels against the
  oracle's FFT-G-IFFT (relative L2 <= 2e-6) and the FD force + CIC
  interpolation of every particle from the same potentials against the
  oracle's stencil and gather (median <= 1e-5, p99 <= 1e-4).
"""
import numpy as np
import pytest

import oracle
import synthetic
from helpers import force_stats, ulp32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WORKLOADS = {"clu256": (512, 4), "clu512": (1024, 4)}


def _workers():
    return 16


def _rfftn64(a):
    import scipy.fft
    return scipy.fft.rfftn(a, workers=_workers())


@pytest.fixture(scope="module", params=list(WORKLOADS))
def prod(request):
    import paper_2512_12629_amd as m
    name = request.param
    n_f, cr = WORKLOADS[name]
    print(f"[production] {name}: generating", flush=True)
    x = synthetic.make(name)
    c = m.Cube2(m.Config(n_fine=n_f, coarse_ratio=cr), n_max=x.shape[1])
    pos, cs, perm = c.pack(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    yield dict(name=name, x=x, c=c, pos=pos, cs=cs, perm=perm, n_f=n_f, cr=cr,
               p=oracle.Params(n_fine=n_f, coarse_ratio=cr))
    del c, pos, cs, perm
    torch.cuda.empty_cache()


def _levels(prod):
    """[(level, H, n, b_level, b_prev)] in the library's level numbering
    (0 = fine), lengths in fine cells."""
    lv = list(reversed(prod["p"].levels()))
    return [(l, H, n, b, bp) for l, (H, n, b, bp) in enumerate(lv)]


def test_production_fft_forward_against_library_fft(prod):
    c = prod["c"]
    for level, H, n, _, _ in _levels(prod):
        print(f"[production] {prod['name']}: R2C level {level} (n = {n})", flush=True)
        rho = c.deposit(prod["pos"], prod["cs"], level)
        spec = c.fft_r2c(rho, level)
        ref = _rfftn64(rho.cpu().numpy().astype(np.float64))
        num = den = 0.0
        for z0 in range(0, n, 64):          # slabs of kz: bounded host memory
            r = torch.from_numpy(ref[z0:z0 + 64]).cuda()
            g = spec[z0:z0 + 64].to(torch.complex128)
            num += float(torch.linalg.vector_norm(g - r) ** 2)
            den += float(torch.linalg.vector_norm(r) ** 2)
            del r, g
        del ref, spec, rho
        err = (num / den) ** 0.5
        assert err < 2e-6, (level, n, err)


def _octant_samples(n, k, seed):
    """k octant points m in [0, n/2]^3: every coordinate is 0, n/2, n/2 - 1
    or 1 with probability 1/8 each, else uniform; plus the 8 corners."""
    rng = np.random.default_rng(seed)
    h = n // 2
    m = rng.integers(0, h + 1, size=(k, 3))
    u = rng.random((k, 3))
    m = np.where(u < 0.125, 0, m)
    m = np.where((u >= 0.125) & (u < 0.25), h, m)
    m = np.where((u >= 0.25) & (u < 0.375), h - 1, m)
    m = np.where((u >= 0.375) & (u < 0.5), 1, m)
    corners = np.array([[a, b, cc] for a in (0, h) for b in (0, h) for cc in (0, h)])
    return np.concatenate([m, corners])


def test_production_green_tables_sampled_against_oracle(prod):
    c = prod["c"]
    for level, H, n, b, bp in _levels(prod):
        print(f"[production] {prod['name']}: Green's table level {level} (n = {n})", flush=True)
        g = c.green_table(level).cpu().numpy()
        pts = _octant_samples(n, 3000, 12629 + n)
        b_prev = bp / H
        ref = np.array([oracle.green_point(n, mm, b / H, b_prev) for mm in pts])
        got = g[pts[:, 2], pts[:, 1], pts[:, 0]].astype(np.float64)   # [mz][my][mx]
        tol = ulp32(ref) + 1e-30
        bad = np.abs(got - ref.astype(np.float32)) > tol
        assert not bad.any(), (level, pts[bad][:5], got[bad][:5], ref[bad][:5])
        del g


def _plane_waves(n, seed, count=12):
    """(modes (count, 3) ints in (-n/2, n/2], amplitudes, phases); distinct
    up to sign, none at k = 0, Nyquist components included."""
    rng = np.random.default_rng(seed)
    h = n // 2
    modes, seen = [], set()
    while len(modes) < count:
        mm = rng.integers(-h + 1, h + 1, size=3)
        if len(modes) % 4 == 0:
            mm[rng.integers(0, 3)] = h          # a Nyquist component
        if len(modes) % 5 == 1:
            mm = rng.integers(-4, 5, size=3)    # a long wave (large G)
        key = tuple(int(v) for v in mm)
        neg = tuple(int((-v + h - 1) % n - h + 1) for v in mm)
        if key == (0, 0, 0) or key in seen or neg in seen:
            continue
        seen.add(key)
        modes.append(mm)
    amp = rng.uniform(0.5, 1.5, count)
    ph = rng.uniform(0, 2 * np.pi, count)
    return np.array(modes, dtype=np.int64), amp, ph


def _wave_mesh(n, modes, amp, ph):
    """rho[z][y][x] = sum_j amp_j cos(2 pi (m_j . (x, y, z) mod n) / n + ph_j),
    in FP64 on the device (an input generator: no step of the method), cast
    to FP32."""
    ar = torch.arange(n, dtype=torch.int64, device="cuda")
    rho = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    for (mx, my, mz), a, p in zip(modes.tolist(), amp.tolist(), ph.tolist()):
        t = ((mz * ar).view(n, 1, 1) + (my * ar).view(1, n, 1) + (mx * ar).view(1, 1, n)) % n
        rho += a * torch.cos(t.to(torch.float64) * (2 * np.pi / n) + p)
        del t
    out = rho.to(torch.float32)
    del rho
    return out


def test_production_potential_of_plane_waves(prod):
    """phi of a sum of plane waves = the same waves scaled by G(k) (the
    convolution theorem with G real and even), on both levels: sampled nodes
    within 2e-6 relative L2 of the closed form."""
    c = prod["c"]
    for level, H, n, b, bp in _levels(prod):
        print(f"[production] {prod['name']}: plane waves level {level} (n = {n})", flush=True)
        modes, amp, ph = _plane_waves(n, 4711 + n)
        Gk = np.array([oracle.green_point(n, np.abs(mm), b / H, bp / H) for mm in modes])
        rho = _wave_mesh(n, modes, amp, ph)
        phi = c.potential(rho, level)
        del rho
        rng = np.random.default_rng(99 + n)
        nodes = rng.integers(0, n, size=(20000, 3))          # (x, y, z)
        got = phi[torch.from_numpy(nodes[:, 2]).cuda(), torch.from_numpy(nodes[:, 1]).cuda(),
                  torch.from_numpy(nodes[:, 0]).cuda()].double().cpu().numpy()
        del phi
        t = (nodes @ modes.T) % n                              # (nodes, modes)
        want = (np.cos(t * (2 * np.pi / n) + ph) * (amp * Gk)).sum(axis=1)
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert err < 2e-6, (level, n, err)


def test_production_potential_and_interp_against_oracle(prod):
    """clu256 only (the oracle's 513^3 Green's table at n = 1024 takes
    minutes on the host): the GPU's potential of its own density on both
    levels against the oracle's FFT-G-IFFT, and the FD + CIC gather of every
    particle from the same potentials."""
    if prod["name"] != "clu256":
        pytest.skip("oracle potential at n = 1024 is covered by the sampled G and plane waves")
    c, p = prod["c"], prod["p"]
    o = oracle.Oracle(p)
    lv = _levels(prod)
    phis = []
    for level, H, n, b, bp in lv:
        print(f"[production] clu256: potential level {level} (n = {n})", flush=True)
        rho = c.deposit(prod["pos"], prod["cs"], level)
        phi = c.potential(rho, level)
        rho64 = rho.cpu().numpy().astype(np.float64)
        ref = oracle.potential(rho64, o.green(len(lv) - 1 - level), workers=_workers())
        got = phi.cpu().numpy().astype(np.float64)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err < 2e-6, (level, err)
        phis.append(phi)
        del rho, rho64, ref
    print("[production] clu256: interpolation", flush=True)
    acc = c.interp(prod["pos"], prod["cs"], phis[0], phis[1]).cpu().numpy()
    q = oracle.quantize(prod["x"], prod["n_f"])
    perm_or, _, _ = oracle.ios_order(q, prod["n_f"])
    xf = oracle.q_to_fine(q[:, perm_or])
    assert np.array_equal(prod["perm"].cpu().numpy(), perm_or.astype(np.int32))
    ref = np.zeros_like(acc, dtype=np.float64)
    for level, H, n, b, bp in lv:
        E = oracle.fd_force(phis[level].cpu().numpy().astype(np.float64))
        ref += oracle.interp(xf, E, H) / H ** 2
        del E
    med, p99, _ = force_stats(acc, ref)
    assert med < 1e-5 and p99 < 1e-4, (med, p99)
