"""Benchmark of the CUBE2 force step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload clu512]

Times K force evaluations (cube2_force: two-level PM + PP, the PP on the
context's side stream beside the PM, inputs resident in HBM) with HIP events
on the caller's stream, which waits for both, then the full step (force +
kick-drift + IOS re-sort), the force adjoint (PM + PP backward), the stages,
and the differentiable leapfrog (Cube2Leapfrog forward over 4 steps with a
checkpoint every 2, then loss.backward()), and prints one JSON line.
value = N / t_force (particles per second per force step);
backward_forward_ratio is the leapfrog's backward time over its forward time.
A CPU baseline (the FP64 oracle, on a bounded sample of the same workload
recipe) is timed on the host.

    python bench.py --standalone      # only the separate PM/PP entry points
                                      # and their adjoints (profiler runs)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthetic  # noqa: E402

HBM_PEAK_GBS = 8000.0
# FP32 VALU without packed math: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA)
VALU_FP32_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12   # 78.64

WORKLOADS = {
    "clu512": dict(n_fine=1024, coarse_ratio=4,
                   desc="512^3 particles, Zel'dovich k^-2 (rms 0.25 H_p) + 8000 Plummer spheres "
                        "x 2048 (a = 0.5 fine cell); fine mesh 1024^3, coarse 256^3; "
                        "b_c=14, b_f=2 (PP cutoff), b_pp=0.2 fine cells"),
    "clu256": dict(n_fine=512, coarse_ratio=4,
                   desc="256^3 particles, Zel'dovich + 1000 Plummer spheres x 2048; fine 512^3, "
                        "coarse 128^3"),
    "clu256_halos": dict(n_fine=512, coarse_ratio=4,
                         desc="256^3 particles, Zel'dovich + 125 Plummer spheres x 16384; fine "
                              "512^3, coarse 128^3"),
    "zel128": dict(n_fine=256, coarse_ratio=0,
                   desc="128^3 particles, Zel'dovich k^-2; single-level 256^3 mesh"),
}

# Algorithmic FP32 flops (FMA = 2) of one in-cutoff PP pair, counted from
# the arithmetic of the compiled inner loop: 3 differences, s = r^2 with its
# offset (3 FMA, 6), the local variable (1), w = 1 - s/b_f^2 (1 FMA, 2),
# 3 Horner FMA (6), w^2, w^4, h w and g (4), 3 accumulating FMA (6).  The
# table index (shift, mask, or) is integer work and is not counted.
PP_FLOPS_PER_PAIR = 28


# VALU instructions per candidate pair of the compiled forward PP inner loop
# (gfx950 ISA: 42 per iteration of the two-pair unrolled loop), and the
# unpacked FP32 VALU issue rate (lane-ops per second).
PP_VALU_PER_PAIR = 21.0
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9


def step_reference_bytes(n_particles: int, meshes) -> float:
    """HBM bytes of one force evaluation in the reference traffic model:
    per level of n^3 cells, the density write (4 B/cell), five read+write
    sweeps over the n^2 (n/2+1) half spectrum (8 B per complex value), one
    read of the octant Green's table, one read of the potential (4 B/cell);
    per particle, two sweeps over the IOS data (10 B each) and the 12 B
    acceleration write."""
    b = 32.0 * n_particles
    for n in meshes:
        h = n // 2 + 1
        b += 4.0 * n ** 3 + 5 * 2 * 8.0 * h * n * n + 4.0 * h ** 3 + 4.0 * n ** 3
    return b


def step_compulsory_bytes(n_particles: int, meshes) -> float:
    """HBM bytes of one force evaluation in the compulsory traffic model:
    per level of n^3 cells, the density write (4 B/cell), one read and one
    write per transform (the real mesh, 4 B/cell, and the half spectrum,
    8 B per complex value, for the forward and the inverse FFT), one read of
    the octant Green's table and one of the potential; per particle as in the
    reference model.  No per-axis FFT reaches it (a 1024^2 plane does not fit
    a CU's LDS), so it is a bound, not a target."""
    b = 32.0 * n_particles
    for n in meshes:
        h = n // 2 + 1
        b += 4.0 * n ** 3 + 2 * (4.0 * n ** 3 + 8.0 * h * n * n) + 4.0 * h ** 3 + 4.0 * n ** 3
    return b


def pair_counts():
    path = os.path.join(ROOT, "tests", "golden", "pair_counts.json")
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pp_kernel_clu512_traffic.txt")
PP_SOURCES = [os.path.join(ROOT, "paper_2512_12629_amd", "csrc", "pp.hip")]


def source_digest(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per pp_kernel launch from the FETCH_SIZE / WRITE_SIZE counter
    passes recorded in the traffic summary, each divided by what the same
    counter reads per byte for a plain copy kernel of known size.  None when
    the summary is absent, covers another workload, or was taken on another
    version of the kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith(("#", " ", "|")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("workload") != workload or kv.get("source_digest") != source_digest(PP_SOURCES):
            return None
        copy_bytes = float(kv["copy_bytes"])
        f_scale = float(kv["copy_fetch_kib"]) * 1024.0 / copy_bytes
        w_scale = float(kv["copy_write_kib"]) * 1024.0 / copy_bytes
        return (float(kv["pp_fetch_kib"]) * 1024.0 / f_scale
                + float(kv["pp_write_kib"]) * 1024.0 / w_scale)
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def fft_bytes_reference(n: int, pitch: int) -> float:
    """Traffic of the 5-sweep FFT-G-IFFT pipeline of one level, bytes.

    x pass: read n^3 reals, write n*n*pitch complex; y pass, z pass (with G),
    inverse y: read+write the spectrum; G octant read once; inverse x: read
    the spectrum, write n^3 reals."""
    spec = n * n * pitch * 8.0
    real = n ** 3 * 4.0
    h = n // 2 + 1
    return (real + spec) + 2 * spec + (2 * spec + h ** 3 * 4.0) + 2 * spec + (spec + real)


def _oracle_force_time(workload: str, scale: int, min_total_s: float = 10.0, max_reps: int = 6):
    """Times of the oracle's full force on the workload recipe at 1/scale^3
    of the volume, repeated until about min_total_s of CPU work is timed."""
    import oracle
    w = WORKLOADS[workload]
    n_p = synthetic.WORKLOADS[workload]["n_p"] // scale
    n_f = w["n_fine"] // scale
    x = synthetic.make(workload, n_p=n_p)
    p = oracle.Params(n_fine=n_f, coarse_ratio=w["coarse_ratio"])
    o = oracle.Oracle(p)
    for lvl in range(len(p.levels())):
        o.green(lvl)                      # tables are built before the timing
    xf = oracle.q_to_fine(oracle.quantize(x, n_f))
    times = []
    while not times or (sum(times) < min_total_s and len(times) < max_reps):
        t0 = time.perf_counter()
        o.accel(xf)
        times.append(time.perf_counter() - t0)
    return x.shape[1], n_f, times


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _single_thread_probe(workload: str, scale: int):
    """One oracle force on the 1/scale^3 sample in a child process limited to
    one OpenMP thread (the thread count is fixed when the runtime starts)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-probe", workload,
                        str(scale)], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(workload: str):
    """Oracle (FP64, as is) on a bounded sample: the same recipe (same sphere
    density) at 1/64 of the volume, timed over repeated evaluations until
    about 10 s of CPU work is covered, on all host threads; and one
    evaluation at 1/512 of the volume on a single thread."""
    scale = 4 if workload == "clu512" else 2
    n, n_f, times = _oracle_force_time(workload, scale)
    dt = sum(times) / len(times)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": n / dt, "unit": "particles/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
           "sample": f"{workload} recipe at 1/{scale ** 3} volume: {n} particles, "
                     f"fine mesh {n_f}^3, full FP64 PM+PP force, mean of {len(times)} "
                     f"evaluations, {dt:.2f} s each, {threads} OpenMP threads (the numpy "
                     f"FFT steps run on one)"}
    st = _single_thread_probe(workload, 2 * scale)
    if st:
        out["single_thread"] = {"value": st["particles"] / st["seconds"], "unit": "particles/s",
                                "sample": f"1/{(2 * scale) ** 3} volume: {st['particles']} "
                                          f"particles, fine mesh {st['n_fine']}^3, one "
                                          f"evaluation, {st['seconds']:.2f} s"}
    return out


def leapfrog_timing(m, c, x_gpu, N, steps: int, ckpt: int, reps: int):
    """Wall time (HIP events on the caller's stream) of the differentiable
    multi-step leapfrog: Cube2Leapfrog forward (steps force + kick-drift
    steps, state checkpoints every ckpt steps, final CIC density) with the
    loss sum (rho - rho_target)^2, and loss.backward() (checkpoint segment
    recomputation, kick-drift and force adjoints, deposit adjoint)."""
    import torch
    from paper_2512_12629_amd.autograd import Cube2Leapfrog
    pos, cs, _ = c.pack(x_gpu)
    amax = float(torch.linalg.vector_norm(c.force(pos, cs), dim=0).max())
    dt = 0.1 * (1.0 / amax) ** 0.5            # 0.1 sqrt(H_f / max|a_0|)
    target = c.deposit(pos, cs, 0)
    del pos, cs
    stream = torch.cuda.current_stream()
    fw, bw = [], []
    for r in range(reps + 1):                   # the first repetition warms up
        x0 = x_gpu.clone().requires_grad_(True)
        v0 = torch.zeros_like(x0).requires_grad_(True)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        e[0].record(stream)
        rho = Cube2Leapfrog.apply(x0, v0, c, steps, dt, dt, ckpt)
        loss = ((rho - target) ** 2).sum()
        e[1].record(stream)
        loss.backward()
        e[2].record(stream)
        torch.cuda.synchronize()
        if r:
            fw.append(e[0].elapsed_time(e[1]))
            bw.append(e[1].elapsed_time(e[2]))
        del x0, v0, rho, loss
    f, b = float(np.median(fw)), float(np.median(bw))
    return {"steps": steps, "ckpt_every": ckpt, "dt": dt, "repetitions": reps,
            "forward_ms": f, "backward_ms": b, "backward_forward_ratio": b / f}


def fp64_comparison(m, cfg, c, pos, cs, N, ms32, stream, timed):
    """The FP64 plain form on the same particles: its force time, the FP32
    speedup over it, and the per-particle error of the FP32 force (and the
    norm-relative error of the FP32 fine potential) against it."""
    import dataclasses
    import torch
    a32 = c.force(pos, cs)
    rho32, fx = c.deposit(pos, cs, 0, fx=True)
    phi32 = c.potential(rho32, 0)
    del rho32
    cfg64 = dataclasses.replace(cfg, flags=cfg.flags | m.CUBE2_FP64_FORM)
    c64 = m.Cube2(cfg64, n_max=N)
    acc64 = torch.empty((3, N), dtype=torch.float64, device="cuda")

    def force64():
        m.cube2_pm_force_f64(c64.ctx, pos, cs, acc64, c64.work)
        m.cube2_pp_force_f64(c64.ctx, pos, cs, acc64, c64.work, accumulate=True)

    force64()
    t64 = timed(force64, 3)
    num = torch.linalg.vector_norm(a32.double() - acc64, dim=0)
    den = torch.linalg.vector_norm(acc64, dim=0).clamp_min(1e-300)
    e = (num / den).cpu().numpy()
    k99 = int(0.99 * (e.size - 1))
    part = np.partition(e, [e.size // 2, k99])
    unit = 2.0 ** -48 if cfg.flags & m.CUBE2_ASSIGN_TSC else 2.0 ** -45  # accumulator unit
    rho64 = fx.to(torch.float64).mul_(unit)
    del fx
    phi64 = c64.potential_f64(rho64, 0)
    perr = float(torch.linalg.vector_norm(phi32.double() - phi64) / torch.linalg.vector_norm(phi64))
    del c64, acc64, rho64, phi64, phi32, a32
    torch.cuda.empty_cache()
    ms64 = float(np.median(t64))
    return {"force_ms": ms64, "fp32_speedup": ms64 / ms32,
            "force_rel_err_median": float(part[e.size // 2]), "force_rel_err_p99": float(part[k99]),
            "force_rel_err_max": float(e.max()), "fine_potential_rel_err": perr}


def pair_force_eq2(r, b):
    """R(r, b) of eq. (2) (G m = 1), the softened pair force the method
    approximates; r, b in fine cells."""
    r = np.asarray(r, dtype=np.float64)
    t = r / b
    inner = (64 / 5 * t - 256 / 5 * t ** 3 + 32 * t ** 4 + 1536 / 35 * t ** 5 - 192 / 5 * t ** 6) / b ** 2
    outer = (3 / 35 / np.maximum(t, 1e-300) ** 2 - 32 / 5 + 256 / 5 * t - 96 * t ** 2 + 256 / 5 * t ** 3
             + 32 * t ** 4 - 1536 / 35 * t ** 5 + 64 / 5 * t ** 6) / b ** 2
    return np.where(t >= 1, 1 / np.maximum(r, 1e-300) ** 2, np.where(t < 0.5, inner, outer))


def pairwise_experiment(args):
    """The pairwise force-accuracy experiment of section 3.1 (Fig. 1) with
    isolated boundaries (appendix A): single particle pairs at random
    positions and orientations in the isolation box, the GPU's total force
    (both PM levels + PP) against the softened pair force R(r, b_pp), per
    log-spaced bin of r: magnitude residual F/R - 1 and direction error
    theta = acos(F.R / F R)."""
    import torch
    import paper_2512_12629_amd as m
    n_f, cr = 256, 4
    flags = m.CUBE2_ISOLATED | (m.CUBE2_ASSIGN_TSC if args.assign == "tsc" else 0)
    cfg = m.Config(n_fine=n_f, coarse_ratio=cr, b_fine=args.pair_b_fine, b_pp=args.pair_b_pp,
                   flags=flags)
    c = m.Cube2(cfg, n_max=2)
    L = n_f / 2                                   # isolation box, fine cells
    edges = np.exp(np.linspace(np.log(0.05), np.log(L / 2), 31))
    rng = np.random.default_rng(12629)
    bins = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        res, th = [], []
        for _ in range(args.pairs_per_bin):
            r = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            # both particles inside [2, L - 2] on every axis
            a0 = 2.0 + np.maximum(-r * u, 0.0) + rng.random(3) * (L - 4.0 - r * np.abs(u))
            xf = np.stack([a0, a0 + r * u], axis=1)
            x32 = (xf / n_f).astype(np.float32)
            pos, cs, perm = c.pack(torch.from_numpy(x32).cuda())
            acc = np.empty((3, 2))
            acc[:, perm.cpu().numpy().astype(np.int64)] = c.force(pos, cs).double().cpu().numpy()
            q = np.floor(x32.astype(np.float64) * (n_f << 15)) / (1 << 15)   # quantised fine positions
            d = q[:, 1] - q[:, 0]
            rq = float(np.linalg.norm(d))
            R = float(pair_force_eq2(rq, cfg.b_pp))
            F = acc[:, 0]
            res.append(np.linalg.norm(F) / R - 1.0)
            th.append(float(np.arccos(np.clip(F @ d / (np.linalg.norm(F) * rq), -1.0, 1.0))))
        res, th = np.array(res), np.array(th)
        bins.append({"r_lo": float(lo), "r_hi": float(hi), "resid_mean": float(res.mean()),
                     "resid_std": float(res.std()), "resid_min": float(res.min()),
                     "resid_max": float(res.max()), "theta_mean": float(th.mean()),
                     "theta_max": float(th.max())})
    allres = np.array([b[k] for b in bins for k in ("resid_min", "resid_max")])
    out = {"experiment": "pairwise force accuracy, isolated boundaries (section 3.1, appendix A)",
           "config": {"n_fine": n_f, "coarse_ratio": cr, "isolation_box_fine_cells": L,
                      "b_coarse": cfg.b_coarse, "b_fine": cfg.b_fine, "b_pp": cfg.b_pp,
                      "assign": args.assign, "pairs_per_bin": args.pairs_per_bin},
           "max_abs_resid": float(np.abs(allres).max()),
           "rms_resid_all_bins": float(np.sqrt(np.mean([b["resid_std"] ** 2 + b["resid_mean"] ** 2
                                                        for b in bins]))),
           "bins": bins}
    print(json.dumps(out))


def pm3_experiment(args):
    """The adaptive PM3 level (section 2.2.3, PM3 paragraph) at the paper's
    softenings (beta = 3.5 on the fine level: b_f = 3.5 fine cells, the PP
    range of 125 neighbour cells; b_pp = 1/16): the two-level force against
    the three-level force with PM3 (H3 = 1/2 fine cell, b3 = 3.5 H3) on the
    tiles that the measured t_PM3 + t_PP model selects, on the same
    particles; the same with PM3 forced on the heaviest tiles, against the
    model's prediction of that change; and the difference of the two- and
    three-level forces (on the forced tiles when the model selects none)."""
    import torch
    import paper_2512_12629_amd as m
    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]
    x_np = synthetic.make(args.workload)
    N = x_np.shape[1]
    cfg = m.Config(n_fine=w["n_fine"], coarse_ratio=w["coarse_ratio"], b_fine=args.pair_b_fine,
                   b_pp=args.pair_b_pp)
    p3 = m.Cube2PM3(cfg, N)
    pos, cs, _ = p3.g.pack(torch.from_numpy(x_np).cuda())
    del x_np
    stream = torch.cuda.current_stream()

    def timed(fn, k):
        ts = []
        for _ in range(k + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts[1:]))

    t_two = timed(lambda: p3.g.force(pos, cs), args.steps)
    print(f"[bench] two-level force {t_two:.2f} ms", file=sys.stderr, flush=True)
    model = p3.calibrate(pos, cs, trial=args.pm3_trial)
    tiles = p3.select(pos, cs)
    print(f"[bench] model {model}; {len(tiles)} PM3 tiles", file=sys.stderr, flush=True)
    t_three = timed(lambda: p3.force(pos, cs, tiles), args.steps)
    # the model against a forced choice: PM3 on the heaviest tiles
    count, _, _ = p3.tile_stats(pos, cs)
    forced = torch.argsort(count, descending=True)[:args.pm3_trial].tolist()
    t_forced = timed(lambda: p3.force(pos, cs, forced), args.steps)
    pred = p3.predicted_change(pos, cs, forced) * 1e3
    pred_sel = p3.predicted_change(pos, cs, tiles) * 1e3 if tiles else 0.0
    if not tiles:
        tiles = forced        # report the difference of the forced choice
    a2 = p3.g.force(pos, cs).double()
    a3 = p3.force(pos, cs, tiles).double()
    num = torch.linalg.vector_norm(a3 - a2, dim=0)
    den = torch.linalg.vector_norm(a2, dim=0).clamp_min(1e-300)
    e = (num / den).cpu().numpy()
    out = {"experiment": "adaptive PM3 level (section 2.2.3) at the paper's softenings",
           "workload": args.workload, "particles": N, "b_fine": cfg.b_fine, "b_pp": cfg.b_pp,
           "h3": p3.h3, "beta3": p3.beta3, "pm3_tiles": len(tiles), "tiles": p3.nt ** 3,
           "two_level_force_ms": t_two, "three_level_force_ms": t_three,
           "speedup": t_two / t_three, "model": model,
           "selected_delta_ms_measured": t_three - t_two, "selected_delta_ms_predicted": pred_sel,
           "forced_heaviest_tiles": len(forced), "forced_force_ms": t_forced,
           "forced_delta_ms_measured": t_forced - t_two, "forced_delta_ms_predicted": pred,
           "rel_diff_median": float(np.median(e)), "rel_diff_p99": float(np.percentile(e, 99))}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clu512", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the force step (for profiler runs)")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the comparison with the FP64 plain form")
    ap.add_argument("--assign", choices=["cic", "tsc"], default="cic",
                    help="mass assignment of the PM levels (CIC, or TSC of eq. 5)")
    ap.add_argument("--pairwise", action="store_true",
                    help="run the pairwise force-accuracy experiment (isolated boundaries) "
                         "instead of the benchmark")
    ap.add_argument("--pairs-per-bin", type=int, default=16)
    ap.add_argument("--pair-b-fine", type=float, default=2.0,
                    help="fine softening (= PP cutoff) of the pairwise experiment; 3.5 is the "
                         "paper's beta = 3.5")
    ap.add_argument("--pair-b-pp", type=float, default=0.2,
                    help="PP softening of the pairwise experiment (the paper's Fig. 1: ~0.06)")
    ap.add_argument("--pm3", action="store_true",
                    help="run the adaptive PM3 experiment (softenings from --pair-b-fine / "
                         "--pair-b-pp, default 3.5 and 1/16 here) instead of the benchmark")
    ap.add_argument("--pm3-trial", type=int, default=512,
                    help="tiles of the PM3 cost-model calibration")
    ap.add_argument("--leapfrog-steps", type=int, default=4,
                    help="steps of the timed differentiable leapfrog (0: skip it)")
    ap.add_argument("--standalone", action="store_true",
                    help="time only the separate entry points (PM force, PP force and their "
                         "adjoints), one after the other, for profiler runs")
    ap.add_argument("--oracle-probe", nargs=2, metavar=("WORKLOAD", "SCALE"),
                    help=argparse.SUPPRESS)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timing, run a plain copy kernel (y = -x) of this many MiB "
                         "read + the same written, as the reference for HBM counter passes")
    args = ap.parse_args()
    if args.oracle_probe:
        n, n_f, times = _oracle_force_time(args.oracle_probe[0], int(args.oracle_probe[1]),
                                           min_total_s=0.0, max_reps=1)
        print(json.dumps({"particles": n, "n_fine": n_f, "seconds": times[0]}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design, not a build)", file=sys.stderr)
        sys.exit(2)

    if args.pairwise:
        pairwise_experiment(args)
        return
    if args.pm3:
        if args.pair_b_fine == 2.0 and args.pair_b_pp == 0.2:
            args.pair_b_fine, args.pair_b_pp = 3.5, 0.0625
        pm3_experiment(args)
        return

    import torch
    import paper_2512_12629_amd as m

    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]
    t_gen = time.perf_counter()
    x_np = synthetic.make(args.workload)
    N = x_np.shape[1]
    print(f"[bench] inputs {args.workload}: N={N} in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    cfg = m.Config(n_fine=w["n_fine"], coarse_ratio=w["coarse_ratio"],
                   flags=m.CUBE2_ASSIGN_TSC if args.assign == "tsc" else 0)
    t_init = time.perf_counter()
    c = m.Cube2(cfg, n_max=N)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t_init
    x = torch.from_numpy(x_np).cuda()
    del x_np
    pos, cs, _ = c.pack(x)
    vel = torch.zeros((3, N), dtype=torch.float32, device="cuda")
    acc = torch.empty((3, N), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def force():
        m.cube2_force(c.ctx, pos, cs, acc, c.work)

    def timed(fn, k):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(k)]
        torch.cuda.synchronize()
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]

    if args.standalone:
        abar = torch.randn((3, N), dtype=torch.float32, device="cuda")
        xbar = torch.empty_like(abar)
        st = {}
        for name, fn in (("pm_force", lambda: m.cube2_pm_force(c.ctx, pos, cs, acc, c.work)),
                         ("pp_force", lambda: m.cube2_pp_force(c.ctx, pos, cs, acc, c.work)),
                         ("pm_force_backward",
                          lambda: m.cube2_pm_force_backward(c.ctx, pos, cs, abar, xbar, c.work)),
                         ("pp_force_backward",
                          lambda: m.cube2_pp_force_backward(c.ctx, pos, cs, abar, xbar, c.work))):
            fn()
            st[name] = float(np.mean(timed(fn, args.steps)))
            print(f"[bench] standalone {name}: {st[name]:.3f} ms", file=sys.stderr, flush=True)
        print(json.dumps({"standalone_ms": st, "workload": args.workload, "steps": args.steps}))
        return

    for _ in range(args.warmup):
        force()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ts = timed(force, args.steps)
    wall = time.perf_counter() - t0
    print(f"[bench] force: {np.median(ts):.3f} ms median over {args.steps}", file=sys.stderr,
          flush=True)
    status = c.status()
    ms = float(np.median(ts))
    out = {
        "metric": "particles/sec per full PM+PP force step; backward/forward time ratio",
        "value": N / (ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "description": w["desc"], "particles": N,
                   "n_fine": w["n_fine"], "coarse_ratio": w["coarse_ratio"],
                   "assign": args.assign},
        "force_ms_mean": float(np.mean(ts)),
        "wall_s_timed": wall, "table_init_s": t_init, "status": status,
    }
    pairs = None
    if not args.no_extras and not args.no_fp64:
        out["fp64_form"] = fp64_comparison(m, cfg, c, pos, cs, N, ms, stream, timed)
    if not args.no_extras:
        # stages (each is one C-ABI entry point on the same stream)
        n_f, pitch_f = c.level_shape(0)
        rho = c.deposit(pos, cs, 0)
        t_pm = timed(lambda: m.cube2_pm_force(c.ctx, pos, cs, acc, c.work), args.steps)
        t_pp = timed(lambda: m.cube2_pp_force(c.ctx, pos, cs, acc, c.work), args.steps)
        t_pot = timed(lambda: m.cube2_potential(c.ctx, 0, rho, rho, c.work), args.steps)
        t_dep = timed(lambda: m.cube2_deposit(c.ctx, pos, cs, 0, rho, None, c.work), args.steps)
        stages = {"pm_force": float(np.mean(t_pm)), "pp_force": float(np.mean(t_pp)),
                  "potential_fine": float(np.mean(t_pot)), "deposit_fine": float(np.mean(t_dep))}
        # full step: force + kick-drift + IOS re-sort (ping-pong state)
        st = [pos, cs, vel]
        bufs = [torch.empty_like(pos), torch.empty_like(cs), torch.empty_like(vel)]
        perm = torch.empty(N, dtype=torch.int32, device="cuda")

        def full_step():
            m.cube2_force(c.ctx, st[0], st[1], acc, c.work)
            m.cube2_kick_drift(c.ctx, st[0], st[1], st[2], acc, 1e-3, 1e-3, bufs[0], bufs[1],
                               bufs[2], perm, c.work)
            for i in range(3):
                st[i], bufs[i] = bufs[i], st[i]

        t_full = timed(full_step, max(2, args.steps // 2))
        # IOS velocities (section 2.3): int16 codes against a bulk field, encode + decode
        nbv = m.cube2_vel_bulk_side(c.ctx)
        vq = torch.empty((3, N), dtype=torch.int16, device="cuda")
        vbulk = torch.empty((3, nbv, nbv, nbv), dtype=torch.float32, device="cuda")
        vsc = torch.empty(1, dtype=torch.float32, device="cuda")
        vdec = torch.empty_like(st[2])

        def vel_codec():
            m.cube2_vel_encode(c.ctx, st[0], st[1], st[2], vq, vbulk, vsc, c.work)
            m.cube2_vel_decode(c.ctx, st[0], st[1], vq, vbulk, vsc, vdec)

        t_vel = timed(vel_codec, max(2, args.steps // 2))
        # adjoint of the force (PM + PP), same positions
        abar = torch.randn((3, N), dtype=torch.float32, device="cuda")
        xbar = torch.empty_like(abar)

        def backward():
            m.cube2_force_backward(c.ctx, st[0], st[1], abar, xbar, c.work)

        stages["kick_drift_resort"] = float(np.mean(t_full)) - ms
        stages["vel_encode_decode"] = float(np.mean(t_vel))
        out["full_step_ms"] = float(np.mean(t_full))
        t_bwd = timed(backward, max(2, args.steps // 2))
        out["force_backward_ms"] = float(np.mean(t_bwd))
        out["force_backward_forward_ratio"] = float(np.mean(t_bwd)) / ms
        t_pmb = timed(lambda: m.cube2_pm_force_backward(c.ctx, st[0], st[1], abar, xbar, c.work),
                      max(2, args.steps // 2))
        t_ppb = timed(lambda: m.cube2_pp_force_backward(c.ctx, st[0], st[1], abar, xbar, c.work),
                      max(2, args.steps // 2))
        stages["pm_force_backward"] = float(np.mean(t_pmb))
        stages["pp_force_backward"] = float(np.mean(t_ppb))
        out["stages_ms"] = stages
        del abar, xbar, bufs, vq, vbulk, vdec, rho
        torch.cuda.empty_cache()
        if args.leapfrog_steps > 0:
            print("[bench] leapfrog forward + backward", file=sys.stderr, flush=True)
            out["leapfrog"] = leapfrog_timing(m, c, x, N, args.leapfrog_steps, 2, 2)
            out["backward_forward_ratio"] = out["leapfrog"]["backward_forward_ratio"]

        # roofline of the dominant kernel
        pairs = pair_counts().get(args.workload)
        t_pp_s = stages["pp_force"] * 1e-3
        fft_bytes = fft_bytes_reference(n_f, pitch_f)
        t_fft_s = stages["potential_fine"] * 1e-3
        if stages["pp_force"] >= stages["potential_fine"] and pairs:
            ach = pairs * PP_FLOPS_PER_PAIR / t_pp_s / 1e12
            out["roofline"] = {"kernel": "pp_kernel", "bound": "alu", "achieved": ach,
                               "peak": VALU_FP32_TFLOPS, "unit": "TFLOP/s",
                               "frac": ach / VALU_FP32_TFLOPS,
                               "traffic": measured_traffic(args.workload),
                               "pairs": pairs, "flops_per_pair": PP_FLOPS_PER_PAIR}
        else:
            ach = fft_bytes / t_fft_s / 1e9
            out["roofline"] = {"kernel": "fine potential (5 FFT sweeps)", "bound": "hbm",
                               "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS, "traffic": None}
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = src.numel() * 4
        del src, dst
    if not args.no_extras and pairs:
        meshes = [w["n_fine"]] + ([w["n_fine"] // w["coarse_ratio"]] if w["coarse_ratio"] else [])
        hbm = step_reference_bytes(N, meshes)
        t_hbm = hbm / (HBM_PEAK_GBS * 1e9)
        hbm_c = step_compulsory_bytes(N, meshes)
        t_hbm_c = hbm_c / (HBM_PEAK_GBS * 1e9)
        t_alu = pairs * PP_VALU_PER_PAIR / VALU_LANE_OPS
        t_flop = pairs * PP_FLOPS_PER_PAIR / (VALU_FP32_TFLOPS * 1e12)
        out["step_roofline"] = {
            "t_roof_ms": (t_hbm + t_flop) * 1e3, "t_hbm_ms": t_hbm * 1e3,
            "t_pp_flop_ms": t_flop * 1e3, "reference_bytes": hbm,
            "pp_flops_per_pair": PP_FLOPS_PER_PAIR, "frac": (t_hbm + t_flop) * 1e3 / ms,
            "instruction_model": {"t_pp_valu_ms": t_alu * 1e3, "pp_valu_per_pair": PP_VALU_PER_PAIR,
                                  "frac": (t_hbm + t_alu) * 1e3 / ms},
            "compulsory_model": {"bytes": hbm_c, "t_hbm_ms": t_hbm_c * 1e3,
                                 "frac": (t_hbm_c + t_flop) * 1e3 / ms}}
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(args.workload)
        except Exception as e:  # the baseline is reported, not required
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
