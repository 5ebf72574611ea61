"""Write leapfrog_fd_zel128.json: FP64 finite-difference derivatives of the
differentiable multi-step leapfrog loss at its stated size, from the oracle
only (plus the seeded input generators):

* workload: 128^3 particles on a Zel'dovich lattice (k^-2 field, rms 0.1 H_p),
  one PM level on a 256^3 mesh + PP (b_f = 2, b_pp = 0.2 fine cells), 10
  kick-drift steps with kick = drift = dt, dt = 0.1 sqrt(1 / max|a_0|) (fine
  cells, unit masses, G = 1) from the oracle's force on the initial positions,
  zero initial velocities;
* loss = sum over the fine mesh of (rho_final - rho_target)^2, rho the CIC
  density of unit masses, rho_target that of a second seeded Zel'dovich draw
  (seed + 1000);
* the oracle's continuous FP64 forward (no position quantisation);
* derivatives with respect to the initial positions in fine cells:
  - along 8 seeded unit directions (synthetic.unit_directions), central
    differences with steps 1e-3 and 5e-4 (both stored).  CIC weights have
    kinks at cell faces, and a step moves a few particles across one; the
    error this adds grows linearly with the step (about 0.5 % at a step of
    0.1), so the steps are small;
  - 256 single components (seeded particles whose initial position is more
    than 1e-3 fine cells from every cell face, seeded axes), central
    differences with step 1e-4.
Each difference is taken as sum (rho+ - rho-)(rho+ + rho- - 2 rho_target) /
(2h), the exact difference of the two losses without the cancellation of two
large sums.

    python tests/golden/make_leapfrog_fd.py --part K --parts P [--tmp DIR]
    python tests/golden/make_leapfrog_fd.py --merge --parts P [--tmp DIR]

Each part (run them in parallel processes) evaluates its share of the
perturbed forwards into DIR; --merge adds the oracle's own reverse-mode
derivatives (oracle.leapfrog_loss_grad on the same trajectory) and writes the
JSON beside this script.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "leapfrog_fd_zel128.json")
N_FINE, STEPS = 256, 10
DIR_SEED, COMP_SEED = 4711, 4712
N_DIRS, N_COMPS = 8, 256
H_DIRS, H_COMP = (1e-3, 5e-4), 1e-4


def setup(workers):
    x = synthetic.make("zel128_grad")
    seed = synthetic.SEED_BASE + list(synthetic.WORKLOADS).index("zel128_grad") + 1
    xt = synthetic.make("zel128_grad", seed=seed + 1000)
    x0f = x.astype(np.float64) * N_FINE
    rho_t = oracle.deposit(xt.astype(np.float64) * N_FINE, N_FINE, 1, quant=False)
    o = oracle.Oracle(oracle.Params(n_fine=N_FINE), quant=False, workers=workers)
    return o, x, x0f, rho_t


def final_density(o, x0f, dt):
    xs, _ = oracle.leapfrog_states(o, x0f, np.zeros_like(x0f), dt, dt, STEPS)
    return oracle.deposit(xs[-1], N_FINE, 1, quant=False)


def fd(o, x0f, dt, rho_t, pert, h):
    rp = final_density(o, x0f + h * pert, dt)
    rm = final_density(o, x0f - h * pert, dt)
    return float(np.sum((rp - rm) * (rp + rm - 2.0 * rho_t)) / (2.0 * h))


def jobs(x0f):
    """All perturbations: ('dir', k, h) and ('comp', particle, axis)."""
    out = [("dir", k, h) for k in range(N_DIRS) for h in H_DIRS]
    frac = x0f - np.floor(x0f)
    ok = np.all((frac > 1e-3) & (frac < 1 - 1e-3), axis=0)
    rng = np.random.default_rng(COMP_SEED)
    parts = rng.choice(np.nonzero(ok)[0], N_COMPS, replace=False)
    axes = rng.integers(0, 3, N_COMPS)
    out += [("comp", int(i), int(a)) for i, a in zip(parts, axes)]
    return out


def run_part(part, parts, tmp, workers):
    o, x, x0f, rho_t = setup(workers)
    a0 = o.accel(x0f)
    dt = float(0.1 * np.sqrt(1.0 / np.linalg.norm(a0, axis=0).max()))
    dirs = synthetic.unit_directions(x0f.shape, N_DIRS, DIR_SEED)
    todo = jobs(x0f)[part::parts]
    path = os.path.join(tmp, f"part{part}.json")
    done = json.load(open(path)) if os.path.exists(path) else {}
    for job in todo:
        key = "%s:%s:%s" % job
        if key in done:
            continue
        t0 = time.time()
        if job[0] == "dir":
            val = fd(o, x0f, dt, rho_t, dirs[job[1]], job[2])
        else:
            pert = np.zeros_like(x0f)
            pert[job[2], job[1]] = 1.0
            val = fd(o, x0f, dt, rho_t, pert, H_COMP)
        done[key] = val
        with open(path + ".tmp", "w") as f:
            json.dump(done, f)
        os.replace(path + ".tmp", path)
        print(f"[part {part}] {key} = {val:.9e} ({time.time() - t0:.1f} s)", flush=True)
    if part == 0:
        rho = final_density(o, x0f, dt)
        with open(os.path.join(tmp, "base.json"), "w") as f:
            json.dump({"dt": dt, "loss": float(np.sum((rho - rho_t) ** 2))}, f)


def merge(parts, tmp):
    base = json.load(open(os.path.join(tmp, "base.json")))
    vals = {}
    for k in range(parts):
        vals.update(json.load(open(os.path.join(tmp, f"part{k}.json"))))
    _, _, x0f, _ = setup(1)
    todo = jobs(x0f)
    missing = [j for j in todo if "%s:%s:%s" % j not in vals]
    if missing:
        raise SystemExit(f"{len(missing)} derivatives missing")
    # the oracle's own reverse mode on the same continuous trajectory, for a
    # three-way comparison (finite differences, oracle adjoint, GPU adjoint)
    o, _, x0f, rho_t = setup(8)
    _, gx, _ = oracle.leapfrog_loss_grad(o, x0f, np.zeros_like(x0f), base["dt"], base["dt"], STEPS,
                                         rho_t)
    dirs = synthetic.unit_directions(x0f.shape, N_DIRS, DIR_SEED)
    out = {
        "workload": "zel128_grad: 128^3 particles, Zel'dovich k^-2 rms 0.1 H_p, 256^3 mesh, "
                    "b_f = 2, b_pp = 0.2, one PM level + PP",
        "oracle_adjoint_dirs": [float(np.sum(gx * dirs[k])) for k in range(N_DIRS)],
        "oracle_adjoint_comps": [float(gx[j[2], j[1]]) for j in todo if j[0] == "comp"],
        "steps": STEPS, "dt": base["dt"], "loss": base["loss"], "n_fine": N_FINE,
        "dir_seed": DIR_SEED, "n_dirs": N_DIRS, "h_dirs": list(H_DIRS),
        "dirs": [[vals["dir:%d:%s" % (k, h)] for h in H_DIRS] for k in range(N_DIRS)],
        "h_comp": H_COMP,
        "comps": [[j[1], j[2], vals["%s:%s:%s" % j]] for j in todo if j[0] == "comp"],
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--part", type=int, default=0)
    ap.add_argument("--parts", type=int, default=1)
    ap.add_argument("--tmp", default="/tmp/leapfrog_fd")
    ap.add_argument("--workers", type=int, default=2)
    ap.add_argument("--merge", action="store_true")
    a = ap.parse_args()
    os.makedirs(a.tmp, exist_ok=True)
    if a.merge:
        merge(a.parts, a.tmp)
    else:
        run_part(a.part, a.parts, a.tmp, a.workers)
