"""The oracle's reverse mode through the differentiable leapfrog at its
stated size (128^3 particles, 256^3 mesh + PP, 10 steps) against FP64
central finite differences of its continuous forward, both stored in
tests/golden/leapfrog_fd_zel128.json by make_leapfrog_fd.py (from the oracle
only): the reverse mode (adjoints of the deposit, of the PM and PP forces and
of the kick-drift, derived in the oracle's docstrings) is pinned by
differences of the forward.

* 256 single components: relative error (to max(|fd|, 1e-3 rms)) median
  <= 1e-5 and p99 <= 2e-3 (measured 3.7e-7 and 8.8e-4: a few components
  whose particle passes a CIC node within the step);
* 8 seeded directions: within 1e-3 of the rms directional derivative plus
  twice the spread between the differences at steps 1e-3 and 5e-4 (the
  cell-face crossings of a step that moves every particle)."""
import json
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "leapfrog_fd_zel128.json")


def test_oracle_reverse_mode_against_finite_differences():
    g = json.load(open(GOLD))
    fd = np.array([c[2] for c in g["comps"]])
    ad = np.array(g["oracle_adjoint_comps"])
    e = np.abs(ad - fd) / np.maximum(np.abs(fd), 1e-3 * np.sqrt(np.mean(fd ** 2)))
    assert np.median(e) <= 1e-5 and np.percentile(e, 99) <= 2e-3, (np.median(e), e.max())
    d = np.array(g["dirs"])
    rms = np.sqrt(np.mean(d[:, 1] ** 2))
    spread = np.abs(d[:, 0] - d[:, 1])
    err = np.abs(np.array(g["oracle_adjoint_dirs"]) - d[:, 1])
    assert np.all(err <= 1e-3 * rms + 2 * spread), (err, 1e-3 * rms + 2 * spread)
