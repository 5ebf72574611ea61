"""Write the exact PP forces used by the GPU parity tests.

    python tests/golden/make_pp_exact.py

For each case the seeded positions are quantised by the oracle (IOS integer
positions, section 2.3) and the PP force of eq. (4d), with R of eq. (2),
b_pp = 0.2 and b_f = 2 fine cells, G m_p = 1, is evaluated in exact rational
arithmetic by ``oracle.exact`` (only the square root is rounded, at 2^-140).
Rows are particles in input order: a_x a_y a_z in fine cells per unit time.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic  # noqa: E402
from oracle import exact  # noqa: E402

CASES = {
    # name: (n_fine, generator)
    "zel_32_ragged": (32, lambda: synthetic.zeldovich(13, 0.25, 103)),
    "clustered_32": (32, lambda: synthetic.clustered(12, 0.25, 1, 256, 0.5 / 32, 105)),
}


def path(name):
    return os.path.join(HERE, f"pp_exact_{name}.txt")


def main():
    for name, (n_f, gen) in CASES.items():
        x = gen()
        q = oracle.quantize(x, n_f)
        acc = exact.pp_accel(q, n_f, 0.2, 2.0)
        header = (f"exact PP force (eq. 4d, R of eq. 2), case {name}: n_fine {n_f}, "
                  f"{x.shape[1]} particles, b_pp 0.2, b_f 2, G m_p 1; rows in input order; "
                  f"written by tests/golden/make_pp_exact.py")
        np.savetxt(path(name), acc.T, fmt="%.17e", header=header)
        print(name, x.shape[1], "particles")


if __name__ == "__main__":
    main()
