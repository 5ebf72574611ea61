"""Write pair_counts.json: the exact number of ordered particle pairs with
0 < r < b_f (the PP work) of each seeded benchmark workload, counted by the
oracle's cell list on the quantised positions.  Calls only oracle/ and the
input generators.

    python tests/golden/make_pair_counts.py [workload ...]
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pair_counts.json")
N_FINE = {"clu512": 1024, "clu256": 512, "zel128": 256, "uniform32": 64}


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        x = synthetic.make(name)
        q = oracle.quantize(x, N_FINE[name])
        del x
        xf = oracle.q_to_fine(q)
        del q
        o = oracle.Oracle(oracle.Params(n_fine=N_FINE[name]))
        data[name] = o.pp_pair_count(xf)
        print(name, data[name], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["uniform32", "zel128", "clu256", "clu512"])
