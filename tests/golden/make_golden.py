"""Write the stored expected values of the large parity tests.

Calls only the CPU oracle (single-threaded FP64) on the seeded synthetic
workloads and records, per workload, the three list sizes and the twelve
energy terms with the sum of |interaction energy| of each term (the
tolerance scale).  Run from the repository root:

    python tests/golden/make_golden.py

It takes a few minutes and ~20 GB of memory for the 1,044,000-atom box.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import reaxff_synth as rs  # noqa: E402
from oracle import TERM_NAMES, Oracle  # noqa: E402


def record(name, params):
    s = rs.workload(name)
    t0 = time.time()
    o = Oracle(s, params)
    far, bonds, hb = (len(x) for x in o.lists())
    e, a = o.energy_abs()
    out = {"atoms": s.n, "far_pairs": far, "bond_entries": bonds, "hb_entries": hb,
           "energies": dict(zip(TERM_NAMES, map(float, e))),
           "abs_sums": dict(zip(TERM_NAMES, map(float, a))),
           "oracle_seconds": round(time.time() - t0, 1)}
    print(name, out, flush=True)
    return out


def main():
    params = rs.draw_params(0)
    data = {"params_seed": 0, "generator": "reaxff_synth.workload", "workloads": {}}
    for name in ("petn_1856", "petn_32480", "petn_1044000"):
        data["workloads"][name] = record(name, params)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_energies.json")
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print("wrote", path)


if __name__ == "__main__":
    main()
