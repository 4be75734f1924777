"""Writes the oracle snapshot fixture.  Calls only the oracle and the seeded
input generator; the GPU library is never involved.

The paper prints no worked QP instance (no forces, objectives or energies), so
this snapshot is not a paper value: it freezes the pinned oracle's output on
the first 8 grasps of the 4-contact sphere workload (seed 16490) so that any
later change to the oracle's arithmetic shows up as a diff that must be
justified.  Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2412_16490_amd import workload as wl  # noqa: E402


def main():
    b = wl.config(0).subset(range(8))
    out = oracle.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench)
    doc = {
        "what": "oracle energies/objectives/forces, sphere m=4 s=6 seed 16490, grasps 0-7",
        "params": {"kappa": 20.0, "beta": 1.0, "eps": 1e-6, "fmax": 1.0, "gamma": 0.0},
        "energy": [float(v) for v in out["energy"]],
        "qobj": [float(v) for v in out["qobj"]],
        "forces": [[float(v) for v in row] for row in out["forces"]],
    }
    with open(os.path.join(HERE, "oracle_snapshot_sphere_m4_s6.json"), "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
