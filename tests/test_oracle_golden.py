"""The oracle still reproduces its frozen snapshot (see tests/golden/README.md)."""
import json
import os

import numpy as np

from paper_2412_16490_amd import workload as wl

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_snapshot(orc):
    with open(os.path.join(HERE, "golden", "oracle_snapshot_sphere_m4_s6.json")) as fh:
        doc = json.load(fh)
    b = wl.config(0).subset(range(8))
    out = orc.solve_batch(b.counts, b.woff, b.points, b.normals, b.mu, b.wrench)
    np.testing.assert_allclose(out["energy"], doc["energy"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["qobj"], doc["qobj"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["forces"], np.array(doc["forces"]), atol=1e-12)
