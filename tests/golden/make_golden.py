"""Writes the oracle regression fixtures in this folder.

Calls only the oracle and the seeded input generator.  The paper prints no
worked numerical example for this path, so these files hold the oracle's own
values for the 32-water system (its pins live in tests/test_oracle_pins.py);
they catch unintended changes to the oracle's arithmetic.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2212_01997_amd import inputs as I  # noqa: E402

KT = 0.01


def case(tau, flags):
    s = I.water32_system()
    core = I.single_atom_cores(s)
    prev = O.bootstrap_prev(s, core, KT)
    g = O.graph_build(s, core, tau, rho_prev=prev, flags=flags)
    h1 = I.h1_diagonal(s, 2, seed=1002)
    r = O.solve(s, g, KT, h1)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(g.nnz, size=64, replace=False))
    return {
        "system": "32 waters, 10 A box, seed 1001; H1 seed 1002; kT 0.01 Ha; one-atom cores",
        "tau": tau, "flags": flags,
        "sizes": [int(x) for x in g.sizes()],
        "nnz": g.nnz,
        "mu": r.mu, "mu1": [float(x) for x in r.mu1],
        "idx": [int(i) for i in idx],
        "rho": [float(r.rho[i]) for i in idx],
        "rho1": [[float(r.rho1[q][i]) for i in idx] for q in range(2)],
    }


if __name__ == "__main__":
    out = {"tau1e-5": case(1e-5, 0), "tau7e-2_paths2": case(7e-2, O.PATHS2),
           "complete": case(1e-5, O.COMPLETE)}
    with open(os.path.join(HERE, "water32_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote water32_oracle.json")
