"""Regression of the oracle against its stored values (tests/golden).

The paper prints no worked numerical example for this path; the fixtures were
written by tests/golden/make_golden.py, which calls only the oracle.  They
guard against unintended changes to the oracle's arithmetic; its correctness
is pinned in test_oracle_pins.py.
"""
import json
import os

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
KT = 0.01


@pytest.mark.parametrize("key", ["tau1e-5", "tau7e-2_paths2", "complete"])
def test_water32_golden(oracle_lib, key):
    O = oracle_lib
    with open(os.path.join(HERE, "golden", "water32_oracle.json")) as f:
        ref = json.load(f)[key]
    s = I.water32_system()
    core = I.single_atom_cores(s)
    prev = O.bootstrap_prev(s, core, KT)
    g = O.graph_build(s, core, ref["tau"], rho_prev=prev, flags=ref["flags"])
    assert [int(x) for x in g.sizes()] == ref["sizes"]
    assert g.nnz == ref["nnz"]
    r = O.solve(s, g, KT, I.h1_diagonal(s, 2, seed=1002))
    assert abs(r.mu - ref["mu"]) <= 1e-13
    assert np.abs(r.mu1 - np.array(ref["mu1"])).max() <= 1e-13
    idx = np.array(ref["idx"])
    assert np.abs(r.rho[idx] - np.array(ref["rho"])).max() <= 1e-13
    assert np.abs(r.rho1[:, idx] - np.array(ref["rho1"])).max() <= 1e-13
