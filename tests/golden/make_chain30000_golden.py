"""Writes chain30000_oracle.json: oracle values for the 30,000-atom chain-in-water
system (6,000-atom C/N/O/S chain in water at 0.1 atoms per cubic angstrom,
72,000 orbitals, 8-atom Morton cores, graph = paths of two of the thresholded
bootstrap density and Hamiltonian at tau = 0.07), six diagonal perturbations,
at kT = 0.003, 0.01 and 0.03 Ha.

Calls only the oracle (its process pool) and the seeded input generator.  The
whole-system arrays are too large to store, so the file keeps mu, mu1 and the
values at 4,096 seeded positions of rho and of each rho1, plus digests of the
graph the values belong to.

    python tests/golden/make_chain30000_golden.py      (about 15 minutes on 8 cores)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2212_01997_amd import inputs as I  # noqa: E402

KTS = (0.003, 0.01, 0.03)
K = 6
TAU = 0.07
N_SAMPLE = 4096


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def graph_digests(sub_orb_ptr, sub_orbs, n_core_orbs, rho_row_ptr, rho_col):
    return {"sub_orb_ptr": digest(np.asarray(sub_orb_ptr, np.int32)),
            "sub_orbs": digest(np.asarray(sub_orbs, np.int32)),
            "n_core_orbs": digest(np.asarray(n_core_orbs, np.int32)),
            "rho_row_ptr": digest(np.asarray(rho_row_ptr, np.int32)),
            "rho_col": digest(np.asarray(rho_col, np.int32))}


def main():
    t0 = time.time()
    s = I.chain30000_system()
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, 0.01, pool=True)
    print(f"bootstrap done {time.time() - t0:.0f} s", flush=True)
    g = O.graph_build(s, core, TAU, rho_prev=prev, flags=O.PATHS2)
    h1 = I.h1_diagonal(s, K, seed=3002)
    idx = np.sort(np.random.default_rng(3).choice(g.nnz, size=N_SAMPLE, replace=False))
    out = {"system": "30,000 atoms (6,000-atom chain in water), seed 3001; H1 seed 3002, K = 6; "
                     "8-atom Morton cores; bootstrap density at kT 0.01; paths of two, tau 0.07",
           "n_sub": int(g.n_sub), "nnz": int(g.nnz),
           "sizes_min": int(g.sizes().min()), "sizes_max": int(g.sizes().max()),
           "prev_digest": digest(prev[2]),
           "graph": graph_digests(g.sub_orb_ptr, g.sub_orbs, g.n_core_orbs, g.rho_row_ptr, g.rho_col),
           "idx": [int(i) for i in idx], "kT": {}}
    for kT in KTS:
        r = O.solve_pool(s, g, kT, h1)
        out["kT"][repr(kT)] = {"mu": r.mu, "mu1": [float(x) for x in r.mu1],
                               "rho": [float(r.rho[i]) for i in idx],
                               "rho1": [[float(r.rho1[q][i]) for i in idx] for q in range(K)]}
        print(f"kT {kT} done {time.time() - t0:.0f} s: mu {r.mu:.12f}", flush=True)
    with open(os.path.join(HERE, "chain30000_oracle.json"), "w") as f:
        json.dump(out, f)
    print("wrote chain30000_oracle.json", flush=True)


if __name__ == "__main__":
    main()
