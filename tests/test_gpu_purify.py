"""Parity of the zero-temperature density by purification on the GPU
(gq_purify: McWeeny iteration on every subgraph, Sec. II.D, Eqs. (Step),
(Recur), (dCollect)) with the step-density oracle (oracle/foe.py), through
the C ABI.

mu is placed in the middle of the gap between the subgraph eigenvalues (all
subgraphs together) around the finite-temperature mu of each system.  Bar:
the collected rows within 64 n u R / g of the oracle, with u the unit
roundoff, n the largest subgraph, R the largest Gershgorin radius of
h_i - mu I and g the distance of the nearest eigenvalue to mu: a rounding
error E made while the eigenvalues of X sit near 1/2 turns the occupied
subspace by about |E| / (g / R), and the early iterations, where g / R is
smallest, dominate.
"""
import sys

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

pytestmark = pytest.mark.gpu

KT = 0.01
U = 2.0 ** -53


def _say(msg):
    print(f"[gpu-purify] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2212_01997_amd import gq
    return gq.Context(0)


@pytest.fixture(scope="module")
def F():
    from oracle import foe
    return foe


def _case(name, O):
    if name == "water32":
        s = I.water32_system()
        core = I.spatial_cores(s, 3)
    elif name == "water60":
        s = I.water_system(60, 12.2, seed=61)
        core = I.spatial_cores(s, 8)
    else:
        s = I.chain_water_system(900, 180, seed=3001)
        core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT, pool=name == "chain900")
    g = O.graph_build(s, core, 0.07, rho_prev=prev, flags=O.PATHS2)
    r = O.solve(s, g, KT) if name != "chain900" else O.solve_pool(s, g, KT)
    return s, core, prev, g, r


def _radius(O, s, g, mu):
    H = O.Csr(s.h_row_ptr, s.h_col, s.h_val)
    R = 0.0
    for i in range(g.n_sub):
        h = O.gather(H, g.orbs(i))
        R = max(R, float(np.abs(h - mu * np.eye(h.shape[0])).sum(axis=1).max()))
    return R


@pytest.mark.parametrize("name", ["water32", "water60", "chain900"])
def test_purify_parity(ctx, oracle_lib, F, name):
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    O = oracle_lib
    s, core, prev, g, r = _case(name, O)
    mu = F.mid_gap(r.eps, r.mu)
    ref, gap = F.purified_density(s, g, mu)
    R = _radius(O, s, g, mu)
    tol = 64 * int(g.sizes().max()) * U * R / gap
    p = GraphPath(ctx, s, core, 0.07, prev, gq.PATHS2)
    it = p.purified_state(mu, max_iter=80)
    got = p.rho.cpu().numpy()
    err = float(np.abs(got - ref).max())
    _say(f"{name}: mu {mu:.6f} gap {gap:.2e} R {R:.2f} iterations {it} "
         f"|drho| {err:.2e} (bar {tol:.2e})")
    assert err <= tol
    assert it < 80
    # the eigenbasis was overwritten: the eigensolve path runs again unchanged
    mu2 = p.ground_state(KT)
    assert abs(mu2 - r.mu) <= 1e-12
    assert np.abs(p.rho.cpu().numpy() - r.rho).max() <= 1e-10


def test_purify_eigenvalue_at_mu(ctx, oracle_lib):
    """mu equal to a subgraph eigenvalue: that state stays at 1/2, the
    iteration cannot converge, GQ_ENOCONV."""
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    O = oracle_lib
    s, core, prev, g, r = _case("water32", O)
    p = GraphPath(ctx, s, core, 0.07, prev, gq.PATHS2)
    mu = float(r.eps[np.argmin(np.abs(r.eps - r.mu))])
    with pytest.raises(gq.GQError, match="not converged"):
        p.purified_state(mu, max_iter=40)


def test_purify_errors(ctx):
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    s = I.water32_system()
    core = I.single_atom_cores(s)
    p = GraphPath(ctx, s, core, 1e-3)
    rho = torch.empty(p.nnz, dtype=torch.float64, device="cuda")
    for kw, msg in ((dict(max_iter=0), "max_iter"), (dict(tol=0.0), "tol"),
                    (dict(tol=float("nan")), "tol")):
        with pytest.raises(gq.GQError, match=msg):
            p.eigs.purify(p.H, -0.2, rho, **kw)
    with pytest.raises(gq.GQError, match="mu"):
        p.eigs.purify(p.H, float("inf"), rho)
    other = I.water_system(6, 8.0, seed=71)
    H2 = gq.DeviceCsr(other.h_row_ptr, other.h_col, other.h_val)
    with pytest.raises(gq.GQError, match="rows"):
        p.eigs.purify(H2, -0.2, rho)


def test_chain30000_sampled(oracle_lib, F):
    """The 30,000-atom chain-in-water system (3,750 subgraphs of 148..638
    orbitals) at the oracle's kT = 0.01 mu (tests/golden/chain30000_oracle.json):
    the graph checked bit-exact against the oracle's digests, the purified
    core rows of eight sampled subgraphs (the smallest, the largest and six
    seeded picks) against the oracle's step rows, each within its own bar."""
    import hashlib
    import json
    import os
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath, bootstrap_prev
    O = oracle_lib
    with open(os.path.join(os.path.dirname(__file__), "golden", "chain30000_oracle.json")) as f:
        gold = json.load(f)
    mu = gold["kT"][repr(KT)]["mu"]
    s = I.chain30000_system()
    core = I.spatial_cores(s, 8)
    ctx = gq.Context(0)
    prev = bootstrap_prev(ctx, s, core, KT)
    graph = gq.Graph.for_system(s, core, 0.07, prev, gq.PATHS2)
    ex = graph.export()
    for name, dig in gold["graph"].items():
        got = hashlib.sha256(np.ascontiguousarray(ex[name], np.int32).tobytes()).hexdigest()[:16]
        assert got == dig, name
    p = GraphPath(ctx, s, core, 0.07, graph=graph)
    it = p.purified_state(mu, max_iter=100)
    blocks = p.rho_blocks.cpu().numpy()
    off = graph.block_offsets()
    sop, orbs, nc = ex["sub_orb_ptr"], ex["sub_orbs"], ex["n_core_orbs"]
    sizes = np.diff(sop)
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes))]
    picks += [int(x) for x in np.random.default_rng(3004).choice(len(sizes), 6, replace=False)]
    H = O.Csr(s.h_row_ptr, s.h_col, s.h_val)
    worst = 0.0
    for i in picks:
        h = O.gather(H, orbs[sop[i]:sop[i + 1]])
        n, c = h.shape[0], int(nc[i])
        w, _ = O.eigh(h)
        gap = float(np.abs(w - mu).min())
        R = float(np.abs(h - mu * np.eye(n)).sum(axis=1).max())
        ref = F.step_rows(h, c, mu)
        got = blocks[off[i]:off[i] + c * n].reshape(c, n)
        err = float(np.abs(got - ref).max())
        bar = 64 * n * U * R / gap
        worst = max(worst, err / bar)
        assert err <= bar, (i, n, gap, err, bar)
    _say(f"chain30000: {it} iterations, worst error / bar {worst:.2e} over {len(picks)} subgraphs")
