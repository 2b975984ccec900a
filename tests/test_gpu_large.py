"""Parity of large subgraphs with the oracle, through the C ABI: the
multi-workgroup reduction to tridiagonal form (768 orbitals and more) and,
above 1,024 orbitals, the divide-and-conquer top merge with its work arrays
in device memory and the eight-wave back-transformation.

Bar: the FP64 bar of the other parity tests (eigenvalues 1e-12, mu 1e-12,
rho, rho1 and mu1 1e-10); split-FP32 responses 1e-6.

Cases:
- 400 waters, 30-atom spatial cores, paths of two at tau 0.02: 40 subgraphs
  of 870..1,213 orbitals, 21 of them above 1,024 (the whole first size
  class);
- the same system with 45-atom cores at tau 0.03: 27 subgraphs of
  703..1,072, three above 1,024, the one-workgroup reduction below 768;
- 2,048 hydrogen atoms on a jittered lattice, complete graph, cores of 128
  atoms: 16 subgraphs at both limits (2,048 orbitals, 128 core orbitals).
"""
import os
import sys

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

pytestmark = pytest.mark.gpu

KT = 0.01


def _say(msg):
    print(f"[gpu-large] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2212_01997_amd import gq
    return gq.Context(0)


def _case(name, O):
    if name == "max2048":
        # 16 x 16 x 8 lattice (1.5 A in x and y, 3 A in z), 24 A box
        s = I.h_lattice_system()
        core = (np.arange(s.n_atoms) // 128).astype(np.int32)
        return s, core, 0.0, O.COMPLETE
    s = I.water_system(400, 22.9, seed=401)
    if name == "mixed21":
        return s, I.spatial_cores(s, 30), 0.02, O.PATHS2
    return s, I.spatial_cores(s, 45), 0.03, O.PATHS2


def _run(ctx, O, name, K, precision=0):
    import torch
    from paper_2212_01997_amd.path import GraphPath
    s, core, tau, flags = _case(name, O)
    g = O.graph_build(s, core, tau, flags=flags)
    sizes = g.sizes()
    _say(f"{name}: {g.n_sub} subgraphs of {sizes.min()}..{sizes.max()}, "
         f"{int((sizes > 1024).sum())} above 1024; oracle")
    h1 = I.h1_diagonal(s, K, seed=4001)
    r = O.solve_pool(s, g, KT, h1, workers=min(16, os.cpu_count() or 1))
    _say(f"{name}: gpu, precision {precision}")
    p = GraphPath(ctx, s, core, tau, None, flags, max_k=K)
    mu = p.ground_state(KT)
    mu1 = p.respond(torch.as_tensor(h1, device="cuda"), precision=precision)
    p.sync()
    eps, _ = p.eigs.export()
    ex = p.graph.export()
    for key in ("sub_orb_ptr", "sub_orbs", "n_core_orbs", "rho_row_ptr", "rho_col"):
        assert np.array_equal(ex[key], getattr(g, key)), key
    err = {"mu": abs(mu - r.mu), "eps": float(np.abs(eps - r.eps).max()),
           "rho": float(np.abs(p.rho.cpu().numpy() - r.rho).max()),
           "rho1": float(np.abs(p.rho1_view(K).cpu().numpy() - r.rho1).max()),
           "mu1": float(np.abs(mu1 - r.mu1).max())}
    _say(f"{name}: " + " ".join(f"{k} {v:.1e}" for k, v in err.items()))
    return sizes, err


@pytest.mark.parametrize("name", ["mixed21", "mixed3"])
def test_large_subgraphs(ctx, oracle_lib, name):
    sizes, err = _run(ctx, oracle_lib, name, 2)
    assert (sizes > 1024).sum() == (21 if name == "mixed21" else 3)
    assert (sizes <= 1024).any()
    assert err["mu"] <= 1e-12 and err["eps"] <= 1e-12
    assert max(err["rho"], err["rho1"], err["mu1"]) <= 1e-10


def test_size_limits(ctx, oracle_lib):
    """16 subgraphs of 2,048 orbitals with cores of 128 orbitals."""
    sizes, err = _run(ctx, oracle_lib, "max2048", 1)
    assert (sizes == 2048).all()
    assert err["mu"] <= 1e-12 and err["eps"] <= 1e-12
    assert max(err["rho"], err["rho1"], err["mu1"]) <= 1e-10


def test_large_split32(ctx, oracle_lib):
    from paper_2212_01997_amd import gq
    _, err = _run(ctx, oracle_lib, "mixed3", 3, precision=gq.PREC_SPLIT32)
    assert err["mu"] <= 1e-12 and err["rho"] <= 1e-10
    assert max(err["rho1"], err["mu1"]) <= 1e-6
