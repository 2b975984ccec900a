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
  atoms: 16 subgraphs at both limits (2,048 orbitals, 128 core orbitals);
- 768 hydrogen atoms likewise: six subgraphs of exactly 768 orbitals;
- 200 isolated waters, complete graph: ten block-diagonal subgraphs of 1,200
  orbitals, where most columns are already reduced (identity reflectors).
Beside the eigensolve path: the zero-temperature density by purification
(batched products) and the non-orthogonal basis on these sizes.
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
    if name == "lattice768":
        # 16 x 16 x 3 lattice: six subgraphs of exactly 768 orbitals, the
        # smallest size the multi-workgroup reduction takes
        s = I.h_lattice_system(shape=(16, 16, 3), spacing=(1.5, 1.5, 3.0), box=24.0, seed=768)
        core = (np.arange(s.n_atoms) // 128).astype(np.int32)
        return s, core, 0.0, O.COMPLETE
    if name == "isolated1200":
        # 200 waters 7 A apart: every subgraph (the whole system) is block
        # diagonal, so most reflectors of the reduction are the identity
        s = I.isolated_molecules_system(200, 7.0, seed=1200)
        core = (np.arange(s.n_atoms) // 60).astype(np.int32)
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


@pytest.mark.parametrize("name", ["lattice768", "isolated1200"])
def test_large_edge_cases(ctx, oracle_lib, name):
    sizes, err = _run(ctx, oracle_lib, name, 1)
    assert (sizes == (768 if name == "lattice768" else 1200)).all()
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


@pytest.mark.parametrize("name", ["mixed3", "mixed21"])
def test_large_capture_replay(oracle_lib, name):
    """A step on subgraphs of 703..1,072 orbitals (both size classes), or of
    870..1,213 (all on the multi-workgroup path, in two halves on two
    streams), recorded once and replayed three times, with eager work in
    between: every replay gives the eager bits."""
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    s, core, tau, flags = _case(name, oracle_lib)
    side = torch.cuda.Stream()
    cx = gq.Context(0, stream=side)
    p = GraphPath(cx, s, core, tau, None, flags, max_k=2)
    h1 = torch.as_tensor(I.h1_diagonal(s, 2, seed=4003), device="cuda")
    h1b = torch.as_tensor(I.h1_diagonal(s, 2, seed=4004), device="cuda")
    torch.cuda.synchronize()

    def step(h):
        p.ground_state(KT, want_mu=False)
        p.respond(h, want_mu1=False)

    p.ground_state(KT)  # mu on the host once; the captured steps reuse it
    step(h1)
    side.synchronize()
    ref = (p.rho.clone(), p.rho1_view(2).clone())
    cx.capture_begin()
    step(h1)
    x = cx.capture_end()
    _say(f"{name}: large step captured")
    for rep in range(3):
        p.rho.zero_()
        p.rho1.zero_()
        torch.cuda.synchronize()
        x.launch()
        side.synchronize()
        assert torch.equal(p.rho, ref[0]), rep
        assert torch.equal(p.rho1_view(2), ref[1]), rep
        step(h1b)
        side.synchronize()
        assert not torch.equal(p.rho1_view(2), ref[1])
    del x


def _gershgorin(O, s, g, mu):
    H = O.Csr(s.h_row_ptr, s.h_col, s.h_val)
    R = 0.0
    for i in range(g.n_sub):
        h = O.gather(H, g.orbs(i))
        R = max(R, float(np.abs(h - mu * np.eye(h.shape[0])).sum(axis=1).max()))
    return R


@pytest.mark.parametrize("name", ["lattice768", "isolated1200"])
def test_large_purify(ctx, oracle_lib, name):
    """The zero-temperature density by purification (batched products over
    the lower tiles of subgraphs of 768 and 1,200 orbitals) against the step
    density of the oracle, within the bar of the purification tests
    (64 n u R / gap: R the largest Gershgorin radius of h_i - mu I, gap the
    distance of the nearest subgraph eigenvalue to mu); then the eigensolve
    path again, unchanged."""
    from oracle import foe as F
    from paper_2212_01997_amd.path import GraphPath
    O = oracle_lib
    s, core, tau, flags = _case(name, O)
    g = O.graph_build(s, core, tau, flags=flags)
    r = O.solve_pool(s, g, KT, workers=min(16, os.cpu_count() or 1))
    mu = F.mid_gap(r.eps, r.mu)
    ref, gap = F.purified_density(s, g, mu)
    tol = 64 * int(g.sizes().max()) * 2.0 ** -53 * _gershgorin(O, s, g, mu) / gap
    p = GraphPath(ctx, s, core, tau, None, flags)
    it = p.purified_state(mu, max_iter=80)
    err = float(np.abs(p.rho.cpu().numpy() - ref).max())
    _say(f"{name} purify: gap {gap:.2e} iterations {it} |drho| {err:.1e} (bar {tol:.1e})")
    assert err <= tol and it < 80
    assert abs(p.ground_state(KT) - r.mu) <= 1e-12
    assert np.abs(p.rho.cpu().numpy() - r.rho).max() <= 1e-10


def test_large_overlap(ctx, oracle_lib):
    """The non-orthogonal basis on six subgraphs of 768 orbitals (Lowdin
    factors by batched products, two eigensolves on the multi-workgroup path)
    against the overlap oracle: mu 1e-12, atomic-orbital rho, rho1 and mu1
    1e-10."""
    import torch
    from oracle import overlap as V
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    O = oracle_lib
    s, core, tau, flags = _case("lattice768", O)
    g = O.graph_build(s, core, tau, flags=flags)
    S = I.overlap_matrix(s)
    h1 = I.h1_diagonal(s, 2, seed=4005)
    ref = V.solve(s, S, g, KT, h1)
    p = GraphPath(ctx, s, core, tau, None, flags, max_k=2, S=S)
    mu = p.ground_state(KT)
    mu1 = p.respond(torch.as_tensor(h1, device="cuda"))
    p.sync()
    err = {"mu": abs(mu - ref.mu), "rho": float(np.abs(p.rho.cpu().numpy() - ref.rho_ao).max()),
           "rho1": float(np.abs(p.rho1_view(2).cpu().numpy() - ref.rho1_ao).max()),
           "mu1": float(np.abs(mu1 - ref.mu1).max())}
    _say("lattice768 overlap: " + " ".join(f"{k} {v:.1e}" for k, v in err.items()))
    assert err["mu"] <= 1e-12
    assert max(err["rho"], err["rho1"], err["mu1"]) <= 1e-10


def test_large_identity_overlap(ctx, oracle_lib):
    """S = I on subgraphs of 1,200 orbitals: the non-orthogonal path equals
    the orthogonal one."""
    import torch
    from paper_2212_01997_amd.path import GraphPath
    s, core, tau, flags = _case("isolated1200", oracle_lib)
    n = s.n_orb
    eye = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    h1 = torch.as_tensor(I.h1_diagonal(s, 1, seed=4006), device="cuda")
    a = GraphPath(ctx, s, core, tau, None, flags, max_k=1, S=eye)
    b = GraphPath(ctx, s, core, tau, None, flags, max_k=1)
    mus = (a.ground_state(KT), b.ground_state(KT))
    mu1s = (a.respond(h1), b.respond(h1))
    a.sync()
    b.sync()
    assert abs(mus[0] - mus[1]) <= 1e-13
    assert (a.rho - b.rho).abs().max().item() <= 1e-12
    assert (a.rho1_view(1) - b.rho1_view(1)).abs().max().item() <= 1e-12
    assert np.abs(mu1s[0] - mu1s[1]).max() <= 1e-12
