"""Parity of the HIP path (through the C ABI) with the oracle, element by element.

Bar (FP64 path): rho, rho1 and mu1 within 1e-10 max-abs, mu within 1e-12,
eigenvalues within 1e-12; graph maps bit-exact.  The oracle's inputs come from
the seeded generator only (its bootstrap density included); the GPU gets the
same inputs.  Large oracle runs use the oracle's process pool (spawned workers,
identical results to its serial path).
"""
import os
import sys

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

pytestmark = pytest.mark.gpu

KT = 0.01
TOL = 1e-10
TOL_MU = 1e-12


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2212_01997_amd import gq
    return gq.Context(0)


def run_gpu(ctx, system, core, tau, prev, flags, kT, h1, precision=0):
    import torch
    from paper_2212_01997_amd.path import GraphPath
    K = h1.shape[0]
    p = GraphPath(ctx, system, core, tau, prev, flags, max_k=K)
    mu = p.ground_state(kT)
    mu1 = p.respond(torch.as_tensor(h1, device="cuda"), precision=precision)
    torch.cuda.synchronize()
    eps, w = p.eigs.export()
    return {"mu": mu, "mu1": mu1, "rho": p.rho.cpu().numpy(),
            "rho1": p.rho1_view(K).cpu().numpy(), "eps": eps, "w": w,
            "graph": p.graph.export(), "path": p}


def run_oracle(O, system, core, tau, prev, flags, kT, h1, pool=False):
    g = O.graph_build(system, core, tau, rho_prev=prev, flags=flags)
    if pool:
        r = O.solve_pool(system, g, kT, h1, workers=min(16, os.cpu_count() or 1))
    else:
        r = O.solve(system, g, kT, h1)
    return g, r


def compare(gpu, g, r, tol=TOL, tol_mu=TOL_MU, tol1=None):
    """tol bounds rho (and rho1, mu1 unless tol1 is given for the response)."""
    tol1 = tol if tol1 is None else tol1
    ex = gpu["graph"]
    for name in ("sub_orb_ptr", "sub_orbs", "n_core_orbs", "rho_row_ptr", "rho_col"):
        assert np.array_equal(ex[name], getattr(g, name)), name
    assert abs(gpu["mu"] - r.mu) <= tol_mu, (gpu["mu"], r.mu)
    assert np.abs(gpu["eps"] - r.eps).max() <= 1e-12
    assert np.abs(gpu["rho"] - r.rho).max() <= tol
    err1 = (np.abs(gpu["mu1"] - r.mu1).max(), np.abs(gpu["rho1"] - r.rho1).max())
    assert err1[0] <= tol1 and err1[1] <= tol1, err1
    return err1


def case_water32(O, tau, flags, kT=KT, K=2):
    s = I.water32_system()
    core = I.single_atom_cores(s)
    prev = O.bootstrap_prev(s, core, KT)
    return s, core, prev, I.h1_diagonal(s, K, seed=1002)


@pytest.mark.parametrize("tau,flags", [(1e-5, 0), (0.07, 1), (1e-5, 2)],
                         ids=["tau1e-5", "paths2_tau0.07", "complete"])
def test_water32(ctx, oracle_lib, tau, flags):
    O = oracle_lib
    s, core, prev, h1 = case_water32(O, tau, flags)
    _say(f"water32 tau={tau} flags={flags}")
    g, r = run_oracle(O, s, core, tau, prev, flags, KT, h1)
    gpu = run_gpu(ctx, s, core, tau, prev, flags, KT, h1)
    compare(gpu, g, r)


@pytest.mark.parametrize("kT", [0.003, 0.03])
def test_water32_temperatures(ctx, oracle_lib, kT):
    O = oracle_lib
    s, core, prev, h1 = case_water32(O, 0.07, 1)
    _say(f"water32 kT={kT}")
    g, r = run_oracle(O, s, core, 0.07, prev, 1, kT, h1)
    gpu = run_gpu(ctx, s, core, 0.07, prev, 1, kT, h1)
    compare(gpu, g, r)


def test_water60_spatial_cores(ctx, oracle_lib):
    """8-atom spatial cores, paths of two: several 64-wide tiles and ragged tails."""
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    h1 = I.h1_diagonal(s, 3, seed=62)
    g, r = run_oracle(O, s, core, 0.07, prev, 1, KT, h1, pool=True)
    _say(f"water60 sizes {g.sizes().min()}..{g.sizes().max()}")
    gpu = run_gpu(ctx, s, core, 0.07, prev, 1, KT, h1)
    compare(gpu, g, r)


def test_chain_in_water(ctx, oracle_lib):
    O = oracle_lib
    s = I.chain_water_system(900, 180, seed=3001)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT, pool=True)
    h1 = I.h1_diagonal(s, 2, seed=3002)
    g, r = run_oracle(O, s, core, 0.07, prev, 1, KT, h1, pool=True)
    _say(f"chain900 sizes {g.sizes().min()}..{g.sizes().max()}")
    gpu = run_gpu(ctx, s, core, 0.07, prev, 1, KT, h1)
    compare(gpu, g, r)


def _h_line(n_atoms, spacing=1.0):
    pos = np.zeros((n_atoms, 3))
    pos[:, 0] = np.arange(n_atoms) * spacing + 0.5
    box = max(n_atoms * spacing + 9.0, 10.0)
    return I.make_system(f"hline{n_atoms}", box, pos, ["H"] * n_atoms, {})


@pytest.mark.parametrize("n_atoms", [63, 64, 65, 130])
def test_tile_edges_complete(ctx, oracle_lib, n_atoms):
    """Subgraphs of exactly 63/64/65/130 orbitals (tile boundaries)."""
    O = oracle_lib
    s = _h_line(n_atoms)
    core = (np.arange(n_atoms) // 9).astype(np.int32)
    h1 = I.h1_diagonal(s, 1, seed=5)
    g, r = run_oracle(O, s, core, 0.0, None, 2, KT, h1)
    assert (g.sizes() == n_atoms).all()
    gpu = run_gpu(ctx, s, core, 0.0, None, 2, KT, h1)
    compare(gpu, g, r)


def test_max_size_complete(ctx, oracle_lib):
    """170 waters, cores of five molecules, complete graph: 34 subgraphs of
    1,020 orbitals (the multi-workgroup reduction, the largest
    divide-and-conquer merge kept in LDS, the largest four-wave register
    back-transform)."""
    O = oracle_lib
    s = I.water_system(170, 17.2, seed=171)
    core = (np.arange(s.n_atoms) // 15).astype(np.int32)
    h1 = I.h1_diagonal(s, 1, seed=172)
    g, r = run_oracle(O, s, core, 0.0, None, 2, KT, h1, pool=True)
    assert (g.sizes() == 1020).all() and g.n_core_orbs.max() <= 32
    _say("max size 1020 gpu")
    gpu = run_gpu(ctx, s, core, 0.0, None, 2, KT, h1)
    compare(gpu, g, r)


def test_tiny_subgraphs(ctx, oracle_lib):
    """Isolated molecules and a lone atom: subgraphs of 1, 3 and 6 orbitals."""
    O = oracle_lib
    w = I.isolated_molecules_system(7, 8.0, seed=9)
    pos = np.concatenate([w.pos, [[w.box - 0.5, w.box - 0.5, w.box - 0.5]]])
    s = I.make_system("iso+H", w.box, pos, w.species + ["H"], {})
    core = I.single_atom_cores(s)
    h1 = I.h1_diagonal(s, 1, seed=10)
    g, r = run_oracle(O, s, core, 1e-6, None, 0, KT, h1)
    assert g.sizes().min() == 1
    gpu = run_gpu(ctx, s, core, 1e-6, None, 0, KT, h1)
    compare(gpu, g, r)


def test_deterministic(ctx, oracle_lib):
    O = oracle_lib
    s, core, prev, h1 = case_water32(O, 0.07, 1)
    a = run_gpu(ctx, s, core, 0.07, prev, 1, KT, h1)
    b = run_gpu(ctx, s, core, 0.07, prev, 1, KT, h1)
    assert a["mu"] == b["mu"]
    assert np.array_equal(a["rho"], b["rho"]) and np.array_equal(a["rho1"], b["rho1"])
    assert np.array_equal(a["mu1"], b["mu1"])


@pytest.fixture(scope="module")
def water1000(oracle_lib):
    """The benchmark workload: 1,000 waters, 8-atom cores, paths of two at
    tau = 0.07 on the bootstrap density; one perturbation."""
    O = oracle_lib
    s = I.water1000_system()
    core = I.spatial_cores(s, 8)
    _say("water1000 oracle bootstrap")
    prev = O.bootstrap_prev(s, core, KT, pool=True)
    h1 = I.h1_diagonal(s, 1, seed=2002)
    _say("water1000 oracle solve")
    g, r = run_oracle(O, s, core, 0.07, prev, 1, KT, h1, pool=True)
    return s, core, prev, h1, g, r


def test_water1000_full_size(ctx, water1000):
    s, core, prev, h1, g, r = water1000
    _say(f"water1000 gpu: sizes {g.sizes().min()}..{g.sizes().max()}")
    gpu = run_gpu(ctx, s, core, 0.07, prev, 1, KT, h1)
    compare(gpu, g, r)


def test_water1000_invariants(ctx, water1000):
    """Properties that hold at any size: Tr rho = N_e, Tr rho1 = 0, and
    H1 = I gives mu1 = 1 with rho1 = 0."""
    s, core, prev, h1, g, r = water1000
    h = np.vstack([h1, np.ones((1, s.n_orb))])
    gpu = run_gpu(ctx, s, core, 0.07, prev, 1, KT, h)
    rows = np.repeat(np.arange(s.n_orb), np.diff(gpu["graph"]["rho_row_ptr"]))
    diag = rows == gpu["graph"]["rho_col"]
    assert abs(gpu["rho"][diag].sum() - s.n_elec) <= 1e-11 * s.n_elec
    assert abs(gpu["rho1"][0][diag].sum()) <= 1e-10
    assert abs(gpu["mu1"][1] - 1.0) <= 1e-12
    assert np.abs(gpu["rho1"][1]).max() <= 1e-10


# ----------------------------------------------------- split-FP32 response
TOL_MIXED = 1e-6


@pytest.mark.parametrize("kT", [0.003, 0.01, 0.03])
def test_split32_water60(ctx, oracle_lib, kT):
    """Split-FP32 congruences: rho stays FP64-exact, rho1 and mu1 within 1e-6
    of the FP64 oracle over the temperature range of the method."""
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    h1 = I.h1_diagonal(s, 3, seed=62)
    g, r = run_oracle(O, s, core, 0.07, prev, 1, kT, h1, pool=True)
    gpu = run_gpu(ctx, s, core, 0.07, prev, 1, kT, h1, precision=1)
    err = compare(gpu, g, r, tol1=TOL_MIXED)
    _say(f"split32 water60 kT={kT}: |dmu1| {err[0]:.2e} |drho1| {err[1]:.2e}")


def test_split32_chain_in_water(ctx, oracle_lib):
    O = oracle_lib
    s = I.chain_water_system(900, 180, seed=3001)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT, pool=True)
    h1 = I.h1_diagonal(s, 2, seed=3002)
    g, r = run_oracle(O, s, core, 0.07, prev, 1, 0.003, h1, pool=True)
    gpu = run_gpu(ctx, s, core, 0.07, prev, 1, 0.003, h1, precision=1)
    err = compare(gpu, g, r, tol1=TOL_MIXED)
    _say(f"split32 chain900 kT=0.003: |dmu1| {err[0]:.2e} |drho1| {err[1]:.2e}")


def test_split32_water1000_full_size(ctx, water1000):
    s, core, prev, h1, g, r = water1000
    gpu = run_gpu(ctx, s, core, 0.07, prev, 1, KT, h1, precision=1)
    err = compare(gpu, g, r, tol1=TOL_MIXED)
    _say(f"split32 water1000: |dmu1| {err[0]:.2e} |drho1| {err[1]:.2e}")


def test_split32_tile_edges(ctx, oracle_lib):
    """Ragged 64-tiles and a window that reaches the end of the spectrum."""
    O = oracle_lib
    s = _h_line(130)
    core = (np.arange(130) // 9).astype(np.int32)
    h1 = I.h1_diagonal(s, 1, seed=5)
    g, r = run_oracle(O, s, core, 0.0, None, 2, 0.03, h1)
    gpu = run_gpu(ctx, s, core, 0.0, None, 2, 0.03, h1, precision=1)
    compare(gpu, g, r, tol1=TOL_MIXED)


def test_split32_wide_window(ctx, oracle_lib):
    """A 300-atom hydrogen chain (a metallic band) at kT = 0.03: each subgraph
    has about 200 states within 8 kT of mu, all refined in FP64."""
    O = oracle_lib
    s = _h_line(300)
    core = (np.arange(300) // 25).astype(np.int32)
    h1 = I.h1_diagonal(s, 2, seed=7)
    g, r = run_oracle(O, s, core, 0.0, None, 2, 0.03, h1)
    sizes = g.sizes()
    start = np.concatenate([[0], np.cumsum(sizes)])
    wide = [int((np.abs(r.eps[start[i]:start[i + 1]] - r.mu) <= 8 * 0.03).sum())
            for i in range(g.n_sub)]
    assert min(wide) > 128, wide
    gpu = run_gpu(ctx, s, core, 0.0, None, 2, 0.03, h1, precision=1)
    err = compare(gpu, g, r, tol1=TOL_MIXED)
    _say(f"split32 wide window ({min(wide)}..{max(wide)} states): |dmu1| {err[0]:.2e} "
         f"|drho1| {err[1]:.2e}")


def test_error_paths(ctx):
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    s = I.water32_system()
    p = GraphPath(ctx, s, I.single_atom_cores(s), 1e-3, max_k=1)
    h1 = torch.zeros((1, s.n_orb), dtype=torch.float64, device="cuda")
    with pytest.raises(gq.GQError, match="call gq_density"):
        p.eigs.response(h1, p.p_blocks)
    p.eigs.solve(p.H)
    with pytest.raises(gq.GQError, match="kT"):
        p.eigs.density(0.0, s.n_elec)
    with pytest.raises(gq.GQError, match="N_e"):
        p.eigs.density(0.01, 2.0 * s.n_orb)
    p.eigs.density(0.01, s.n_elec)
    with pytest.raises(gq.GQError, match="max_k"):
        p.eigs.response(torch.zeros((2, s.n_orb), dtype=torch.float64, device="cuda"), p.p_blocks)


def test_enoconv_from_iteration_cap(ctx):
    """A leaf iteration cap of zero, set from the host, makes the eigensolver
    report non-convergence: every kernel ends normally and the next
    synchronising call returns GQ_ENOCONV; the default cap then succeeds."""
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    s = I.water32_system()
    p = GraphPath(ctx, s, I.single_atom_cores(s), 1e-3, max_k=1)
    ctx.set_iteration_cap(0)
    try:
        with pytest.raises(gq.GQError, match="did not converge") as ei:
            p.ground_state(KT)
        assert ei.value.status == -3
    finally:
        ctx.set_iteration_cap(60)
    mu = p.ground_state(KT)
    assert np.isfinite(mu)
    with pytest.raises(gq.GQError):
        ctx.set_iteration_cap(-1)


def test_size_limits_rejected(ctx):
    """Subgraphs above 2,048 orbitals and cores above 128 orbitals are refused
    when the workspace is created, with the limit in the message."""
    from paper_2212_01997_amd import gq
    s = I.water_system(350, 22.4, seed=181)  # 2,100 orbitals
    g = gq.Graph.for_system(s, (np.arange(s.n_atoms) // 15).astype(np.int32), 0.0, None,
                            gq.COMPLETE)
    assert g.info.max_n == 2100
    with pytest.raises(gq.GQError, match="exceeds the limit 2048"):
        gq.Eigs(ctx, g, 1)
    w = I.water32_system()
    core = (np.arange(w.n_atoms) // 66).astype(np.int32)  # 22 waters: 132 core orbitals
    g2 = gq.Graph.for_system(w, core, 1e-3)
    assert g2.info.max_c > 128
    with pytest.raises(gq.GQError, match="exceeds the limit 128"):
        gq.Eigs(ctx, g2, 1)


@pytest.mark.parametrize("atoms_per_core", [30, 45])
def test_large_cores(ctx, oracle_lib, atoms_per_core):
    """Cores of 30 and 45 atoms (60 and 90 core orbitals: two and three blocks
    of the 32-row core products), the shape of the paper's largest runs: rho,
    mu, rho1 and mu1 against the oracle (FP64 and split-FP32), the core-charge
    response (the diagonal-only path) and the non-orthogonal rows."""
    import torch
    from oracle import krylov as Kr, overlap as Ov
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = (np.arange(s.n_atoms) // atoms_per_core).astype(np.int32)
    prev = O.bootstrap_prev(s, core, KT)
    g = O.graph_build(s, core, 0.07, rho_prev=prev, flags=O.PATHS2)
    assert int(g.n_core_orbs.max()) > 32 * (1 if atoms_per_core == 30 else 2)
    h1 = I.h1_diagonal(s, 2, seed=182)
    ref = O.solve(s, g, KT, h1)
    p = GraphPath(ctx, s, core, 0.07, prev, gq.PATHS2, max_k=2)
    mu = p.ground_state(KT)
    assert abs(mu - ref.mu) <= TOL_MU
    assert np.abs(p.rho.cpu().numpy() - ref.rho).max() <= TOL
    h1d = torch.as_tensor(h1, device="cuda")
    for precision, tol in ((gq.PREC_FP64, TOL), (gq.PREC_SPLIT32, 1e-6)):
        mu1 = p.respond(h1d, precision=precision)
        p.sync()
        err = (np.abs(p.rho1_view(2).cpu().numpy() - ref.rho1).max(), np.abs(mu1 - ref.mu1).max())
        _say(f"cores of {atoms_per_core} atoms precision={precision}: |drho1| {err[0]:.1e} "
             f"|dmu1| {err[1]:.1e}")
        assert max(err) <= tol
    gamma = I.coulomb_kernel(s)
    v = I.charge_vectors(s, 2, seed=183)
    q1_ref, _ = Kr.charge_response(s, g, KT, gamma, v)
    cm = gq.ChargeModel(ctx, p.graph, gamma, kmax=2)
    q1, _ = cm.response(p.eigs, torch.as_tensor(v, device="cuda"))
    assert np.abs(q1.cpu().numpy() - q1_ref).max() <= TOL
    S = I.overlap_matrix(s)
    ov = Ov.solve(s, S, g, KT, h1)
    po = GraphPath(ctx, s, core, 0.07, prev, gq.PATHS2, max_k=2, S=S)
    po.ground_state(KT)
    po.respond(h1d)
    po.sync()
    assert np.abs(po.rho.cpu().numpy() - ov.rho_ao).max() <= TOL
    assert np.abs(po.rho1_view(2).cpu().numpy() - ov.rho1_ao).max() <= TOL


# ------------------------------------------------ the 30,000-atom system at full size
def test_chain30000_full_size_sampled():
    """The 30,000-atom chain-in-water system (3,750 subgraphs of 148..638
    orbitals, K = 6) at kT = 0.003, 0.01, 0.03: the graph bit-exact (digests of
    the oracle's maps), mu and mu1 against the oracle, rho and rho1 at 4,096
    sampled positions; FP64 within 1e-10, split-FP32 response within 1e-6.
    The stored values come from tests/golden/make_chain30000_golden.py (oracle only)."""
    import hashlib
    import json
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath, bootstrap_prev
    with open(os.path.join(os.path.dirname(__file__), "golden", "chain30000_oracle.json")) as f:
        gold = json.load(f)
    s = I.chain30000_system()
    core = I.spatial_cores(s, 8)
    ctx = gq.Context(0)
    prev = bootstrap_prev(ctx, s, core, KT)
    graph = gq.Graph.for_system(s, core, 0.07, prev, gq.PATHS2)
    ex = graph.export()
    for name, dig in gold["graph"].items():
        got = hashlib.sha256(np.ascontiguousarray(ex[name], np.int32).tobytes()).hexdigest()[:16]
        assert got == dig, name
    K = 6
    p = GraphPath(ctx, s, core, 0.07, graph=graph, max_k=K)
    h1 = torch.as_tensor(I.h1_diagonal(s, K, seed=3002), device="cuda")
    idx = np.array(gold["idx"])
    for kT in (0.003, 0.01, 0.03):
        g = gold["kT"][repr(kT)]
        mu = p.ground_state(kT)
        for precision, tol in ((0, TOL), (1, 1e-6)):
            mu1 = p.respond(h1, precision=precision)
            p.sync()
            rho = p.rho.cpu().numpy()[idx]
            rho1 = p.rho1_view(K).cpu().numpy()[:, idx]
            err = (abs(mu - g["mu"]), np.abs(rho - np.array(g["rho"])).max(),
                   np.abs(mu1 - np.array(g["mu1"])).max(), np.abs(rho1 - np.array(g["rho1"])).max())
            _say(f"chain30000 kT={kT} precision={precision}: |dmu| {err[0]:.1e} |drho| {err[1]:.1e} "
                 f"|dmu1| {err[2]:.1e} |drho1| {err[3]:.1e}")
            assert err[0] <= TOL_MU and err[1] <= TOL
            assert err[2] <= tol and err[3] <= tol
