"""The boundary's optional forms against the oracle and the plain forms.

- General (CSR) perturbations: X = Q^T h1_s Q from the gathered h1_s, for
  sparse perturbations on H's pattern and fully dense ones, FP64 within 1e-10
  and split-FP32 within 1e-6 of the oracle's CSR path (Eq. (ddlambda),
  Sec. IV.A); a diagonal perturbation given as CSR equals the diagonal kind.
- Warm-started chemical potential (Sec. II.G): the same root as a cold start
  from any guess.
- Context arena: results equal those of workspaces that allocate, the arena is
  handed back, and a workspace that does not fit is refused.
"""
import sys

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

pytestmark = pytest.mark.gpu

KT = 0.01
TOL = 1e-10
TOL_MIXED = 1e-6


def _say(msg):
    print(f"[gpu-boundary] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2212_01997_amd import gq
    return gq.Context(0)


def _device_csrs(mats):
    from paper_2212_01997_amd import gq
    return [gq.DeviceCsr(*m) for m in mats]


def _run_csr(ctx, s, core, tau, prev, flags, kT, mats, precision=0):
    import torch
    from paper_2212_01997_amd.path import GraphPath
    K = len(mats)
    p = GraphPath(ctx, s, core, tau, prev, flags, max_k=K, general_h1=True)
    mu = p.ground_state(kT)
    dm = _device_csrs(mats)
    mu1 = p.respond(dm, precision=precision)
    torch.cuda.synchronize()
    return mu, mu1, p.rho.cpu().numpy(), p.rho1_view(K).cpu().numpy(), p


def _check_vs_oracle(O, s, core, tau, prev, flags, kT, mats, gpu, tol1):
    g = O.graph_build(s, core, tau, rho_prev=prev, flags=flags)
    r = O.solve(s, g, kT, list(mats))
    mu, mu1, rho, rho1, _ = gpu
    assert abs(mu - r.mu) <= 1e-12
    assert np.abs(rho - r.rho).max() <= TOL
    err = (np.abs(mu1 - r.mu1).max(), np.abs(rho1 - r.rho1).max())
    assert err[0] <= tol1 and err[1] <= tol1, err
    return err


@pytest.mark.parametrize("precision,tol1", [(0, TOL), (1, TOL_MIXED)], ids=["fp64", "split32"])
def test_csr_pattern_water32(ctx, oracle_lib, precision, tol1):
    O = oracle_lib
    s = I.water32_system()
    core = I.single_atom_cores(s)
    prev = O.bootstrap_prev(s, core, KT)
    mats = I.h1_on_pattern(s, 2, seed=1003)
    _say(f"csr pattern water32 precision={precision}")
    gpu = _run_csr(ctx, s, core, 0.07, prev, 1, KT, mats, precision)
    err = _check_vs_oracle(O, s, core, 0.07, prev, 1, KT, mats, gpu, tol1)
    _say(f"  |dmu1| {err[0]:.2e} |drho1| {err[1]:.2e}")


@pytest.mark.parametrize("precision,tol1", [(0, TOL), (1, TOL_MIXED)], ids=["fp64", "split32"])
def test_csr_dense_water32_complete(ctx, oracle_lib, precision, tol1):
    """Fully dense H1 on the complete graph (192-orbital subgraphs: three
    64-tiles and a ragged one)."""
    O = oracle_lib
    s = I.water32_system()
    core = I.single_atom_cores(s)
    mats = I.h1_dense(s, 1, seed=1004)
    _say(f"csr dense water32 complete precision={precision}")
    gpu = _run_csr(ctx, s, core, 1e-5, None, 2, KT, mats, precision)
    err = _check_vs_oracle(O, s, core, 1e-5, None, 2, KT, mats, gpu, tol1)
    _say(f"  |dmu1| {err[0]:.2e} |drho1| {err[1]:.2e}")


@pytest.mark.parametrize("precision,tol1", [(0, TOL), (1, TOL_MIXED)], ids=["fp64", "split32"])
def test_csr_water60(ctx, oracle_lib, precision, tol1):
    """8-atom spatial cores, paths of two (subgraphs spanning several tiles),
    three perturbations on H's pattern."""
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    mats = I.h1_on_pattern(s, 3, seed=63)
    _say(f"csr water60 precision={precision}")
    gpu = _run_csr(ctx, s, core, 0.07, prev, 1, KT, mats, precision)
    err = _check_vs_oracle(O, s, core, 0.07, prev, 1, KT, mats, gpu, tol1)
    _say(f"  |dmu1| {err[0]:.2e} |drho1| {err[1]:.2e}")


def test_diagonal_as_csr_equals_diagonal(ctx, oracle_lib):
    """The two kinds are two routes to the same X: a diagonal perturbation
    given as CSR agrees with the diagonal kind to rounding."""
    import torch
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    d = I.h1_diagonal(s, 2, seed=62)
    mats = [(np.arange(s.n_orb + 1, dtype=np.int32), np.arange(s.n_orb, dtype=np.int32), row)
            for row in d]
    mu, mu1c, rho, rho1c, p = _run_csr(ctx, s, core, 0.07, prev, 1, KT, mats)
    mu1d = p.respond(torch.as_tensor(d, device="cuda"))
    torch.cuda.synchronize()
    rho1d = p.rho1_view(2).cpu().numpy()
    assert np.abs(mu1c - mu1d).max() <= 1e-12
    assert np.abs(rho1c - rho1d).max() <= 1e-12


def test_csr_needs_general_workspace(ctx):
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    s = I.water32_system()
    p = GraphPath(ctx, s, I.single_atom_cores(s), 1e-3, max_k=1)
    p.ground_state(KT)
    dm = _device_csrs(I.h1_on_pattern(s, 1, seed=5))
    with pytest.raises(gq.GQError, match="GQ_EIGS_GENERAL_H1"):
        p.eigs.response(dm, p.p_blocks)
    bad = gq.DeviceCsr(np.zeros(3, np.int32), np.zeros(0, np.int32), np.zeros(0))
    q = GraphPath(ctx, s, I.single_atom_cores(s), 1e-3, max_k=1, general_h1=True)
    q.ground_state(KT)
    with pytest.raises(gq.GQError, match="rows"):
        q.eigs.response([bad], q.p_blocks)
    torch.cuda.synchronize()


@pytest.mark.parametrize("shift", [0.0, 1e-9, -3e-4, 0.05, -0.6, 40.0])
def test_warm_start_same_root(ctx, oracle_lib, shift):
    """Guesses at the root, near it, far from it and outside the spectrum
    all give the cold-start root (to the last bits of the bracket) and the
    same density."""
    O = oracle_lib
    from paper_2212_01997_amd.path import GraphPath
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    p = GraphPath(ctx, s, core, 0.07, prev, 1, max_k=1)
    mu0 = p.ground_state(KT)
    rho0 = p.rho.cpu().numpy()
    mu = p.ground_state(KT, mu_guess=mu0 + shift)
    rho = p.rho.cpu().numpy()
    _say(f"warm start shift {shift}: mu {mu!r} cold {mu0!r}")
    assert abs(mu - mu0) <= 4 * np.spacing(abs(mu0))
    assert np.abs(rho - rho0).max() <= 1e-13


def test_arena_context(oracle_lib):
    """Workspaces on a context with an arena: the same bits as on a plain
    context, the arena is returned on destruction, and a workspace larger
    than the free arena is refused with GQ_ENOMEM."""
    import gc
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    h1 = torch.as_tensor(I.h1_diagonal(s, 2, seed=62), device="cuda")
    plain = gq.Context(0)
    a = GraphPath(plain, s, core, 0.07, prev, 1, max_k=2)
    mu_a = a.ground_state(KT)
    mu1_a = a.respond(h1)
    arena_ctx = gq.Context(0, arena_bytes=256 << 20)
    b = GraphPath(arena_ctx, s, core, 0.07, prev, 1, max_k=2)
    used, size = arena_ctx.arena_used()
    assert size == 256 << 20 and used >= b.graph.footprint(2)
    mu_b = b.ground_state(KT)
    mu1_b = b.respond(h1)
    torch.cuda.synchronize()
    assert mu_a == mu_b and np.array_equal(mu1_a, mu1_b)
    assert np.array_equal(a.rho.cpu().numpy(), b.rho.cpu().numpy())
    assert np.array_equal(a.rho1.cpu().numpy(), b.rho1.cpu().numpy())
    del b
    gc.collect()
    assert arena_ctx.arena_used()[0] == 0
    small = gq.Context(0, arena_bytes=1 << 20)
    with pytest.raises(gq.GQError, match="arena"):
        GraphPath(small, s, core, 0.07, prev, 1, max_k=2)
