"""Parity of the non-orthogonal basis on the GPU (gq_submatrix_solve_overlap:
Lowdin factor of every overlap submatrix, h = z h_ao z, C = z Q; then the
atomic-orbital density and response rows, Sec. II.D and Sec. IV.B) with the
oracle (oracle/overlap.py), through the C ABI.

Bar: mu within 1e-12, rho and rho1 (atomic-orbital rows) and mu1 within
1e-10, the FP64 bar of the orthogonal path: the overlap submatrices are
well conditioned (eigenvalues in [0.3, 2] by construction), so the extra
congruences add rounding of the same order as the eigensolve's.
"""
import sys

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

pytestmark = pytest.mark.gpu

KT = 0.01
TOL = 1e-10


def _say(msg):
    print(f"[gpu-overlap] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2212_01997_amd import gq
    return gq.Context(0)


@pytest.fixture(scope="module")
def V():
    from oracle import overlap
    return overlap


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
    return s, core, prev, g


@pytest.mark.parametrize("name,K,general", [("water32", 3, False), ("water60", 3, False),
                                            ("water32", 2, True), ("chain900", 0, False)])
def test_overlap_parity(ctx, oracle_lib, V, name, K, general):
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    O = oracle_lib
    s, core, prev, g = _case(name, O)
    S = I.overlap_matrix(s)
    h1 = (I.h1_on_pattern(s, K, seed=77) if general else I.h1_diagonal(s, K, seed=77)) if K else None
    ref = V.solve(s, S, g, KT, h1)
    p = GraphPath(ctx, s, core, 0.07, prev, gq.PATHS2, max_k=max(K, 1), general_h1=general, S=S)
    mu = p.ground_state(KT)
    err = {"mu": abs(mu - ref.mu), "rho": float(np.abs(p.rho.cpu().numpy() - ref.rho_ao).max())}
    if K:
        dev = ([gq.DeviceCsr(*m) for m in h1] if general
               else torch.as_tensor(h1, device="cuda"))
        mu1 = p.respond(dev)
        p.sync()
        err["rho1"] = float(np.abs(p.rho1_view(K).cpu().numpy() - ref.rho1_ao).max())
        err["mu1"] = float(np.abs(mu1 - ref.mu1).max())
    _say(f"{name} K={K} general={general}: " + " ".join(f"{k} {v:.1e}" for k, v in err.items()))
    assert err["mu"] <= 1e-12
    assert max(v for k, v in err.items() if k != "mu") <= TOL


def test_identity_overlap_matches_orthogonal_path(ctx, oracle_lib):
    """S = I: the overlap path equals the orthogonal GPU path."""
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    O = oracle_lib
    s, core, prev, g = _case("water32", O)
    n = s.n_orb
    eye = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    h1 = torch.as_tensor(I.h1_diagonal(s, 2, seed=78), device="cuda")
    a = GraphPath(ctx, s, core, 0.07, prev, gq.PATHS2, max_k=2, S=eye)
    b = GraphPath(ctx, s, core, 0.07, prev, gq.PATHS2, max_k=2)
    mus = (a.ground_state(KT), b.ground_state(KT))
    mu1s = (a.respond(h1), b.respond(h1))
    a.sync()
    b.sync()
    assert abs(mus[0] - mus[1]) <= 1e-13
    assert (a.rho - b.rho).abs().max().item() <= 1e-12
    assert (a.rho1_view(2) - b.rho1_view(2)).abs().max().item() <= 1e-12
    assert np.abs(mu1s[0] - mu1s[1]).max() <= 1e-12


def test_overlap_static_response_matches(ctx, oracle_lib):
    """gq_response_static on a workspace solved with an overlap gives the
    bits of gq_response."""
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    O = oracle_lib
    s, core, prev, g = _case("water32", O)
    h1 = torch.as_tensor(I.h1_diagonal(s, 3, seed=79), device="cuda")
    p = GraphPath(ctx, s, core, 0.07, prev, gq.PATHS2, max_k=3, S=I.overlap_matrix(s))
    p.ground_state(KT)
    p.respond(h1)
    p.sync()
    ref = p.p_blocks.clone()
    out = torch.empty_like(ref)
    p.eigs.response_static(h1, out)
    p.sync()
    assert torch.equal(out, ref)


def test_overlap_errors(ctx, oracle_lib):
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    s = I.water32_system()
    core = I.spatial_cores(s, 3)
    S = I.overlap_matrix(s)
    Sd = gq.DeviceCsr(*S)
    plain = GraphPath(ctx, s, core, 1e-3)
    with pytest.raises(gq.GQError, match="GQ_EIGS_OVERLAP"):
        plain.eigs.solve_overlap(plain.H, Sd)
    # an overlap with one negative diagonal entry is not positive definite
    bad = (S[0], S[1], S[2].copy())
    rows = np.repeat(np.arange(s.n_orb), np.diff(S[0]))
    bad[2][np.flatnonzero(rows == S[1])[5]] = -1.0
    p = GraphPath(ctx, s, core, 1e-3, S=bad)
    with pytest.raises(gq.GQError, match="not positive definite"):
        p.ground_state(KT)
    p = GraphPath(ctx, s, core, 1e-3, max_k=1, S=S)
    p.ground_state(KT)
    h1 = torch.as_tensor(I.h1_diagonal(s, 1, seed=80), device="cuda")
    with pytest.raises(gq.GQError, match="FP64"):
        p.respond(h1, precision=gq.PREC_SPLIT32)
    cm = gq.ChargeModel(ctx, p.graph, I.coulomb_kernel(s), kmax=1)
    with pytest.raises(gq.GQError, match="orthogonal basis"):
        cm.response(p.eigs, torch.zeros((1, s.n_atoms), dtype=torch.float64, device="cuda"))
    with pytest.raises(gq.GQError, match="rows"):
        other = I.water_system(6, 8.0, seed=71)
        p.eigs.solve_overlap(gq.DeviceCsr(other.h_row_ptr, other.h_col, other.h_val), Sd)
