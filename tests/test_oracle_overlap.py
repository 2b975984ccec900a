"""Pins of the non-orthogonal-basis oracle (oracle/overlap.py, Sec. II.D,
Eqs. (DD)-(ksSmall) and the atomic-orbital congruence; Sec. IV.B) against
what the mathematics fixes:

- S = I reduces it to the orthogonal oracle (mu, rho, rho1, mu1) and the
  atomic-orbital rows to the orthogonalized ones.
- Lowdin factor: z^T s z = I and z = z^T.
- Generalized eigenproblem (scipy's eigh(h_ao, s), an independent route that
  does not depend on the choice of z): the subgraph eigenvalues, and the
  atomic-orbital density rows 2 C f C^T from its eigenvectors, collected.
- With a complete graph every subgraph is the whole system: the Mulliken
  count Tr(D_ao S) equals the electron count and Tr(D1_ao S) is zero.
- The atomic-orbital response rows equal the 4-point central difference of
  the collected atomic-orbital density under H + lambda diag(h1), mu
  re-solved (the canonical response).
CPU only.
"""
import copy

import numpy as np
import pytest
import scipy.linalg

from paper_2212_01997_amd import inputs as I

KT = 0.01


@pytest.fixture(scope="module")
def V(oracle_lib):
    from oracle import overlap
    return overlap


@pytest.fixture(scope="module")
def small(oracle_lib):
    O = oracle_lib
    s = I.water_system(6, 8.0, seed=71)
    core = I.spatial_cores(s, 3)
    g = O.graph_build(s, core, 1e-5)
    return s, g, I.overlap_matrix(s), I.h1_diagonal(s, 2, seed=72)


def _shift(system, d, lam):
    s = copy.copy(system)
    rows = np.repeat(np.arange(system.n_orb), np.diff(system.h_row_ptr))
    val = system.h_val.copy()
    diag = rows == system.h_col
    val[diag] += lam * d[rows[diag]]
    s.h_val = val
    return s


def test_identity_overlap_is_orthogonal_case(oracle_lib, V, small):
    O = oracle_lib
    s, g, _, h1 = small
    n = s.n_orb
    eye = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    r = V.solve(s, eye, g, KT, h1)
    ref = O.solve(s, g, KT, h1)
    assert abs(r.mu - ref.mu) <= 1e-13
    assert np.abs(r.rho - ref.rho).max() <= 1e-12
    assert np.abs(r.rho_ao - ref.rho).max() <= 1e-12
    assert np.abs(r.rho1_ao - ref.rho1).max() <= 1e-11
    assert np.abs(r.mu1 - ref.mu1).max() <= 1e-11


def test_identity_overlap_general_perturbation(oracle_lib, V, small):
    O = oracle_lib
    s, g, _, _ = small
    n = s.n_orb
    eye = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    h1 = I.h1_on_pattern(s, 2, seed=75)
    r = V.solve(s, eye, g, KT, h1)
    ref = O.solve(s, g, KT, h1)
    assert np.abs(r.rho1_ao - ref.rho1).max() <= 1e-11
    assert np.abs(r.mu1 - ref.mu1).max() <= 1e-11


def test_lowdin_factor(oracle_lib, V, small):
    O = oracle_lib
    s, g, S, _ = small
    sub = O.gather(O.Csr(*S), g.orbs(0))
    z = V.lowdin(sub)
    assert np.abs(z.T @ sub @ z - np.eye(len(z))).max() <= 1e-13
    assert np.abs(z - z.T).max() <= 1e-14
    with pytest.raises(ValueError):
        V.lowdin(np.diag([1.0, -0.5]))


def test_generalized_eigenproblem(oracle_lib, V, small):
    O = oracle_lib
    s, g, S, _ = small
    r = V.solve(s, S, g, KT)
    H = O.Csr(s.h_row_ptr, s.h_col, s.h_val)
    Sc = O.Csr(*S)
    ref = np.zeros(g.nnz)
    for i in range(g.n_sub):
        orbs = g.orbs(i)
        c = int(g.n_core_orbs[i])
        w, C = scipy.linalg.eigh(O.gather(H, orbs), O.gather(Sc, orbs))
        e = r.eps[g.sub_orb_ptr[i]:g.sub_orb_ptr[i + 1]]
        assert np.abs(np.sort(e) - w).max() <= 1e-12
        f = 1.0 / (1.0 + np.exp((w - r.mu) / KT))
        O.collect(g, i, np.ascontiguousarray(2.0 * (C[:c] * f) @ C.T), ref)
    assert np.abs(r.rho_ao - ref).max() <= 1e-11
    assert np.abs(r.rho_ao - r.rho).max() > 1e-3  # the basis matters


def test_complete_graph_mulliken_counts(oracle_lib, V):
    O = oracle_lib
    s = I.water_system(4, 8.0, seed=73)
    core = I.spatial_cores(s, 3)
    g = O.graph_build(s, core, 0.0, flags=O.COMPLETE)
    S = I.overlap_matrix(s)
    h1 = I.h1_diagonal(s, 1, seed=74)
    r = V.solve(s, S, g, KT, h1)
    n = s.n_orb
    Sd = I.csr_to_dense(*S, n)
    D = I.csr_to_dense(g.rho_row_ptr, g.rho_col, r.rho_ao, n)
    D1 = I.csr_to_dense(g.rho_row_ptr, g.rho_col, r.rho1_ao[0], n)
    assert abs(np.trace(D @ Sd) - s.n_elec) <= 1e-10
    assert abs(np.trace(D1 @ Sd)) <= 1e-10
    assert np.abs(D - D.T).max() <= 1e-12


def test_response_is_finite_difference(oracle_lib, V, small):
    s, g, S, h1 = small
    r = V.solve(s, S, g, KT, h1)
    lam = 1e-4
    for k in range(h1.shape[0]):
        q = {j: V.solve(_shift(s, h1[k], j * lam), S, g, KT).rho_ao for j in (-2, -1, 1, 2)}
        fd = (8 * (q[1] - q[-1]) - (q[2] - q[-2])) / (12 * lam)
        assert np.abs(fd - r.rho1_ao[k]).max() <= 1e-8


def test_general_response_is_finite_difference(oracle_lib, V, small):
    """A perturbation on the whole pattern of H (off-diagonal entries too)."""
    s, g, S, _ = small
    h1 = I.h1_on_pattern(s, 1, seed=76)
    r = V.solve(s, S, g, KT, h1)
    lam = 1e-4
    q = {}
    for j in (-2, -1, 1, 2):
        sj = copy.copy(s)
        sj.h_val = s.h_val + j * lam * h1[0][2]
        q[j] = V.solve(sj, S, g, KT).rho_ao
    fd = (8 * (q[1] - q[-1]) - (q[2] - q[-2])) / (12 * lam)
    assert np.abs(fd - r.rho1_ao[0]).max() <= 1e-8
