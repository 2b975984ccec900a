"""Pins of the charge-response / preconditioner / Krylov-kernel oracle
(oracle/krylov.py, Sec. V) against what the mathematics fixes.

- The charge response equals the central finite difference (4-point) of the
  collected core charges under H +- lambda H1[v], graph fixed, mu re-solved.
- On a system with one core holding every atom, k0 with alpha = 0 is the
  inverse of the finite-difference Jacobian of f = rho_0[n] - n (the
  column-sum shift is then the canonical mu1, Sec. V.A).
- Column sums of every core Jacobian are -1 (charge conservation, Sec. V.A).
- The Krylov vectors are orthonormal.
- With m equal to the number of atoms the low-rank operator
  sum_ij v_i M_ij f_{v_j}^T is (K0 J)^-1 and n'' = -omega^2 J^-1 f, the
  Newton step; J from finite differences, not from the response code.
CPU only.
"""
import copy

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

KT = 0.01


def _shift(system, d, lam):
    """System with H + lam * diag(d) over the orbitals."""
    s = copy.copy(system)
    rows = np.repeat(np.arange(system.n_orb), np.diff(system.h_row_ptr))
    val = system.h_val.copy()
    diag = rows == system.h_col
    val[diag] += lam * d[rows[diag]]
    s.h_val = val
    return s


def _fd_charges(O, K, system, graph, gamma, v, lam=1e-4):
    """4-point central difference of rho_0 along H1[v]."""
    d = K.orbital_diagonal(system, K.atom_potential(gamma, v))
    q = {}
    for k in (-2, -1, 1, 2):
        r = O.solve(_shift(system, d, k * lam), graph, KT)
        q[k] = K.core_charges(system, graph, r.rho)
    return (8 * (q[1] - q[-1]) - (q[2] - q[-2])) / (12 * lam)


def _fd_jacobian(O, K, system, graph, gamma):
    n = system.n_atoms
    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        J[:, j] = _fd_charges(O, K, system, graph, gamma, e) - e
    return J


@pytest.fixture(scope="module")
def small():
    s = I.water_system(6, 8.0, seed=71)
    return s, I.coulomb_kernel(s)


@pytest.fixture(scope="module")
def K(oracle_lib):
    from oracle import krylov
    return krylov


def test_charge_response_is_the_derivative(oracle_lib, K, small):
    O = oracle_lib
    s, gamma = small
    g = O.graph_build(s, I.single_atom_cores(s), 1e-3)
    v = I.charge_vectors(s, 2, seed=72)
    q1, _ = K.charge_response(s, g, KT, gamma, v)
    for i in range(2):
        fd = _fd_charges(O, K, s, g, gamma, v[i])
        assert np.abs(q1[i] - fd).max() <= 1e-9 * max(1.0, np.abs(fd).max())
    # the perturbation moves no charge in total (Tr rho1 = 0)
    assert np.abs(q1.sum(axis=1)).max() <= 1e-12


def test_one_core_preconditioner_is_the_inverse_jacobian(oracle_lib, K, small):
    O = oracle_lib
    s, gamma = small
    core = np.zeros(s.n_atoms, dtype=np.int32)
    g = O.graph_build(s, core, 0.0)
    mu = O.solve(s, g, KT).mu
    k0s, js = K.preconditioner(s, g, KT, gamma, 0.0, mu)
    J = _fd_jacobian(O, K, s, g, gamma)
    assert np.abs(js[0] - J).max() <= 1e-8
    Jinv = np.linalg.inv(J)
    assert np.abs(k0s[0] - Jinv).max() <= 1e-7 * np.abs(Jinv).max()


def test_column_sums_and_regularisation(oracle_lib, K, small):
    O = oracle_lib
    s, gamma = small
    g = O.graph_build(s, I.spatial_cores(s, 3), 1e-3)
    mu = O.solve(s, g, KT).mu
    alpha = 0.3
    k0s, js = K.preconditioner(s, g, KT, gamma, alpha, mu)
    for k0, j in zip(k0s, js):
        assert np.abs(j.sum(axis=0) + 1.0).max() <= 1e-12
        m = len(j)
        assert np.abs(k0 @ (j - alpha * np.eye(m)) - np.eye(m)).max() <= 1e-12


def test_full_rank_krylov_is_the_newton_step(oracle_lib, K, small):
    O = oracle_lib
    s, gamma = small
    g = O.graph_build(s, I.single_atom_cores(s), 1e-3)
    r = O.solve(s, g, KT)
    k0s, _ = K.preconditioner(s, g, KT, gamma, 0.2, r.mu)
    q0 = K.core_charges(s, g, r.rho)
    n = q0 + I.charge_vectors(s, 1, seed=73)[0]
    m = s.n_atoms
    out = K.krylov_kernel(s, g, KT, gamma, k0s, n, m, omega=1.3)
    V = out["V"]
    assert np.abs(V @ V.T - np.eye(m)).max() <= 1e-12
    J = _fd_jacobian(O, K, s, g, gamma)
    K0 = np.zeros((m, m))
    for i in range(m):
        e = np.zeros(m)
        e[i] = 1.0
        K0[:, i] = K.apply_k0(s, g, k0s, e)
    low_rank = V.T @ out["M"] @ out["F"]
    ref = np.linalg.inv(K0 @ J)
    assert np.abs(low_rank - ref).max() <= 1e-6 * np.abs(ref).max()
    newton = -1.3 ** 2 * np.linalg.solve(J, q0 - n)
    assert np.abs(out["ndd"] - newton).max() <= 1e-6 * np.abs(newton).max()


def test_low_rank_vectors_orthonormal(oracle_lib, K):
    O = oracle_lib
    s = I.water32_system()
    gamma = I.coulomb_kernel(s)
    g = O.graph_build(s, I.single_atom_cores(s), 1e-3)
    r = O.solve(s, g, KT)
    k0s, _ = K.preconditioner(s, g, KT, gamma, 0.2, r.mu)
    n = K.core_charges(s, g, r.rho) + I.charge_vectors(s, 1, seed=13)[0]
    out = K.krylov_kernel(s, g, KT, gamma, k0s, n, 4)
    assert np.abs(out["V"] @ out["V"].T - np.eye(4)).max() <= 1e-12
    assert np.abs(out["O"] - out["O"].T).max() <= 1e-14 * np.abs(out["O"]).max()
