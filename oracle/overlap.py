"""Reference oracle for the graph-based density and canonical response in a
non-orthogonal basis (arXiv:2212.01997, Sec. II.D, Eqs. (DD0)-(ksSmall) and
the atomic-orbital congruence after them; Sec. IV.B for the response).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite; the GPU library
neither imports nor links it.  Plain numpy on top of the pinned C oracle
(oracle.py), which supplies every eigensolve, Fermi row, divided difference
and response row; the steps below follow the paper's order and notation.

Per subgraph i: s = S[orbs, orbs] and h_ao = H[orbs, orbs] (principal
submatrices of the composite overlap and Hamiltonian), z = s^(-1/2) (the
Lowdin choice of the inverse factor with z^T s z = I), h = z^T h_ao z
(Eq. (ksSmall)), h = Q diag(eps) Q^T (Eq. (SmallKS)).  The shared mu and the
canonical mu1 are fixed on the traces of the collected density in the
orthogonalized form (Eq. (DD)), exactly as in the orthogonal case; the
atomic-orbital rows are the core rows of z d z^T, that is
2 C_c diag(f) C^T with C = z Q.  A perturbation H1 given in the atomic-orbital
basis enters as h1 = z^T h1_ao z, so Q^T h1 Q = C^T h1_ao C, and the
atomic-orbital response rows are 2 C_c [(C^T h1_ao C) o dF + mu1 beta
diag(f (1 - f))] C^T, the core rows of z d1 z^T.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import oracle as O


def lowdin(s):
    """z = s^(-1/2) from the pinned eigensolve; s must be positive definite."""
    w, v = O.eigh(s)
    if w.min() <= 0.0:
        raise ValueError(f"overlap submatrix not positive definite (smallest eigenvalue {w.min()})")
    return (v * w ** -0.5) @ v.T


@dataclass
class Result:
    mu: float
    rho: np.ndarray        # [nnz] collected orthogonalized density (Eq. (DD))
    rho_ao: np.ndarray     # [nnz] collected atomic-orbital density rows
    rho1_ao: np.ndarray    # [K, nnz] collected atomic-orbital response rows
    mu1: np.ndarray        # [K]
    eps: np.ndarray        # [sum n] eigenvalues of h = z^T h_ao z, subgraph by subgraph


def solve(system, S, graph, kT, h1=None, n_elec=None) -> Result:
    """The whole path in a non-orthogonal basis.  S is a host CSR triple
    (row_ptr, col, val); h1 the atomic-orbital perturbations: a [K, N] array of
    diagonals, a list of K host CSR triples, or None."""
    H = O.Csr(system.h_row_ptr, system.h_col, system.h_val)
    Sc = O.Csr(*S)
    if h1 is None:
        pert = []
    elif isinstance(h1, np.ndarray):
        pert = [O.Csr.diagonal(row) for row in np.atleast_2d(h1)]
    else:
        pert = [O.Csr(*m) for m in h1]
    K = len(pert)
    ne = system.n_elec if n_elec is None else n_elec
    subs = []
    for s in range(graph.n_sub):
        orbs = graph.orbs(s)
        c = int(graph.n_core_orbs[s])
        z = lowdin(O.gather(Sc, orbs))
        h = z.T @ O.gather(H, orbs) @ z
        e, q = O.eigh(h)
        subs.append((orbs, c, z, e, q, O.core_weights(q, c)))
    eps = np.concatenate([x[3] for x in subs])
    mu = O.find_mu(eps, np.concatenate([x[5] for x in subs]), kT, ne)
    rho = np.zeros(graph.nnz)
    rho_ao = np.zeros(graph.nnz)
    lam_ao = np.zeros((K, graph.nnz))
    mur_ao = np.zeros(graph.nnz)
    tlam = np.zeros((K, graph.n_sub))
    tmu = np.zeros(graph.n_sub)
    for s, (orbs, c, z, e, q, _) in enumerate(subs):
        C = z @ q
        O.collect(graph, s, O.core_rows(q, e, c, mu, kT), rho)
        O.collect(graph, s, O.core_rows(C, e, c, mu, kT), rho_ao)
        _, tmu[s] = O.mu_response_rows(q, e, c, mu, kT)
        O.collect(graph, s, O.mu_response_rows(C, e, c, mu, kT)[0], mur_ao)
        if K:
            dF = O.divided_differences(e, mu, kT)
            for k in range(K):
                # the orthogonalized perturbation fixes the trace (mu1); the
                # same X = Q^T h1 Q = C^T h1_ao C gives the atomic-orbital rows
                h1_ao = O.gather(pert[k], orbs)
                _, tlam[k, s] = O.lambda_response_rows(q, dF, z.T @ h1_ao @ z, c)
                rows_ao, _ = O.lambda_response_rows(C, dF, h1_ao, c)
                O.collect(graph, s, rows_ao, lam_ao[k])
    mu1 = np.array([O.mu1(tlam[k], tmu) for k in range(K)])
    rho1_ao = lam_ao + mu1[:, None] * mur_ao[None, :]
    return Result(mu, rho, rho_ao, rho1_ao, mu1, eps)
