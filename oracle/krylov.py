"""Reference oracle for the charge response, the subgraph preconditioner and
the preconditioned low-rank Krylov kernel of graph-based shadow molecular
dynamics (arXiv:2212.01997, Sec. V).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite and nothing else; the
GPU library neither imports nor links it.  Plain numpy on top of the pinned
C oracle (oracle.py): every per-subgraph eigensolve, divided difference and
response row comes from there, and the vector steps below follow the paper's
order and notation.

Notation (Sec. IV.B and V): n is the vector of atomic charges (electron
populations here); a charge vector v acts on every orbital of atom I through
the potential (gamma v)_I, H1[v] = diag(gamma v) over the orbitals; rho_0[n]
collects per atom the diagonal of the core rows of the ground-state density;
f = rho_0 - n is the residual and J its Jacobian; K0 = {k0^(k)} the
block-diagonal preconditioner over the core atoms of every subgraph; v_i the
orthonormal Krylov vectors, f_{v_i} = K0 J v_i, O_ij = f_{v_i} . f_{v_j},
M = O^-1.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def atom_potential(gamma, v):
    """(gamma v)_I for the atom-by-atom kernel gamma given as a CSR triple."""
    rp, col, val = gamma
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    return np.bincount(rows, weights=val * np.asarray(v)[col], minlength=n)


def orbital_diagonal(system, V):
    """The diagonal of H1: every orbital of atom I carries the potential V_I."""
    return np.repeat(np.asarray(V, dtype=np.float64), np.diff(system.atom_orb_ptr))


def core_charges(system, graph, rho_vals):
    """rho_0 per atom (Eq. (assemble_rho0)): the diagonal entries rho_aa of the
    collected core rows, summed over the orbitals a of each atom."""
    N = system.n_orb
    rows = np.repeat(np.arange(N), np.diff(graph.rho_row_ptr))
    diag = np.zeros(N)
    hit = rows == graph.rho_col
    diag[rows[hit]] = np.asarray(rho_vals)[hit]
    atom_of = np.repeat(np.arange(system.n_atoms), np.diff(system.atom_orb_ptr))
    return np.bincount(atom_of, weights=diag, minlength=system.n_atoms)


def charge_response(system, graph, kT, gamma, vs):
    """The derivative of rho_0 along each charge vector v (the first term of
    the directional derivative, Eq. (dfdv)): the graph-based canonical response
    (Eqs. (D1), (dmu_1)) to H1[v] = diag(gamma v), its core charges collected.
    Returns ([K, n_atoms] responses, the oracle's whole-path result)."""
    vs = np.atleast_2d(vs)
    h1 = np.array([orbital_diagonal(system, atom_potential(gamma, v)) for v in vs])
    r = O.solve(system, graph, kT, h1)
    return np.array([core_charges(system, graph, r.rho1[q]) for q in range(len(vs))]), r


def _core_atom_orbitals(system, graph, s):
    """The core atoms of subgraph s and, for each, its local orbital indices
    (the core orbitals come first in the subgraph, atom after atom)."""
    a0 = graph.sub_ptr[s]
    atoms = graph.sub_atoms[a0:a0 + graph.n_core_atoms[s]]
    aop = system.atom_orb_ptr
    out, at = [], 0
    for I in atoms:
        k = int(aop[I + 1] - aop[I])
        out.append(np.arange(at, at + k))
        at += k
    return atoms, out


def preconditioner(system, graph, kT, gamma, alpha, mu):
    """Sec. V.A, Eq. (PreCond): for every subgraph k the core-atom Jacobian
    j^(k) (Eqs. (Jacob), (TwoDer)) from the responses to a unit charge on each
    core atom J (H1 = the potential of that charge, gamma[., J] on every
    orbital, restricted to the subgraph), with the chemical-potential response
    of each column chosen so that the column sums over the core are -1, and
    k0^(k) = (j^(k) - alpha I)^-1.  Returns (k0 blocks, j blocks), one
    m_k x m_k array per subgraph (m_k core atoms)."""
    H = O.Csr(system.h_row_ptr, system.h_col, system.h_val)
    rp, col, val = gamma
    atom_of = np.repeat(np.arange(system.n_atoms), np.diff(system.atom_orb_ptr))
    k0s, js = [], []
    for s in range(graph.n_sub):
        orbs = graph.orbs(s)
        c = int(graph.n_core_orbs[s])
        e, z = O.eigh(O.gather(H, orbs))
        dF = O.divided_differences(e, mu, kT)
        Mrows, _ = O.mu_response_rows(z, e, c, mu, kT)
        atoms, loc = _core_atom_orbitals(system, graph, s)
        m = len(atoms)
        b = np.array([Mrows[li, li].sum() for li in loc])
        a = np.zeros((m, m))
        sub_atoms = atom_of[orbs]
        for j, J in enumerate(atoms):
            gJ = np.zeros(system.n_atoms)
            gJ[col[rp[J]:rp[J + 1]]] = val[rp[J]:rp[J + 1]]  # gamma[., J] (symmetric)
            P, _ = O.lambda_response_rows(z, dF, np.diag(gJ[sub_atoms]), c)
            a[:, j] = [P[li, li].sum() for li in loc]
        mu1 = -a.sum(axis=0) / b.sum()
        j_c = a + np.outer(b, mu1) - np.eye(m)
        js.append(j_c)
        k0s.append(np.linalg.inv(j_c - alpha * np.eye(m)))
    return k0s, js


def apply_k0(system, graph, k0s, x):
    """K0 x (Eq. (PreCond)): each block acts on the core atoms of its
    subgraph; the cores partition the atoms."""
    y = np.zeros(system.n_atoms)
    for s in range(graph.n_sub):
        a0 = graph.sub_ptr[s]
        atoms = graph.sub_atoms[a0:a0 + graph.n_core_atoms[s]]
        y[atoms] = k0s[s] @ np.asarray(x)[atoms]
    return y


def krylov_kernel(system, graph, kT, gamma, k0s, n, m, omega=1.0):
    """Sec. V.B: the preconditioned low-rank Krylov approximation of the
    kernel acting on the residual (Eqs. (LowRankEEOM), (ElEOM)).

    1. f = rho_0[n] - n, v_1 = K0 f / |K0 f| (Eqs. (v1_prim), (v1));
    2.-3. for i = 1..m: the response of rho_0 along v_i, and
          f_{v_i} = K0 (d rho_0 / d lambda - v_i);
    4. v_{i+1} = f_{v_i} orthogonalised against v_1..v_i and normalised
       (modified Gram-Schmidt, two passes, so that the vectors stay
       orthonormal to rounding when the Krylov space nearly saturates);
    then O_ij = f_{v_i} . f_{v_j}, M = O^-1 and
    n'' = -omega^2 sum_ij v_i M_ij (f_{v_j} . K0 f)."""
    r0 = O.solve(system, graph, kT)
    q0 = core_charges(system, graph, r0.rho)
    res = q0 - np.asarray(n, dtype=np.float64)
    Kf = apply_k0(system, graph, k0s, res)
    V = [Kf / np.linalg.norm(Kf)]
    F = []
    for i in range(m):
        q1, _ = charge_response(system, graph, kT, gamma, V[i])
        F.append(apply_k0(system, graph, k0s, q1[0] - V[i]))
        if i + 1 < m:
            w = F[i].copy()
            for _ in range(2):
                for j in range(i + 1):
                    w = w - (w @ V[j]) * V[j]
            V.append(w / np.linalg.norm(w))
    V = np.array(V)
    F = np.array(F)
    Ov = F @ F.T
    Mm = np.linalg.inv(Ov)
    coef = Mm @ (F @ Kf)
    ndd = -omega ** 2 * (V.T @ coef)
    return {"mu": r0.mu, "q0": q0, "residual": res, "K0f": Kf, "V": V, "F": F, "O": Ov,
            "M": Mm, "ndd": ndd}
