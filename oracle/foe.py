"""Reference oracle for the zero-temperature subgraph density of the
recursive Fermi-operator expansion (arXiv:2212.01997, Sec. II.D, Eqs. (Step),
(Recur), (dCollect)).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite and the CPU-baseline
leg of the benchmark; the GPU library neither imports nor links it.

The recursion of Eq. (Recur) converges to the Heaviside step function of the
subgraph matrix, Eq. (Step), which has a plain definition: in the eigenbasis
of h^(i), occupation 1 for eigenvalues below mu and 0 above.  This module is
that definition written out on top of the pinned C eigensolve (oracle.py);
how the limit is reached (the purification polynomials) does not enter.  An
eigenvalue equal to mu has no defined step: the functions raise.

Spin: the core rows carry the factor 2 of the doubly occupied orbitals, as the
finite-temperature rows of oracle.py do.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def step_rows(h, c, mu):
    """2 Theta(mu I - h)[0:c, :] for one dense symmetric subgraph matrix h."""
    w, z = O.eigh(h)
    if np.any(w == mu):
        raise ValueError("an eigenvalue equals mu: the step function is not defined there")
    occ = (w < mu).astype(np.float64)
    return 2.0 * (z[:c] * occ) @ z.T


def purified_density(system, graph, mu):
    """Eq. (dCollect): the collected core rows of every subgraph's step
    density.  Returns (values on the graph's pattern [nnz], the smallest
    distance of a subgraph eigenvalue to mu)."""
    H = O.Csr(system.h_row_ptr, system.h_col, system.h_val)
    rho = np.zeros(graph.nnz)
    gap = np.inf
    for s in range(graph.n_sub):
        h = O.gather(H, graph.orbs(s))
        c = int(graph.n_core_orbs[s])
        w, _ = O.eigh(h)
        gap = min(gap, float(np.abs(w - mu).min()))
        O.collect(graph, s, step_rows(h, c, mu), rho)
    return rho, gap


def mid_gap(eps, mu):
    """The midpoint between the subgraph eigenvalues (all subgraphs together)
    just below and just above mu: a chemical potential with no eigenvalue
    nearer than half that gap."""
    e = np.asarray(eps, dtype=np.float64)
    return 0.5 * (e[e < mu].max() + e[e > mu].min())
