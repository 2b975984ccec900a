"""Graph estimation and partition of the oracle against a dense brute force.

Sec. II.E: the graph is the thresholded density of a previous step together
with the thresholded Hamiltonian, optionally extended by paths of length two;
Sec. II.C / Fig. 1: a subgraph is a core plus every vertex joined to it.
The brute force below builds the same objects with dense boolean matrices.
"""
import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I


def brute_graph(system, core, tau, rho_dense=None, paths2=False, complete=False):
    aop = system.atom_orb_ptr
    na = system.n_atoms
    atom_of = np.repeat(np.arange(na), np.diff(aop))
    M = np.zeros((na, na), bool)
    mats = [system.dense_h()] + ([rho_dense] if rho_dense is not None else [])
    for X in mats:
        r, c = np.nonzero((np.abs(X) >= tau) & (X != 0))
        M[atom_of[r], atom_of[c]] = True
    M |= M.T
    np.fill_diagonal(M, False)
    if paths2:
        M = M | ((M.astype(int) @ M.astype(int)) > 0)
        np.fill_diagonal(M, False)
    n_sub = core.max() + 1
    subs = []
    for s in range(n_sub):
        cs = np.nonzero(core == s)[0]
        if complete:
            halo = np.setdiff1d(np.arange(na), cs)
        else:
            halo = np.setdiff1d(np.nonzero(M[cs].any(axis=0))[0], cs)
        atoms = np.concatenate([cs, halo])
        orbs = np.concatenate([np.arange(aop[a], aop[a + 1]) for a in atoms])
        nco = int(sum(aop[a + 1] - aop[a] for a in cs))
        subs.append((atoms, len(cs), orbs, nco))
    rows = []
    for a in range(system.n_orb):
        s = core[atom_of[a]]
        rows.append(np.sort(subs[s][2]))
    return subs, rows


def check_equal(g, subs, rows):
    assert g.n_sub == len(subs)
    for s, (atoms, nca, orbs, nco) in enumerate(subs):
        assert np.array_equal(g.sub_atoms[g.sub_ptr[s]:g.sub_ptr[s + 1]], atoms)
        assert g.n_core_atoms[s] == nca
        assert np.array_equal(g.orbs(s), orbs)
        assert g.n_core_orbs[s] == nco
    for a, cols in enumerate(rows):
        assert np.array_equal(g.rho_col[g.rho_row_ptr[a]:g.rho_row_ptr[a + 1]], cols)


@pytest.fixture(scope="module")
def cfg1():
    return I.water32_system()


@pytest.fixture(scope="module")
def cfg1_rho(cfg1, oracle_lib):
    O = oracle_lib
    g = O.graph_build(cfg1, I.single_atom_cores(cfg1), 0.0)
    r = O.solve(cfg1, g, 0.01)
    rows = np.repeat(np.arange(g.n_orb), np.diff(g.rho_row_ptr))
    D = np.zeros((cfg1.n_orb, cfg1.n_orb))
    D[rows, g.rho_col] = r.rho
    return (g.rho_row_ptr, g.rho_col, r.rho), D


@pytest.mark.parametrize("tau,paths2,complete,cores", [
    (1e-2, False, False, 1), (3e-2, False, False, 1), (2e-2, True, False, 1),
    (1e-3, False, False, 3), (5e-2, False, True, 3), (3e-2, False, False, 8),
])
def test_graph_against_bruteforce(oracle_lib, cfg1, cfg1_rho, tau, paths2, complete, cores):
    O = oracle_lib
    core = (I.single_atom_cores(cfg1) if cores == 1 else
            I.spatial_cores(cfg1, cores))
    prev, D = cfg1_rho
    flags = (O.PATHS2 if paths2 else 0) | (O.COMPLETE if complete else 0)
    g = O.graph_build(cfg1, core, tau, rho_prev=prev, flags=flags)
    subs, rows = brute_graph(cfg1, core, tau, D, paths2, complete)
    check_equal(g, subs, rows)
    assert g.nnz == sum(len(r) for r in rows)


def test_graph_without_density(oracle_lib):
    O = oracle_lib
    s = I.water_system(20, 9.0, seed=99)
    core = I.spatial_cores(s, 4)
    g = O.graph_build(s, core, 0.03)
    subs, rows = brute_graph(s, core, 0.03)
    check_equal(g, subs, rows)


def test_spatial_cores_are_dense_and_compact():
    s = I.water1000_system()
    core = I.spatial_cores(s, 8)
    counts = np.bincount(core)
    assert counts.min() == 8 and counts.max() == 8 and len(counts) == 375


def test_graph_errors(oracle_lib, cfg1):
    O = oracle_lib
    core = I.single_atom_cores(cfg1)
    with pytest.raises(O.OracleError, match="tau"):
        O.graph_build(cfg1, core, -1.0)
    bad = core.copy()
    bad[bad == 5] = 200
    with pytest.raises(O.OracleError, match="dense"):
        O.graph_build(cfg1, bad, 1e-2)
    import copy
    s = copy.copy(cfg1)
    # drop one off-diagonal entry: the pattern is no longer symmetric
    rp = s.h_row_ptr.copy()
    col = np.delete(s.h_col, 1)
    val = np.delete(s.h_val, 1)
    rp[1:] -= 1
    s.h_row_ptr, s.h_col, s.h_val = rp, col, val
    with pytest.raises(O.OracleError, match="symmetric"):
        O.graph_build(s, core, 1e-2)
    s2 = copy.copy(cfg1)
    aop = s2.atom_orb_ptr.copy()
    aop[3] = aop[2]
    s2.atom_orb_ptr = aop
    with pytest.raises(O.OracleError, match="increasing"):
        O.graph_build(s2, core, 1e-2)
