"""The C-ABI boundary without a GPU: the library loads, exports every symbol
include/gq.h declares, and its host-side graph_build agrees bit for bit with
the oracle's (integer work).  No device computation runs here."""
import os
import re

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gq():
    from paper_2212_01997_amd import gq as G
    if not os.path.exists(G.LIB_PATH):
        from paper_2212_01997_amd import build
        build.build()
    G.lib()
    return G


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "gq.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gq_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(gq):
    import ctypes
    L = ctypes.CDLL(gq.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(gq._SIGS)
    assert b"gfx950" in gq.lib().gq_version()


def _compare_graph(G, O, system, core, tau, prev=None, flags=0):
    g_or = O.graph_build(system, core, tau, rho_prev=prev, flags=flags)
    g_gq = G.Graph.for_system(system, core, tau, rho_prev=prev, flags=flags)
    ex = g_gq.export()
    for name in ("sub_ptr", "sub_atoms", "n_core_atoms", "sub_orb_ptr", "sub_orbs",
                 "n_core_orbs", "rho_row_ptr", "rho_col"):
        assert np.array_equal(ex[name], getattr(g_or, name)), name
    info = g_gq.info
    sizes = np.diff(ex["sub_orb_ptr"])
    assert info.n_sub == g_or.n_sub and info.nnz == g_or.nnz
    assert info.max_n == sizes.max() and info.min_n == sizes.min()
    assert info.sum_n2 == int((sizes.astype(np.int64) ** 2).sum())
    off = g_gq.block_offsets()
    assert off[-1] == info.nnz
    assert np.array_equal(np.diff(off), ex["n_core_orbs"].astype(np.int64) * sizes)


@pytest.mark.parametrize("tau,flags,cores", [(1e-5, 0, 1), (0.07, 1, 1), (0.0, 2, 1),
                                             (0.02, 0, 8), (0.07, 1, 8), (0.2, 1, 1),
                                             (0.15, 1, 3), (0.3, 1, 1)])
def test_graph_build_matches_oracle(gq, oracle_lib, tau, flags, cores):
    O = oracle_lib
    s = I.water32_system()
    core = I.single_atom_cores(s) if cores == 1 else I.spatial_cores(s, cores)
    prev = O.bootstrap_prev(s, core, 0.01)
    _compare_graph(gq, O, s, core, tau, prev, flags)


def test_graph_build_matches_oracle_chain(gq, oracle_lib):
    """Mixed elements (4-orbital heavy atoms), sparse thresholds, paths of two:
    the many-threaded host build against the oracle."""
    O = oracle_lib
    s = I.chain_water_system(900, 180, seed=3001)
    for cores, tau in ((1, 0.2), (8, 0.07), (3, 0.12)):
        core = I.single_atom_cores(s) if cores == 1 else I.spatial_cores(s, cores)
        g0 = O.graph_build(s, core, 0.0)
        prev = (g0.rho_row_ptr, g0.rho_col, np.linspace(0.5, 1e-4, g0.nnz))
        _compare_graph(gq, O, s, core, tau, prev, 1)


def test_graph_build_matches_oracle_water1000(gq, oracle_lib):
    O = oracle_lib
    s = I.water1000_system()
    core = I.spatial_cores(s, 8)
    g0 = O.graph_build(s, core, 0.0)
    # any previous density pattern exercises the threshold; use |H| scaled
    prev = (g0.rho_row_ptr, g0.rho_col, np.linspace(1.0, 1e-4, g0.nnz))
    _compare_graph(gq, O, s, core, 0.07, prev, 1)


def test_graph_build_errors(gq):
    s = I.water32_system()
    core = I.single_atom_cores(s)
    H = (s.h_row_ptr, s.h_col, s.h_val)
    with pytest.raises(gq.GQError, match="EINVAL.*tau"):
        gq.Graph(s.n_atoms, s.atom_orb_ptr, H, core, -1.0)
    bad = core.copy()
    bad[bad == 3] = 500
    with pytest.raises(gq.GQError, match="dense"):
        gq.Graph(s.n_atoms, s.atom_orb_ptr, H, bad, 0.01)
    rp = s.h_row_ptr.copy()
    rp[1:] -= 1
    with pytest.raises(gq.GQError, match="symmetric"):
        gq.Graph(s.n_atoms, s.atom_orb_ptr, (rp, np.delete(s.h_col, 1), np.delete(s.h_val, 1)),
                 core, 0.01)
    aop = s.atom_orb_ptr.copy()
    aop[3] = aop[2]
    with pytest.raises(gq.GQError, match="increasing"):
        gq.Graph(s.n_atoms, aop, H, core, 0.01)
    with pytest.raises(gq.GQError, match="flags"):
        gq.Graph(s.n_atoms, s.atom_orb_ptr, H, core, 0.01, flags=8)
    # an empty system has no subgraph to solve
    with pytest.raises(gq.GQError, match="empty system"):
        gq.Graph(0, np.zeros(1, np.int32),
                 (np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0)),
                 np.zeros(0, np.int32), 0.01)


def test_footprint_counts_buffers(gq):
    s = I.water32_system()
    g = gq.Graph.for_system(s, I.single_atom_cores(s), 0.0, flags=gq.COMPLETE)
    i = g.info
    f1, f6 = g.footprint(1), g.footprint(6)
    assert f1 >= 3 * i.sum_n2 * 8 + 2 * i.nnz * 8
    assert f6 > f1
