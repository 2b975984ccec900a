"""The oracle's process-pool driver against its serial path.

`solve_pool` spreads the independent per-subgraph work (gather, eigensolve,
core rows, response rows) over worker processes and runs every sum that
couples subgraphs (the chemical potential of Sec. II.G, mu1 of Eq. (dmu_1))
in the parent, in ascending subgraph order.  Its results must therefore be
the serial `solve`'s bit for bit, for any number of workers: a subgraph dealt
to the wrong worker, recomputed eigenpairs that differ, a reduction summed in
another order or a response combined with the wrong mu1 all break equality.
The serial path is the one pinned by `test_oracle_pins.py`.
"""
import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

KT = 0.01


def _same(a, b):
    assert a.mu == b.mu, (a.mu, b.mu)
    for name in ("rho", "rho1", "mu1", "eps"):
        x, y = getattr(a, name), getattr(b, name)
        assert x.shape == y.shape, name
        assert np.array_equal(x, y), (name, float(np.abs(x - y).max()))


def _water32(O, tau, flags):
    s = I.water32_system()
    core = I.single_atom_cores(s)
    prev = O.bootstrap_prev(s, core, KT)
    g = O.graph_build(s, core, tau, rho_prev=prev, flags=flags)
    return s, g, I.h1_diagonal(s, 2, seed=1002)


@pytest.mark.parametrize("tau,flags", [(1e-5, 0), (0.07, 1), (1e-5, 2)],
                         ids=["tau1e-5", "paths2_tau0.07", "complete"])
def test_pool_equals_serial_water32(oracle_lib, tau, flags):
    O = oracle_lib
    s, g, h1 = _water32(O, tau, flags)
    ref = O.solve(s, g, KT, h1)
    for workers in (1, 3):
        _same(O.solve_pool(s, g, KT, h1, workers=workers), ref)


def test_pool_equals_serial_water60(oracle_lib):
    """8-atom spatial cores, paths of two, three perturbations; 1, 3 and 16
    workers (16 exceeds the 23 subgraphs' share per worker only for some)."""
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    g = O.graph_build(s, core, 0.07, rho_prev=prev, flags=O.PATHS2)
    h1 = I.h1_diagonal(s, 3, seed=62)
    ref = O.solve(s, g, KT, h1)
    for workers in (1, 3, 16):
        _same(O.solve_pool(s, g, KT, h1, workers=workers), ref)


def test_pool_equals_serial_chain_in_water(oracle_lib):
    """A 300-atom chain-in-water system: uneven subgraph sizes, so the
    size-ordered deal puts different counts on each worker."""
    O = oracle_lib
    s = I.chain_water_system(300, 60, seed=3011)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    g = O.graph_build(s, core, 0.07, rho_prev=prev, flags=O.PATHS2)
    assert g.sizes().min() < g.sizes().max()
    h1 = I.h1_diagonal(s, 2, seed=3012)
    ref = O.solve(s, g, KT, h1)
    _same(O.solve_pool(s, g, KT, h1, workers=5), ref)


def test_pool_bootstrap_equals_serial(oracle_lib):
    """The previous-step density the large tests and the stored 30,000-atom
    values start from: pool and serial give the same array."""
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    a = O.bootstrap_prev(s, core, KT, pool=False)
    b = O.bootstrap_prev(s, core, KT, pool=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
