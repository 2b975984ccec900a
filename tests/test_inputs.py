"""The seeded input generator: geometry constraints and Hamiltonian shape."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2212_01997_amd import inputs as I


def _min_image_pairs(pos, box, r):
    t = cKDTree(np.mod(pos, box), boxsize=box)
    p = t.query_pairs(r, output_type="ndarray")
    d = pos[p[:, 0]] - pos[p[:, 1]]
    d -= box * np.round(d / box)
    return p, np.sqrt((d * d).sum(axis=1))


@pytest.mark.parametrize("make", [lambda: I.water32_system(), lambda: I.water1000_system(),
                                  lambda: I.chain_water_system(900, 180, seed=3001)])
def test_geometry_constraints(make):
    s = make()
    sp = np.array(s.species)
    mol = np.full(s.n_atoms, -1)
    nch = s.meta.get("n_chain", 0)
    mol[nch:] = np.arange(s.n_atoms - nch) // 3
    p, r = _min_image_pairs(s.pos, s.box, 2.5)
    a, b = p[:, 0], p[:, 1]
    inter = (mol[a] != mol[b]) | (mol[a] < 0)
    chain_bond = (mol[a] < 0) & (mol[b] < 0) & (np.abs(a - b) == 1)
    assert r[inter & ~chain_bond].min() >= 1.5 - 1e-9
    oo = (sp[a] == "O") & (sp[b] == "O") & (mol[a] >= 0) & (mol[b] >= 0)
    if oo.any():
        assert r[oo].min() >= 2.5 - 1e-9


def test_hamiltonian_shape():
    s = I.water32_system()
    H = s.dense_h()
    assert np.array_equal(H, H.T)
    assert s.n_orb == 192 and s.n_elec == 256
    off = H[~np.eye(s.n_orb, dtype=bool)]
    nz = off[off != 0]
    assert nz.max() < 0 and nz.min() >= -0.5 and nz.max() <= -0.5 * np.exp(-4.0 / 1.2) + 1e-15
    assert set(np.round(np.diag(H), 2)) == {-0.87, -0.33, -0.24}


def test_chain30000_shape():
    s = I.chain30000_system()
    assert s.n_atoms == 30000 and s.n_orb == 72000
    assert abs(s.box - (30000 / 0.1) ** (1 / 3)) < 1e-9
    assert s.n_elec % 2 == 0


def test_h1_per_atom_shift():
    s = I.water32_system()
    h1 = I.h1_diagonal(s, 3, seed=4)
    assert h1.shape == (3, s.n_orb)
    for I_ in range(s.n_atoms):
        blk = h1[:, s.atom_orb_ptr[I_]:s.atom_orb_ptr[I_ + 1]]
        assert np.all(blk == blk[:, :1])
