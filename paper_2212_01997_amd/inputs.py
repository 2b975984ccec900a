"""Seeded synthetic systems for the graph-based density / response path.

This module only builds inputs: geometries, the orthogonal tight-binding
Hamiltonian H (CSR), diagonal perturbations H1, core partitions and electron
counts.  It contains none of the method's arithmetic (no eigensolve, no Fermi
function, no graph construction) and is shared by the oracle-side tests and
the GPU-side tests and benchmark.

The paper's own workloads are SCC-DFTB water, ammonium-hydroxide and solvated
Trp-cage structures (Sec. VI); those structures and parameter sets are not
available, so seeded synthetic stand-ins with the same shape are generated
here:

* water boxes: rigid molecules (O-H 0.96 A, H-O-H 104.5 deg), random
  orientation, random sequential addition with O-O >= 2.5 A and every
  intermolecular atom pair >= 1.5 A (minimum image);
* a chain of C/N/O/S heavy atoms (1.5 A steps, self-avoiding random walk)
  embedded in such water at 0.1 atoms / A^3.

Hamiltonian (Hartree, Angstrom): on-site energies are diagonal per orbital;
every orbital pair on two distinct atoms closer than 4 A (minimum image)
couples with -0.5 exp(-r/1.2).  There is no angular dependence.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
from scipy.spatial import cKDTree

# orbitals per element and their on-site energies (Ha): s first, then p
ORBITALS = {
    "H": (-0.24,),
    "O": (-0.87, -0.33, -0.33, -0.33),
    "C": (-0.50, -0.19, -0.19, -0.19),
    "N": (-0.68, -0.26, -0.26, -0.26),
    "S": (-0.63, -0.26, -0.26, -0.26),
}
VALENCE = {"H": 1, "O": 6, "C": 4, "N": 5, "S": 6}

HOP_PREFACTOR = -0.5
HOP_DECAY = 1.2
HOP_CUTOFF = 4.0

OH_BOND = 0.96
HOH_ANGLE = math.radians(104.5)


@dataclass
class System:
    """A synthetic orthogonal tight-binding system.

    H is stored as CSR with ascending column indices in every row; the
    pattern is symmetric and contains the diagonal.
    """
    name: str
    box: float
    pos: np.ndarray            # [n_atoms, 3] float64
    species: list              # [n_atoms] element symbols
    atom_orb_ptr: np.ndarray   # [n_atoms + 1] int32
    h_row_ptr: np.ndarray      # [N + 1] int32
    h_col: np.ndarray          # [nnz] int32
    h_val: np.ndarray          # [nnz] float64
    n_elec: float
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return len(self.species)

    @property
    def n_orb(self) -> int:
        return int(self.atom_orb_ptr[-1])

    def dense_h(self) -> np.ndarray:
        n = self.n_orb
        out = np.zeros((n, n))
        rows = np.repeat(np.arange(n), np.diff(self.h_row_ptr))
        out[rows, self.h_col] = self.h_val
        return out


# ---------------------------------------------------------------- geometry

def _random_rotations(rng, count):
    """Uniform random rotation matrices from unit quaternions."""
    q = rng.normal(size=(count, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    r = np.empty((count, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def _water_template():
    half = HOH_ANGLE / 2
    return np.array([
        [0.0, 0.0, 0.0],
        [OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0],
        [-OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0],
    ])


class _Grid:
    """Cell list under periodic boundaries for incremental insertion."""

    def __init__(self, box, cell):
        self.box = box
        self.nc = max(1, int(box // cell))
        self.cell = box / self.nc
        self.cells = {}
        self.pos = []
        self.tag = []

    def _key(self, p):
        c = np.floor(np.mod(p, self.box) / self.cell).astype(int) % self.nc
        return tuple(c)

    def add(self, p, tag):
        idx = len(self.pos)
        self.pos.append(np.asarray(p, dtype=float))
        self.tag.append(tag)
        self.cells.setdefault(self._key(p), []).append(idx)

    def near(self, p):
        """Indices of stored points in the 27 cells around p."""
        cx, cy, cz = self._key(p)
        out = []
        rng = (-1, 0, 1) if self.nc >= 3 else range(-(self.nc // 2), self.nc - self.nc // 2)
        seen = set()
        for dx in rng:
            for dy in rng:
                for dz in rng:
                    k = ((cx + dx) % self.nc, (cy + dy) % self.nc, (cz + dz) % self.nc)
                    if k in seen:
                        continue
                    seen.add(k)
                    out.extend(self.cells.get(k, ()))
        return out

    def min_dist(self, p, idx, tag_filter=None):
        if not idx:
            return np.inf
        pts = np.array([self.pos[i] for i in idx])
        d = pts - p
        d -= self.box * np.round(d / self.box)
        r = np.sqrt((d * d).sum(axis=1))
        if tag_filter is not None:
            mask = np.array([tag_filter(self.tag[i]) for i in idx])
            if not mask.any():
                return np.inf
            r = r[mask]
        return r.min()


def place_waters(rng, n_mol, box, fixed=None, oo_min=2.5, inter_min=1.5, batch=2048,
                 max_rounds=4000):
    """Random sequential addition of rigid waters into a periodic box, in
    batches: every candidate keeps `inter_min` from all placed atoms (waters
    and the `fixed` foreign atoms) and its O keeps `oo_min` from placed
    oxygens; conflicts inside a batch are resolved greedily in candidate
    order.  Returns an [n_mol*3, 3] array in O, H, H order per molecule."""
    tmpl = _water_template()
    placed = np.zeros((0, 3)) if fixed is None else np.mod(np.asarray(fixed, float), box)
    oxy = np.zeros((0, 3))
    out = []
    n_done = 0
    rounds = 0
    while n_done < n_mol:
        rounds += 1
        if rounds > max_rounds:
            raise RuntimeError(f"water placement stalled ({n_done}/{n_mol} placed)")
        centers = rng.uniform(0.0, box, size=(batch, 3))
        rots = _random_rotations(rng, batch)
        mol = np.mod(centers[:, None, :] + np.einsum("aj,bij->bai", tmpl, rots), box)  # [B,3,3]
        ok = np.ones(batch, bool)
        if len(placed):
            t_all = cKDTree(placed, boxsize=box)
            d, _ = t_all.query(mol.reshape(-1, 3), k=1)
            ok &= (d.reshape(batch, 3) >= inter_min).all(axis=1)
        if len(oxy):
            t_o = cKDTree(oxy, boxsize=box)
            d, _ = t_o.query(mol[:, 0, :], k=1)
            ok &= d >= oo_min
        idx = np.nonzero(ok)[0]
        if len(idx) == 0:
            continue
        cand = mol[idx]
        flat = cand.reshape(-1, 3)
        tree = cKDTree(flat, boxsize=box)
        pairs = tree.query_pairs(max(oo_min, inter_min), output_type="ndarray")
        conflict = [[] for _ in range(len(idx))]
        if len(pairs):
            a, b = pairs[:, 0], pairs[:, 1]
            ma, mb = a // 3, b // 3
            dv = flat[a] - flat[b]
            dv -= box * np.round(dv / box)
            r = np.sqrt((dv * dv).sum(axis=1))
            both_o = (a % 3 == 0) & (b % 3 == 0)
            bad = (ma != mb) & ((r < inter_min) | (both_o & (r < oo_min)))
            for x, y in zip(ma[bad], mb[bad]):
                conflict[max(x, y)].append(min(x, y))
        taken = np.zeros(len(idx), bool)
        for m in range(len(idx)):
            if n_done >= n_mol:
                break
            if any(taken[o] for o in conflict[m]):
                continue
            taken[m] = True
            out.append(cand[m])
            n_done += 1
        acc = cand[taken]
        placed = np.concatenate([placed, acc.reshape(-1, 3)])
        oxy = np.concatenate([oxy, acc[:, 0, :]])
    return np.concatenate(out, axis=0) if out else np.zeros((0, 3))


def chain_walk(rng, n_chain, box, step=1.5, min_sep=2.4, retries=100, max_fails=4):
    """Self-avoiding random walk of heavy atoms under periodic boundaries.

    Every new atom keeps `min_sep` from all chain atoms except its
    predecessor; after `retries` failed directions the walk backtracks.
    """
    grid = _Grid(box, min_sep)
    pts = [rng.uniform(0.0, box, size=3)]
    grid.add(pts[0], 0)
    fails = [0]
    while len(pts) < n_chain:
        prev = pts[-1]
        placed = False
        for _ in range(retries):
            d = rng.normal(size=3)
            d *= step / np.linalg.norm(d)
            cand = np.mod(prev + d, box)
            idx = [i for i in grid.near(cand) if grid.tag[i] != len(pts) - 1]
            if grid.min_dist(cand, idx) >= min_sep:
                pts.append(cand)
                grid.add(cand, len(pts) - 1)
                fails.append(0)
                placed = True
                break
        if not placed:
            # backtrack one atom; an atom whose continuation failed more than
            # `max_fails` times is itself taken back (escapes dead ends)
            while True:
                if len(pts) <= 1:
                    raise RuntimeError("chain walk stuck at the first atom")
                last = len(pts) - 1
                key = grid._key(pts[last])
                grid.cells[key].remove(last)
                grid.pos.pop()
                grid.tag.pop()
                pts.pop()
                fails.pop()
                fails[-1] += 1
                if fails[-1] <= max_fails:
                    break
                fails[-1] = 0
    return np.array(pts)


# ------------------------------------------------------------- Hamiltonian

def build_hamiltonian(pos, species, box, cutoff=HOP_CUTOFF):
    """Orthogonal tight-binding H as CSR (sorted columns, symmetric pattern)."""
    n_atoms = len(species)
    norb = np.array([len(ORBITALS[s]) for s in species], dtype=np.int64)
    atom_orb_ptr = np.zeros(n_atoms + 1, dtype=np.int64)
    np.cumsum(norb, out=atom_orb_ptr[1:])
    n = int(atom_orb_ptr[-1])
    if box < 2 * cutoff:
        raise ValueError("box must be at least twice the hopping cutoff")

    tree = cKDTree(np.mod(pos, box), boxsize=box)
    pairs = tree.query_pairs(cutoff, output_type="ndarray")
    ii, jj = pairs[:, 0], pairs[:, 1]
    d = pos[ii] - pos[jj]
    d -= box * np.round(d / box)
    r = np.sqrt((d * d).sum(axis=1))
    hop = HOP_PREFACTOR * np.exp(-r / HOP_DECAY)

    rows, cols, vals = [], [], []
    # off-diagonal blocks, both orientations
    for a_idx, b_idx in ((ii, jj), (jj, ii)):
        na = norb[a_idx]
        nb = norb[b_idx]
        cnt = na * nb
        pair_of = np.repeat(np.arange(len(a_idx)), cnt)
        start = np.zeros(len(a_idx) + 1, dtype=np.int64)
        np.cumsum(cnt, out=start[1:])
        local = np.arange(int(start[-1])) - start[pair_of]
        nb_rep = nb[pair_of]
        rows.append(atom_orb_ptr[a_idx][pair_of] + local // nb_rep)
        cols.append(atom_orb_ptr[b_idx][pair_of] + local % nb_rep)
        vals.append(hop[pair_of])
    onsite = np.concatenate([np.array(ORBITALS[s]) for s in species])
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(onsite)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    np.cumsum(row_ptr, out=row_ptr)
    return (atom_orb_ptr.astype(np.int32), row_ptr.astype(np.int32),
            cols.astype(np.int32), vals.astype(np.float64))


def electron_count(species, n_water=None):
    """Valence electrons; one more is added if the total is odd."""
    ne = sum(VALENCE[s] for s in species)
    if ne % 2:
        ne += 1
    return float(ne)


def make_system(name, box, pos, species, meta):
    aop, rp, col, val = build_hamiltonian(pos, species, box)
    return System(name=name, box=float(box), pos=np.asarray(pos, dtype=np.float64),
                  species=list(species), atom_orb_ptr=aop, h_row_ptr=rp,
                  h_col=col, h_val=val, n_elec=electron_count(species), meta=meta)


def water_system(n_mol, box, seed, name=None):
    rng = np.random.default_rng(seed)
    pos = place_waters(rng, n_mol, box)
    species = ["O", "H", "H"] * n_mol
    return make_system(name or f"water{n_mol}", box, pos, species,
                        {"kind": "water", "n_mol": n_mol, "seed": seed})


CHAIN_MIX = (("C", 0.62), ("N", 0.17), ("O", 0.20), ("S", 0.01))


def chain_water_system(n_atoms, n_chain, seed, density=0.1, name=None):
    """Heavy-atom chain embedded in water at `density` atoms / A^3."""
    rng = np.random.default_rng(seed)
    box = (n_atoms / density) ** (1.0 / 3.0)
    chain = chain_walk(rng, n_chain, box)
    elems = [e for e, _ in CHAIN_MIX]
    probs = np.array([p for _, p in CHAIN_MIX])
    chain_species = list(rng.choice(elems, size=n_chain, p=probs / probs.sum()))
    n_mol = (n_atoms - n_chain) // 3
    water = place_waters(rng, n_mol, box, fixed=chain)
    pos = np.concatenate([chain, water], axis=0)
    species = chain_species + ["O", "H", "H"] * n_mol
    return make_system(name or f"chain{n_chain}_water{n_mol}", box, pos, species,
                        {"kind": "chain+water", "n_chain": n_chain, "n_mol": n_mol,
                         "seed": seed})


def h_lattice_system(shape=(16, 16, 8), spacing=(1.5, 1.5, 3.0), box=24.0, jitter=0.15,
                     seed=2048):
    """Hydrogen atoms on a rectangular lattice (one s orbital each) in a cubic
    periodic box, each moved by up to `jitter` A per axis: a system whose
    complete-graph subgraphs have exactly prod(shape) orbitals."""
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(*[np.arange(k) for k in shape], indexing="ij"),
                 axis=-1).reshape(-1, 3).astype(np.float64)
    pos = g * np.asarray(spacing) + 0.5 + rng.uniform(-jitter, jitter, size=g.shape)
    return make_system(f"hlattice{len(pos)}", box, pos, ["H"] * len(pos),
                       {"kind": "h_lattice", "shape": list(shape), "seed": seed})


def isolated_molecules_system(n_mol, spacing, seed):
    """Waters on a cubic lattice `spacing` apart: H is block diagonal when
    spacing - 2 A > 4 A (used to check the disconnected case)."""
    rng = np.random.default_rng(seed)
    m = int(math.ceil(n_mol ** (1.0 / 3.0)))
    box = m * spacing
    tmpl = _water_template()
    rots = _random_rotations(rng, n_mol)
    pos = []
    k = 0
    for ix in range(m):
        for iy in range(m):
            for iz in range(m):
                if k == n_mol:
                    break
                c = np.array([ix, iy, iz], dtype=float) * spacing + spacing / 2
                pos.append(c + tmpl @ rots[k].T)
                k += 1
    pos = np.mod(np.concatenate(pos, axis=0), box)
    species = ["O", "H", "H"] * n_mol
    return make_system(f"isolated{n_mol}", box, pos, species,
                        {"kind": "isolated", "n_mol": n_mol, "seed": seed})


# ---------------------------------------------------------- perturbations

def h1_diagonal(system, k, seed, sigma=0.05):
    """K diagonal perturbations: one N(0, sigma) shift per atom, applied to
    every orbital of that atom.  Returns float64 [K, N]."""
    rng = np.random.default_rng(seed)
    shifts = rng.normal(0.0, sigma, size=(k, system.n_atoms))
    norb = np.diff(system.atom_orb_ptr)
    return np.repeat(shifts, norb, axis=1).astype(np.float64)


def h1_on_pattern(system, k, seed, sigma=0.05):
    """K symmetric perturbations on the sparsity pattern of H (every stored
    entry of H, diagonal included, gets an N(0, sigma) value; entry (b, a)
    mirrors (a, b)).  Returns a list of K host CSR triples (row_ptr, col, val)."""
    rng = np.random.default_rng(seed)
    n = system.n_orb
    rows = np.repeat(np.arange(n), np.diff(system.h_row_ptr))
    col = system.h_col
    out = []
    for _ in range(k):
        dense = np.zeros((n, n))
        dense[rows, col] = rng.normal(0.0, sigma, size=len(col))
        dense = np.triu(dense) + np.triu(dense, 1).T
        out.append((system.h_row_ptr.copy(), col.copy(), dense[rows, col].copy()))
    return out


def h1_dense(system, k, seed, sigma=0.05):
    """K fully dense symmetric N x N perturbations with N(0, sigma) entries,
    as host CSR triples with every entry stored."""
    rng = np.random.default_rng(seed)
    n = system.n_orb
    out = []
    for _ in range(k):
        a = rng.normal(0.0, sigma, size=(n, n))
        a = np.triu(a) + np.triu(a, 1).T
        out.append((np.arange(0, n * n + 1, n, dtype=np.int32),
                    np.tile(np.arange(n, dtype=np.int32), n), a.ravel().copy()))
    return out


# ------------------------------------------------- overlap (non-orthogonal basis)
def overlap_matrix(system, decay=0.6, min_eig=0.3):
    """A synthetic overlap S for a non-orthogonal basis on the pattern of H:
    unit diagonal, zero between distinct orbitals of one atom, and between
    orbitals of atoms at distance r (< 4 A) a value t exp(-r/decay), with
    t = (1 - min_eig) / (largest off-diagonal row sum), so that Gershgorin
    bounds every eigenvalue of S (and of every principal submatrix) below by
    min_eig: S is symmetric positive definite.  r is recovered from the hopping
    -0.5 exp(-r/1.2) stored in H.  Returns a host CSR triple."""
    n = system.n_orb
    rows = np.repeat(np.arange(n), np.diff(system.h_row_ptr))
    off = rows != system.h_col
    v = np.zeros(len(system.h_col))
    v[off] = (system.h_val[off] / HOP_PREFACTOR) ** (HOP_DECAY / decay)
    t = (1.0 - min_eig) / np.bincount(rows, weights=v, minlength=n).max()
    val = t * v
    val[~off] = 1.0
    return system.h_row_ptr.copy(), system.h_col.copy(), val


# ------------------------------------------------- charge model (Sec. V)
# A stand-in for the charge-dependent potential of SCC-DFTB: atomic charges n
# act on every orbital of atom I through the potential (gamma n)_I, so the
# perturbation from a charge vector v is H1[v] = diag over orbitals of
# (gamma v).  gamma_II = U_I (on-site interaction per element, Ha), and for
# I != J within the cutoff (minimum image) a screened Coulomb form
# exp(-r/s) / sqrt(r^2 + (2/(U_I + U_J))^2) with r and s in bohr.  The values
# are chosen here (free-atom-like magnitudes), not taken from a parameter
# set.
HUBBARD_U = {"H": 0.42, "C": 0.36, "N": 0.43, "O": 0.50, "S": 0.33}
BOHR = 0.529177210903  # Angstrom per bohr
COULOMB_SCREEN = 6.0   # bohr
COULOMB_CUTOFF = 8.0   # Angstrom (at most half the box)


def coulomb_kernel(system, cutoff=COULOMB_CUTOFF):
    """Symmetric atom-by-atom kernel gamma as a host CSR triple (row_ptr, col,
    val), ascending columns, diagonal included."""
    n = system.n_atoms
    cut = min(cutoff, 0.5 * system.box - 1e-9)
    U = np.array([HUBBARD_U[s] for s in system.species])
    pos = np.mod(system.pos, system.box)
    tree = cKDTree(pos, boxsize=system.box)
    pairs = tree.query_pairs(cut, output_type="ndarray")
    ii, jj = pairs[:, 0], pairs[:, 1]
    d = pos[ii] - pos[jj]
    d -= system.box * np.round(d / system.box)
    r = np.sqrt((d * d).sum(axis=1)) / BOHR
    a = 2.0 / (U[ii] + U[jj])
    g = np.exp(-r / COULOMB_SCREEN) / np.sqrt(r * r + a * a)
    rows = np.concatenate([ii, jj, np.arange(n)])
    cols = np.concatenate([jj, ii, np.arange(n)])
    vals = np.concatenate([g, g, U])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    np.cumsum(rp, out=rp)
    return rp.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64)


def charge_vectors(system, k, seed, sigma=0.05):
    """K seeded charge vectors over the atoms, N(0, sigma) per atom."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, sigma, size=(k, system.n_atoms))


# -------------------------------------------------------------- partitions

def single_atom_cores(system):
    return np.arange(system.n_atoms, dtype=np.int32)


def _spread_bits(v):
    v = v.astype(np.uint64) & np.uint64(0x3FF)
    out = np.zeros_like(v)
    for b in range(10):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def spatial_cores(system, core_size):
    """Morton (Z-order) sort of positions quantised to box/1024, ties broken
    by atom index, cut into consecutive chunks of `core_size` atoms."""
    q = np.floor(np.mod(system.pos, system.box) / system.box * 1024.0).astype(np.int64)
    q = np.clip(q, 0, 1023)
    key = (_spread_bits(q[:, 0]) | (_spread_bits(q[:, 1]) << np.uint64(1))
           | (_spread_bits(q[:, 2]) << np.uint64(2)))
    order = np.lexsort((np.arange(system.n_atoms), key))
    core = np.empty(system.n_atoms, dtype=np.int32)
    core[order] = (np.arange(system.n_atoms) // core_size).astype(np.int32)
    return core


# ------------------------------------------------------------ the benchmark systems

def water32_system(seed=1001):
    """32 waters in a 10 A box (96 atoms, 192 orbitals, N_e = 256)."""
    return water_system(32, 10.0, seed, name="water32")


def water1000_system(seed=2001):
    """1,000 waters in a 31 A box (3,000 atoms, 6,000 orbitals)."""
    return water_system(1000, 31.0, seed, name="water1000")


def chain30000_system(seed=3001):
    """A 6,000-atom C/N/O/S chain in water: 30,000 atoms at 0.1 atoms / A^3."""
    return chain_water_system(30000, 6000, seed, name="chain30000")


@dataclass
class ServingTrace:
    """Arrival-ordered requests: request j asks for system `system[j]` of the
    pool with `K[j]` perturbations drawn from seed `h1_seed[j]`."""
    arrival: np.ndarray        # [n] seconds
    system: np.ndarray         # [n] index into `pool`
    K: np.ndarray              # [n]
    h1_seed: np.ndarray        # [n]
    pool: list                 # [(kind, n_atoms, seed)]


def serving_trace(n_requests=200, rate=20.0, n_systems=24, lo=500, hi=20000, seed=5001):
    """Poisson arrivals at `rate` per second; system sizes log-uniform over
    [lo, hi] atoms, water or chain-in-water with probability 1/2 (chain = 20%
    of the atoms); K uniform over 1..8.  The requests draw their systems from
    a pool of `n_systems` seeded systems (each request its own perturbations)."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), n_systems))
    kinds = rng.random(n_systems) < 0.5
    pool = []
    for i in range(n_systems):
        n = int(round(sizes[i] / 3.0)) * 3
        pool.append(("chain" if kinds[i] else "water", n, seed * 100 + i))
    gaps = rng.exponential(1.0 / rate, n_requests)
    return ServingTrace(arrival=np.cumsum(gaps) - gaps[0],
                        system=rng.integers(0, n_systems, n_requests),
                        K=rng.integers(1, 9, n_requests),
                        h1_seed=seed * 1000 + np.arange(n_requests), pool=pool)


WATER_DENSITY = 1000 / 31.0 ** 3  # molecules per cubic angstrom of the 1,000-water box


def pool_system(kind, n_atoms, seed):
    """A serving-pool system: n_atoms/3 waters at the 1,000-water box density,
    or a chain of 20% of the atoms in water at 0.1 atoms per cubic angstrom."""
    if kind == "water":
        n_mol = n_atoms // 3
        return water_system(n_mol, (n_mol / WATER_DENSITY) ** (1.0 / 3.0), seed)
    return chain_water_system(n_atoms, max(2, int(round(0.2 * n_atoms))), seed)


def csr_to_dense(row_ptr, col, val, n):
    out = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    out[rows, col] = val
    return out
