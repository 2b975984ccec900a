"""Pins of the zero-temperature step-density oracle (oracle/foe.py, Sec. II.D,
Eqs. (Step), (dCollect)) against what the mathematics fixes, none of them
through the oracle's own eigensolve route alone:

- 2x2 closed form: Theta(mu - h) is the spectral projector (h - l+ I)/(l- - l+)
  for mu between the two eigenvalues, 0 below both and I above both.
- Sylvester's law of inertia: Tr Theta(mu - h) equals the number of negative
  pivots of the LDL^T factorisation of h - mu I (scipy's Bunch-Kaufman).
- Idempotency d^2 = d and [d, h] = 0.
- The zero-temperature limit of the pinned finite-temperature core rows: the
  Fermi rows at kT = gap / 40 equal the step rows within the exp(-40) bound.
- A McWeeny iteration in plain numpy (matrix products only) from
  X_0 = I/2 - (h - mu I)/(2R) converges to the oracle's rows.
- Collected over a graph: mu below every subgraph eigenvalue gives 0, above
  every one gives 2 I on the core rows.
CPU only.
"""
import numpy as np
import pytest
import scipy.linalg

from paper_2212_01997_amd import inputs as I


@pytest.fixture(scope="module")
def F(oracle_lib):
    from oracle import foe
    return foe


def _sym(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    return 0.5 * (a + a.T)


def _negative_pivots(a):
    """Negative eigenvalues of a from its LDL^T factorisation (inertia)."""
    _, d, _ = scipy.linalg.ldl(a)
    count, i, n = 0, 0, a.shape[0]
    while i < n:
        if i + 1 < n and d[i + 1, i] != 0.0:  # a 2x2 pivot block
            blk = d[i:i + 2, i:i + 2]
            det = blk[0, 0] * blk[1, 1] - blk[0, 1] * blk[1, 0]
            tr = blk[0, 0] + blk[1, 1]
            count += 1 if det < 0 else (2 if tr < 0 else 0)
            i += 2
        else:
            count += d[i, i] < 0
            i += 1
    return count


def test_two_by_two_closed_form(F):
    a, b, c = 0.3, -0.7, -0.4
    h = np.array([[a, b], [b, c]])
    r = np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    lm, lp = 0.5 * (a + c) - r, 0.5 * (a + c) + r
    proj = (h - lp * np.eye(2)) / (lm - lp)
    assert np.abs(F.step_rows(h, 2, 0.5 * (lm + lp)) - 2.0 * proj).max() <= 1e-14
    assert np.abs(F.step_rows(h, 1, 0.5 * (lm + lp)) - 2.0 * proj[:1]).max() <= 1e-14
    assert np.abs(F.step_rows(h, 2, lm - 1.0)).max() == 0.0
    assert np.abs(F.step_rows(h, 2, lp + 1.0) - 2.0 * np.eye(2)).max() <= 1e-14
    with pytest.raises(ValueError):
        F.step_rows(np.diag([1.0, 2.0]), 2, 1.0)


@pytest.mark.parametrize("seed,mu", [(1, 0.0), (2, -1.3), (3, 2.1)])
def test_trace_is_inertia(F, seed, mu):
    h = _sym(40, seed)
    d = F.step_rows(h, 40, mu) / 2.0
    assert abs(np.trace(d) - _negative_pivots(h - mu * np.eye(40))) <= 1e-10


def test_idempotent_and_commuting(F):
    h = _sym(50, 4)
    d = F.step_rows(h, 50, 0.2) / 2.0
    assert np.abs(d @ d - d).max() <= 1e-12
    assert np.abs(d @ h - h @ d).max() <= 1e-12 * np.abs(h).max() * 50
    assert np.abs(d - d.T).max() <= 1e-13


@pytest.fixture(scope="module")
def subgraph(oracle_lib):
    O = oracle_lib
    s = I.water32_system()
    core = I.spatial_cores(s, 3)
    g = O.graph_build(s, core, 0.07, rho_prev=O.bootstrap_prev(s, core, 0.01), flags=O.PATHS2)
    H = O.Csr(s.h_row_ptr, s.h_col, s.h_val)
    h = O.gather(H, g.orbs(0))
    return s, g, h, int(g.n_core_orbs[0])


def test_zero_temperature_limit_of_fermi_rows(oracle_lib, F, subgraph):
    O = oracle_lib
    _, _, h, c = subgraph
    w, z = O.eigh(h)
    k = int(np.argmax(np.diff(w)))  # the widest gap of the spectrum
    mu = F.mid_gap(w, 0.5 * (w[k] + w[k + 1]))
    gap = np.abs(w - mu).min()
    assert gap > 1e-3
    kT = gap / 40.0
    fermi = O.core_rows(z, w, c, mu, kT)
    assert np.abs(fermi - F.step_rows(h, c, mu)).max() <= 2.0 * len(w) * np.exp(-40.0)


def test_mcweeny_iteration_converges_to_step(F, subgraph):
    _, _, h, c = subgraph
    n = h.shape[0]
    w = np.linalg.eigvalsh(h)
    k = n // 4 + int(np.argmax(np.diff(w[n // 4:3 * n // 4])))  # a gap inside the spectrum
    mu = 0.5 * (w[k] + w[k + 1])
    R = np.abs(h - mu * np.eye(n)).sum(axis=1).max()
    x = 0.5 * np.eye(n) - (h - mu * np.eye(n)) / (2.0 * R)
    for _ in range(200):
        x2 = x @ x
        if np.abs(x2 - x).max() <= 1e-13:
            break
        x = 3.0 * x2 - 2.0 * x2 @ x
    assert np.abs(2.0 * x[:c] - F.step_rows(h, c, mu)).max() <= 1e-10


def test_collected_limits(oracle_lib, F, subgraph):
    s, g, _, _ = subgraph
    lo, gap_lo = F.purified_density(s, g, -50.0)
    assert np.abs(lo).max() == 0.0 and gap_lo > 0
    hi, _ = F.purified_density(s, g, 50.0)
    rows = np.repeat(np.arange(g.n_orb), np.diff(g.rho_row_ptr))
    expect = np.where(rows == g.rho_col, 2.0, 0.0)
    assert np.abs(hi - expect).max() <= 1e-12


def test_mid_gap(F):
    eps = np.array([-1.0, -0.3, 0.1, 0.4, 2.0])
    mu = F.mid_gap(eps, 0.0)
    assert mu == pytest.approx(-0.1)
    assert np.abs(eps - mu).min() == pytest.approx(0.2)
