"""ctypes front end of the reference oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  Imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark; never by the GPU library.  The C side is a
plain single-threaded FP64 implementation of the paper's method
(arXiv:2212.01997, Secs. II and IV).  `solve_pool` runs the same per-subgraph
routines in worker processes for large systems; every reduction that couples
subgraphs (mu, mu1) still runs in fixed subgraph order in the parent, so its
results equal the serial ones bit for bit (pinned against the serial path in
tests/test_oracle_pool.py for 1, 3, 5 and 16 workers).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

PATHS2 = 1
COMPLETE = 2
FN_FERMI, FN_IDENT, FN_SQUARE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP64, IEEE semantics, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Csr(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class _Graph(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_orb", C.c_int32), ("n_sub", C.c_int32),
                ("sub_ptr", C.POINTER(C.c_int32)), ("sub_atoms", C.POINTER(C.c_int32)),
                ("n_core_atoms", C.POINTER(C.c_int32)), ("sub_orb_ptr", C.POINTER(C.c_int32)),
                ("sub_orbs", C.POINTER(C.c_int32)), ("n_core_orbs", C.POINTER(C.c_int32)),
                ("rho_row_ptr", C.POINTER(C.c_int32)), ("rho_col", C.POINTER(C.c_int32)),
                ("nnz", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.orc_last_error.restype = C.c_char_p
        L.orc_graph_build.argtypes = [C.c_int32, ip, C.POINTER(_Csr), C.POINTER(_Csr), ip,
                                      C.c_double, C.c_int32, C.POINTER(_Graph)]
        L.orc_graph_free.argtypes = [C.POINTER(_Graph)]
        L.orc_gather.argtypes = [C.POINTER(_Csr), C.c_int32, ip, dp]
        L.orc_eigh.argtypes = [C.c_int32, dp, dp, dp]
        L.orc_core_weights.argtypes = [C.c_int32, C.c_int32, dp, dp]
        L.orc_occupation.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_find_mu.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_double, dp]
        L.orc_fermi.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_fermi.restype = C.c_double
        L.orc_divided_differences.argtypes = [C.c_int32, dp, C.c_double, C.c_double, dp]
        L.orc_core_rows.argtypes = [C.c_int32, C.c_int32, dp, dp, C.c_double, C.c_double,
                                    C.c_int32, dp]
        L.orc_mu_response_rows.argtypes = [C.c_int32, C.c_int32, dp, dp, C.c_double,
                                           C.c_double, dp, dp]
        L.orc_lambda_response_rows.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp, dp]
        L.orc_mu1.argtypes = [C.c_int32, dp, dp]
        L.orc_mu1.restype = C.c_double
        L.orc_collect.argtypes = [C.POINTER(_Graph), C.c_int32, dp, dp]
        L.orc_solve.argtypes = [C.POINTER(_Graph), C.POINTER(_Csr), C.c_double, C.c_double,
                                C.c_int32, C.c_int32, C.POINTER(_Csr), dp, dp, dp, dp, dp]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise OracleError(f"oracle status {rc}: {lib().orc_last_error().decode()}")


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Csr:
    """Keeps the numpy buffers of a CSR alive next to its ctypes struct."""

    def __init__(self, row_ptr, col, val):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.n = len(self.row_ptr) - 1
        self.s = _Csr(self.n, len(self.col), self.row_ptr.ctypes.data, self.col.ctypes.data,
                      self.val.ctypes.data)

    @staticmethod
    def diagonal(d):
        d = np.asarray(d, dtype=np.float64)
        n = len(d)
        return Csr(np.arange(n + 1), np.arange(n), d)

    @staticmethod
    def from_dense(a, keep_zero_pattern=None):
        n = a.shape[0]
        mask = a != 0 if keep_zero_pattern is None else keep_zero_pattern
        rows, cols = np.nonzero(mask)
        rp = np.zeros(n + 1, dtype=np.int64)
        np.add.at(rp, rows + 1, 1)
        return Csr(np.cumsum(rp), cols, a[rows, cols])


@dataclass
class Graph:
    n_atoms: int
    n_orb: int
    n_sub: int
    sub_ptr: np.ndarray
    sub_atoms: np.ndarray
    n_core_atoms: np.ndarray
    sub_orb_ptr: np.ndarray
    sub_orbs: np.ndarray
    n_core_orbs: np.ndarray
    rho_row_ptr: np.ndarray
    rho_col: np.ndarray

    @property
    def nnz(self):
        return int(self.rho_row_ptr[-1])

    def sizes(self):
        return np.diff(self.sub_orb_ptr)

    def orbs(self, s):
        return self.sub_orbs[self.sub_orb_ptr[s]:self.sub_orb_ptr[s + 1]]

    def cstruct(self):
        g = _Graph()
        g.n_atoms, g.n_orb, g.n_sub = self.n_atoms, self.n_orb, self.n_sub
        self._keep = []
        for name in ("sub_ptr", "sub_atoms", "n_core_atoms", "sub_orb_ptr", "sub_orbs",
                     "n_core_orbs", "rho_row_ptr", "rho_col"):
            arr = np.ascontiguousarray(getattr(self, name), dtype=np.int32)
            self._keep.append(arr)
            setattr(g, name, _ip(arr))
        g.nnz = self.nnz
        return g


def graph_build(system, core_of_atom, tau, rho_prev=None, flags=0) -> Graph:
    """Sec. II.E / II.C: estimate the graph and partition it into subgraphs."""
    H = Csr(system.h_row_ptr, system.h_col, system.h_val)
    rp = None if rho_prev is None else Csr(*rho_prev)
    core = np.ascontiguousarray(core_of_atom, dtype=np.int32)
    aop = np.ascontiguousarray(system.atom_orb_ptr, dtype=np.int32)
    g = _Graph()
    rc = lib().orc_graph_build(system.n_atoms, _ip(aop), C.byref(H.s),
                               C.byref(rp.s) if rp is not None else None, _ip(core),
                               float(tau), int(flags), C.byref(g))
    _check(rc)
    ns, N = g.n_sub, g.n_orb

    def grab(ptr, n):
        return np.ctypeslib.as_array(ptr, shape=(n,)).copy() if n > 0 else np.zeros(0, np.int32)

    sub_ptr = grab(g.sub_ptr, ns + 1)
    sub_orb_ptr = grab(g.sub_orb_ptr, ns + 1)
    rho_row_ptr = grab(g.rho_row_ptr, N + 1)
    out = Graph(g.n_atoms, N, ns, sub_ptr, grab(g.sub_atoms, int(sub_ptr[-1])),
                grab(g.n_core_atoms, ns), sub_orb_ptr, grab(g.sub_orbs, int(sub_orb_ptr[-1])),
                grab(g.n_core_orbs, ns), rho_row_ptr, grab(g.rho_col, int(rho_row_ptr[-1])))
    lib().orc_graph_free(C.byref(g))
    return out


def gather(csr: Csr, orbs):
    orbs = np.ascontiguousarray(orbs, dtype=np.int32)
    n = len(orbs)
    h = np.zeros(n * n)
    _check(lib().orc_gather(C.byref(csr.s), n, _ip(orbs), _dp(h)))
    return h.reshape(n, n, order="F")


def eigh(a):
    """Householder + implicit QL eigensolve: returns (w ascending, Z)."""
    a = np.asfortranarray(a, dtype=np.float64)
    n = a.shape[0]
    w = np.zeros(n)
    z = np.zeros(n * n)
    _check(lib().orc_eigh(n, _dp(a.ravel(order="F")), _dp(w), _dp(z)))
    return w, z.reshape(n, n, order="F")


def core_weights(z, c):
    z = np.asfortranarray(z)
    n = z.shape[0]
    w = np.zeros(n)
    lib().orc_core_weights(n, c, _dp(z.ravel(order="F")), _dp(w))
    return w


def occupation(e, w, mu, kT, n_elec):
    e = np.ascontiguousarray(e, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    F = C.c_double()
    dF = C.c_double()
    lib().orc_occupation(len(e), _dp(e), _dp(w), mu, kT, n_elec, C.byref(F), C.byref(dF))
    return F.value, dF.value


def find_mu(e, w, kT, n_elec):
    e = np.ascontiguousarray(e, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    mu = C.c_double()
    _check(lib().orc_find_mu(len(e), _dp(e), _dp(w), kT, n_elec, C.byref(mu)))
    return mu.value


def fermi(e, mu, kT):
    return np.array([lib().orc_fermi(float(x), mu, kT) for x in np.atleast_1d(e)])


def divided_differences(e, mu, kT):
    e = np.ascontiguousarray(e, dtype=np.float64)
    n = len(e)
    out = np.zeros(n * n)
    lib().orc_divided_differences(n, _dp(e), mu, kT, _dp(out))
    return out.reshape(n, n, order="F")


def core_rows(z, e, c, mu, kT, fn=FN_FERMI):
    z = np.asfortranarray(z)
    n = z.shape[0]
    out = np.zeros(c * n)
    lib().orc_core_rows(n, c, _dp(z.ravel(order="F")), _dp(np.ascontiguousarray(e)), mu, kT,
                        fn, _dp(out))
    return out.reshape(c, n)


def mu_response_rows(z, e, c, mu, kT):
    z = np.asfortranarray(z)
    n = z.shape[0]
    out = np.zeros(c * n)
    tr = C.c_double()
    lib().orc_mu_response_rows(n, c, _dp(z.ravel(order="F")), _dp(np.ascontiguousarray(e)),
                               mu, kT, _dp(out), C.byref(tr))
    return out.reshape(c, n), tr.value


def lambda_response_rows(z, dF, h1, c):
    z = np.asfortranarray(z)
    n = z.shape[0]
    out = np.zeros(c * n)
    tr = C.c_double()
    lib().orc_lambda_response_rows(n, c, _dp(z.ravel(order="F")),
                                   _dp(np.asfortranarray(dF).ravel(order="F")),
                                   _dp(np.asfortranarray(h1).ravel(order="F")), _dp(out),
                                   C.byref(tr))
    return out.reshape(c, n), tr.value


def mu1(tlam, tmu):
    tlam = np.ascontiguousarray(tlam, dtype=np.float64)
    tmu = np.ascontiguousarray(tmu, dtype=np.float64)
    return lib().orc_mu1(len(tlam), _dp(tlam), _dp(tmu))


def collect(graph: Graph, s, rows, vals):
    gs = graph.cstruct()
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    lib().orc_collect(C.byref(gs), s, _dp(rows), _dp(vals))


@dataclass
class Result:
    rho: np.ndarray        # [nnz] collected density values (graph pattern)
    mu: float
    rho1: np.ndarray       # [K, nnz]
    mu1: np.ndarray        # [K]
    eps: np.ndarray        # [sum n] eigenvalues, subgraph by subgraph, ascending


def _h1_csrs(h1, n_orb):
    """Perturbations: a [K, N] array of diagonals or a list of (row_ptr, col, val)."""
    if h1 is None:
        return []
    if isinstance(h1, np.ndarray):
        h1 = np.atleast_2d(h1)
        return [Csr.diagonal(row) for row in h1]
    return [Csr(*m) for m in h1]


def solve(system, graph: Graph, kT, h1=None, n_elec=None, fn=FN_FERMI) -> Result:
    """Serial whole path (Sec. II + Sec. IV) on the given graph."""
    H = Csr(system.h_row_ptr, system.h_col, system.h_val)
    mats = _h1_csrs(h1, system.n_orb)
    K = len(mats)
    arr = (_Csr * max(K, 1))()
    for q, m in enumerate(mats):
        arr[q] = m.s
    gs = graph.cstruct()
    rho = np.zeros(graph.nnz)
    rho1 = np.zeros((K, graph.nnz))
    mu1v = np.zeros(max(K, 1))
    eps = np.zeros(int(graph.sub_orb_ptr[-1]))
    mu = C.c_double()
    ne = system.n_elec if n_elec is None else n_elec
    _check(lib().orc_solve(C.byref(gs), C.byref(H.s), kT, ne, fn, K, arr, _dp(rho),
                           C.byref(mu), _dp(rho1), _dp(mu1v), _dp(eps)))
    return Result(rho, mu.value, rho1, mu1v[:K].copy(), eps)


# ------------------------------------------------- per-subgraph worker pool

_W = {}


def _w_init(system_arrays, graph, h1_diag):
    _W["H"] = Csr(*system_arrays)
    _W["g"] = graph
    _W["h1"] = h1_diag
    _W["Z"] = {}


def _w_eig(subs):
    out = []
    g = _W["g"]
    for s in subs:
        orbs = g.orbs(s)
        h = gather(_W["H"], orbs)
        e, z = eigh(h)
        _W["Z"][s] = (e, z)
        out.append((s, e, core_weights(z, int(g.n_core_orbs[s]))))
    return out


def _w_rows(args):
    subs, mu, kT, fn = args
    g = _W["g"]
    out = []
    for s in subs:
        e, z = _W["Z"][s]
        c = int(g.n_core_orbs[s])
        rows = core_rows(z, e, c, mu, kT, fn)
        item = {"s": s, "rows": rows}
        h1 = _W["h1"]
        if h1 is not None and fn == FN_FERMI:
            M, tmu = mu_response_rows(z, e, c, mu, kT)
            dF = divided_differences(e, mu, kT)
            orbs = g.orbs(s)
            P, tl = [], []
            for q in range(h1.shape[0]):
                p, t = lambda_response_rows(z, dF, np.diag(h1[q, orbs]), c)
                P.append(p)
                tl.append(t)
            item.update(M=M, tmu=tmu, P=P, tlam=tl)
        out.append(item)
    return out


def solve_pool(system, graph: Graph, kT, h1_diag=None, n_elec=None, fn=FN_FERMI,
               workers=None) -> Result:
    """Same results as `solve` for diagonal perturbations, with the independent
    per-subgraph work spread over worker processes.  Subgraphs are dealt out
    round-robin by descending size; every cross-subgraph sum runs afterwards in
    ascending subgraph order."""
    import multiprocessing as mp
    workers = workers or min(16, os.cpu_count() or 1)
    ns = graph.n_sub
    order = np.argsort(-graph.sizes(), kind="stable")
    chunks = [list(map(int, order[w::workers])) for w in range(workers)]
    chunks = [c for c in chunks if c]
    h1 = None if h1_diag is None else np.atleast_2d(np.asarray(h1_diag, dtype=np.float64))
    ctx = mp.get_context("spawn")  # safe after a GPU runtime is initialised
    sa = (system.h_row_ptr, system.h_col, system.h_val)
    eps_l, wts_l = [None] * ns, [None] * ns
    items = [None] * ns
    # one process per chunk keeps its eigenvectors between the two phases
    with ctx.Pool(len(chunks), initializer=_w_init, initargs=(sa, graph, h1)) as pool:
        # pin chunk -> process by running each phase as one task per process
        res = _pinned_map(pool, _w_eig, chunks)
        for part in res:
            for s, e, w in part:
                eps_l[s], wts_l[s] = e, w
        eps = np.concatenate(eps_l)
        wts = np.concatenate(wts_l)
        ne = system.n_elec if n_elec is None else n_elec
        mu = find_mu(eps, wts, kT, ne) if fn == FN_FERMI else 0.0
        res = _pinned_map(pool, _w_rows, [(c, mu, kT, fn) for c in chunks])
        for part in res:
            for it in part:
                items[it["s"]] = it
    rho = np.zeros(graph.nnz)
    for s in range(ns):
        collect(graph, s, items[s]["rows"], rho)
    K = 0 if h1 is None or fn != FN_FERMI else h1.shape[0]
    rho1 = np.zeros((K, graph.nnz))
    mu1v = np.zeros(K)
    if K:
        tmu = np.array([items[s]["tmu"] for s in range(ns)])
        for q in range(K):
            tl = np.array([items[s]["tlam"][q] for s in range(ns)])
            m1 = mu1(tl, tmu)
            mu1v[q] = m1
            for s in range(ns):
                collect(graph, s, items[s]["P"][q] + m1 * items[s]["M"], rho1[q])
    return Result(rho, mu, rho1, mu1v, eps)


def _pinned_map(pool, fn, chunks):
    """Run fn(chunk_i) so that chunk i always lands on the same worker: each
    worker takes exactly one task per phase, in worker-start order."""
    # Pool hands tasks to idle workers in arbitrary order, so state kept in a
    # worker must not be assumed to match a chunk.  Workers therefore recompute
    # what they lack: the eigen phase stores results keyed by subgraph and the
    # rows phase recomputes any eigenpairs not found locally.
    return pool.map(_pinned_call, [(fn, c) for c in chunks], chunksize=1)


def _pinned_call(arg):
    fn, c = arg
    if fn is _w_rows:
        subs = c[0]
        missing = [s for s in subs if s not in _W["Z"]]
        if missing:
            _w_eig(missing)
    return fn(c)


def bootstrap_prev(system, core_of_atom, kT, pool=False):
    """Previous-step density for the graph estimate (Sec. II.E): one pass of the
    method on the graph of every nonzero of H (the m = 1 power estimate of
    Sec. II.E).  Returns the CSR triple (row_ptr, col, val) for `rho_prev`."""
    g0 = graph_build(system, core_of_atom, 0.0)
    r0 = (solve_pool if pool else solve)(system, g0, kT)
    return (g0.rho_row_ptr, g0.rho_col, r0.rho)
