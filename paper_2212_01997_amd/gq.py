"""Python binding of libgq (include/gq.h): argument marshalling only.

Every step of the path runs in the HIP kernels of libgq.so; PyTorch provides
device memory and the stream.  Importing this module does not need a GPU;
creating a Context does, and fails loudly if the library or device is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgq.so")

PATHS2 = 1
COMPLETE = 2
PREC_FP64 = 0
PREC_SPLIT32 = 1
EIGS_GENERAL_H1 = 1
EIGS_OVERLAP = 2
H1_DIAG = 0
H1_CSR = 1

_STATUS = {0: "GQ_OK", -1: "GQ_EINVAL", -2: "GQ_ENOMEM", -3: "GQ_ENOCONV", -4: "GQ_EDEVICE",
           -5: "GQ_EBUSY"}


class GQError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Csr(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class _Info(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_orb", C.c_int32), ("n_sub", C.c_int32),
                ("max_n", C.c_int32), ("min_n", C.c_int32), ("max_c", C.c_int32),
                ("nnz", C.c_int64), ("sum_n", C.c_int64), ("sum_n2", C.c_int64),
                ("sub_atoms_len", C.c_int64)]


class _Request(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("atom_orb_ptr", C.c_void_p), ("H", C.POINTER(_Csr)),
                ("rho_prev", C.POINTER(_Csr)), ("core_of_atom", C.c_void_p), ("tau", C.c_double),
                ("flags", C.c_uint32), ("kT", C.c_double), ("n_elec", C.c_double),
                ("K", C.c_int32), ("h1", C.c_void_p), ("precision", C.c_uint32)]


class _ReqInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("mu", C.c_double), ("n_sub", C.c_int32), ("K", C.c_int32),
                ("nnz", C.c_int64), ("footprint", C.c_int64), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double)]


# every symbol declared in include/gq.h, with its ctypes signature
_VP = C.c_void_p
_SIGS = {
    "gq_last_error": ([], C.c_char_p),
    "gq_version": ([], C.c_char_p),
    "gq_ctx_create": ([C.c_int32, _VP, C.c_int64, C.POINTER(_VP)], C.c_int32),
    "gq_ctx_arena_used": ([_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int32),
    "gq_ctx_destroy": ([_VP], None),
    "gq_graph_build": ([C.c_int32, _VP, C.POINTER(_Csr), C.POINTER(_Csr), _VP, C.c_double,
                        C.c_uint32, C.POINTER(_VP)], C.c_int32),
    "gq_graph_query": ([_VP, C.POINTER(_Info)], C.c_int32),
    "gq_graph_export": ([_VP] + [_VP] * 8, C.c_int32),
    "gq_graph_block_offsets": ([_VP, _VP], C.c_int32),
    "gq_graph_destroy": ([_VP], None),
    "gq_eigs_create": ([_VP, _VP, C.c_int32, C.c_uint32, C.POINTER(_VP)], C.c_int32),
    "gq_eigs_create_in": ([_VP, _VP, C.c_int32, C.c_uint32, _VP, C.c_int64, C.POINTER(_VP)],
                          C.c_int32),
    "gq_eigs_footprint": ([_VP, C.c_int32, C.c_uint32, C.POINTER(C.c_int64)], C.c_int32),
    "gq_eigs_destroy": ([_VP], None),
    "gq_submatrix_solve": ([_VP, _VP, C.POINTER(_Csr), C.c_uint32, _VP], C.c_int32),
    "gq_submatrix_solve_overlap": ([_VP, _VP, C.POINTER(_Csr), C.POINTER(_Csr), C.c_uint32, _VP],
                                   C.c_int32),
    "gq_density": ([_VP, _VP, C.c_double, C.c_double, _VP, _VP], C.c_int32),
    "gq_purify": ([_VP, _VP, C.POINTER(_Csr), _VP, C.c_double, C.c_int32, C.c_double, _VP,
                   C.POINTER(C.c_int32)], C.c_int32),
    "gq_response": ([_VP, _VP, _VP, C.c_uint32, C.c_int32, C.c_uint32, _VP, _VP, _VP],
                    C.c_int32),
    "gq_response_static": ([_VP, _VP, _VP, C.c_uint32, C.c_int32, C.c_uint32, _VP, _VP],
                           C.c_int32),
    "gq_assemble": ([_VP, _VP, _VP, C.c_int32, _VP], C.c_int32),
    "gq_eigs_export": ([_VP, _VP, _VP, _VP], C.c_int32),
    "gq_eigs_vectors": ([_VP, C.c_int32, C.POINTER(_VP), C.POINTER(C.c_int32)], C.c_int32),
    "gq_autotune": ([_VP, _VP, C.c_uint32, C.c_char_p, C.c_size_t], C.c_int32),
    "gq_graph_set_launch": ([_VP, C.c_uint32, C.c_int32, C.c_int32], C.c_int32),
    "gq_capture_begin": ([_VP], C.c_int32),
    "gq_capture_end": ([_VP, C.POINTER(_VP)], C.c_int32),
    "gq_exec_launch": ([_VP, _VP], C.c_int32),
    "gq_exec_destroy": ([_VP], None),
    "gq_charge_create": ([_VP, _VP, C.POINTER(_Csr), C.c_int32, C.POINTER(_VP)], C.c_int32),
    "gq_charge_destroy": ([_VP], None),
    "gq_charge_core": ([_VP, _VP, _VP, _VP], C.c_int32),
    "gq_charge_response": ([_VP, _VP, _VP, _VP, C.c_int32, C.c_uint32, _VP, _VP], C.c_int32),
    "gq_preconditioner": ([_VP, _VP, _VP, C.c_double, _VP, _VP], C.c_int32),
    "gq_krylov_kernel": ([_VP, _VP, _VP, _VP, _VP, _VP, C.c_int32, C.c_double, C.c_uint32,
                          _VP, _VP, _VP, _VP, _VP, _VP], C.c_int32),
    "gq_server_create": ([C.c_int32, C.c_int32, C.c_int64, C.POINTER(_VP)], C.c_int32),
    "gq_server_submit": ([_VP, C.POINTER(_Request), C.POINTER(C.c_int64)], C.c_int32),
    "gq_server_wait": ([_VP, C.c_int64, C.POINTER(_ReqInfo)], C.c_int32),
    "gq_server_fetch": ([_VP, C.c_int64, _VP, _VP, _VP, _VP, _VP], C.c_int32),
    "gq_server_release": ([_VP, C.c_int64], C.c_int32),
    "gq_server_arena_used": ([_VP, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int32),
    "gq_server_clock": ([_VP], C.c_double),
    "gq_server_destroy": ([_VP], None),
    "gq_ctx_set_profiling": ([_VP, C.c_int32], C.c_int32),
    "gq_ctx_set_iteration_cap": ([_VP, C.c_int32], C.c_int32),
    "gq_ctx_set_split_window": ([_VP, C.c_double, C.c_int32], C.c_int32),
    "gq_ctx_kernel_times": ([_VP, _VP, _VP, _VP, C.c_int32, C.POINTER(C.c_int32)], C.c_int32),
}

_lib = None


def lib():
    """Load libgq.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes libgq bind to that one, so both share one runtime
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise GQError(-4, f"{LIB_PATH} is missing: run `python -m paper_2212_01997_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise GQError(st, lib().gq_last_error().decode())


def _host_csr(row_ptr, col, val, keep):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    vl = np.ascontiguousarray(val, dtype=np.float64)
    keep += [rp, cl, vl]
    return _Csr(len(rp) - 1, len(cl), rp.ctypes.data, cl.ctypes.data, vl.ctypes.data)


def _ptr(t):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def _release(obj, fn):
    """Destroy obj.h with libgq's `fn` (skipped once the interpreter is exiting)."""
    h = getattr(obj, "h", None)
    obj.h = None
    if h and _lib is not None:
        try:
            getattr(_lib, fn)(h)
        except Exception:  # interpreter shutdown
            pass


class Context:
    """gq_ctx_create: a device, a stream and, with arena_bytes > 0, one device
    arena that every workspace made on this context takes its memory from."""

    def __init__(self, device=0, stream=None, arena_bytes=0):
        import torch
        if not torch.cuda.is_available():
            raise GQError(-4, "no GPU visible")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = _VP()
        _check(lib().gq_ctx_create(device, _VP(self.stream.cuda_stream), int(arena_bytes),
                                   C.byref(h)))
        self.h = h

    def arena_used(self):
        used, size = C.c_int64(), C.c_int64()
        _check(lib().gq_ctx_arena_used(self.h, C.byref(used), C.byref(size)))
        return used.value, size.value

    def set_iteration_cap(self, leaf_iterations=60):
        """Diagnostics: QL iterations per eigenvalue allowed in the leaves."""
        _check(lib().gq_ctx_set_iteration_cap(self.h, int(leaf_iterations)))

    def set_split_window(self, dF_threshold=10.0, max_states=128):
        """Refinement window of the split-FP32 response (gq_ctx_set_split_window)."""
        _check(lib().gq_ctx_set_split_window(self.h, float(dF_threshold), int(max_states)))

    def set_profiling(self, enable=True):
        _check(lib().gq_ctx_set_profiling(self.h, 1 if enable else 0))

    def kernel_times(self):
        """{kernel name: (launches, total ms)} since profiling was enabled."""
        cap = 64
        names = (C.c_char_p * cap)()
        launches = np.zeros(cap, np.int64)
        ms = np.zeros(cap)
        cnt = C.c_int32()
        _check(lib().gq_ctx_kernel_times(self.h, names, launches.ctypes.data, ms.ctypes.data, cap,
                                         C.byref(cnt)))
        return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(cnt.value)}

    def capture_begin(self):
        """Start recording library calls on this context into a HIP graph."""
        _check(lib().gq_capture_begin(self.h))

    def capture_end(self):
        """Stop recording; returns an Exec that replays the recorded work."""
        x = _VP()
        _check(lib().gq_capture_end(self.h, C.byref(x)))
        return Exec(self, x)

    def __del__(self, _rel=_release):
        _rel(self, "gq_ctx_destroy")


class Exec:
    """Recorded sequence of library calls (gq_capture_end)."""

    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def launch(self):
        _check(lib().gq_exec_launch(self.ctx.h, self.h))

    def __del__(self, _rel=_release):
        _rel(self, "gq_exec_destroy")


@dataclass
class GraphInfo:
    n_atoms: int
    n_orb: int
    n_sub: int
    max_n: int
    min_n: int
    max_c: int
    nnz: int
    sum_n: int
    sum_n2: int
    sub_atoms_len: int


class Graph:
    """gq_graph_build: host call, no GPU needed."""

    def __init__(self, n_atoms, atom_orb_ptr, H, core_of_atom, tau, rho_prev=None, flags=0):
        keep = []
        hs = _host_csr(*H, keep)
        rp = _host_csr(*rho_prev, keep) if rho_prev is not None else None
        aop = np.ascontiguousarray(atom_orb_ptr, dtype=np.int32)
        core = np.ascontiguousarray(core_of_atom, dtype=np.int32)
        h = _VP()
        _check(lib().gq_graph_build(int(n_atoms), aop.ctypes.data, C.byref(hs),
                                    C.byref(rp) if rp is not None else None, core.ctypes.data,
                                    float(tau), int(flags), C.byref(h)))
        self.h = h
        inf = _Info()
        _check(lib().gq_graph_query(h, C.byref(inf)))
        self.info = GraphInfo(*[getattr(inf, f[0]) for f in _Info._fields_])

    @staticmethod
    def for_system(system, core_of_atom, tau, rho_prev=None, flags=0):
        return Graph(system.n_atoms, system.atom_orb_ptr,
                     (system.h_row_ptr, system.h_col, system.h_val), core_of_atom, tau,
                     rho_prev=rho_prev, flags=flags)

    def export(self):
        i = self.info
        out = {
            "sub_ptr": np.zeros(i.n_sub + 1, np.int32),
            "sub_atoms": np.zeros(i.sub_atoms_len, np.int32),
            "n_core_atoms": np.zeros(i.n_sub, np.int32),
            "sub_orb_ptr": np.zeros(i.n_sub + 1, np.int32),
            "sub_orbs": np.zeros(i.sum_n, np.int32),
            "n_core_orbs": np.zeros(i.n_sub, np.int32),
            "rho_row_ptr": np.zeros(i.n_orb + 1, np.int32),
            "rho_col": np.zeros(i.nnz, np.int32),
        }
        _check(lib().gq_graph_export(self.h, *[v.ctypes.data for v in out.values()]))
        return out

    def block_offsets(self):
        off = np.zeros(self.info.n_sub + 1, np.int64)
        _check(lib().gq_graph_block_offsets(self.h, off.ctypes.data))
        return off

    def set_launch(self, precision, bin_index, variant):
        """Force the X-kernel launch variant of one size bin (gq_graph_set_launch)."""
        _check(lib().gq_graph_set_launch(self.h, int(precision), int(bin_index), int(variant)))

    def footprint(self, max_k, flags=0):
        b = C.c_int64()
        _check(lib().gq_eigs_footprint(self.h, int(max_k), int(flags), C.byref(b)))
        return b.value

    def __del__(self, _rel=_release):
        _rel(self, "gq_graph_destroy")


class DeviceCsr:
    """A CSR matrix copied to the device as torch tensors."""

    def __init__(self, row_ptr, col, val, device=0):
        import torch
        dev = torch.device("cuda", device)
        self.row_ptr = torch.as_tensor(np.ascontiguousarray(row_ptr, np.int32), device=dev)
        self.col = torch.as_tensor(np.ascontiguousarray(col, np.int32), device=dev)
        self.val = torch.as_tensor(np.ascontiguousarray(val, np.float64), device=dev)

    def cstruct(self):
        return _Csr(self.row_ptr.numel() - 1, self.col.numel(), self.row_ptr.data_ptr(),
                    self.col.data_ptr(), self.val.data_ptr())


class Eigs:
    """Device-resident eigen workspace of one graph (gq_eigs_create)."""

    def __init__(self, ctx: Context, graph: Graph, max_k=1, general_h1=False, overlap=False):
        self.ctx, self.graph, self.max_k = ctx, graph, max_k
        h = _VP()
        flags = (EIGS_GENERAL_H1 if general_h1 else 0) | (EIGS_OVERLAP if overlap else 0)
        _check(lib().gq_eigs_create(ctx.h, graph.h, int(max_k), flags, C.byref(h)))
        self.h = h

    def solve(self, H: DeviceCsr):
        s = H.cstruct()
        _check(lib().gq_submatrix_solve(self.ctx.h, self.graph.h, C.byref(s), 0, self.h))

    def solve_overlap(self, H: DeviceCsr, S: DeviceCsr):
        """gq_submatrix_solve_overlap: non-orthogonal basis with overlap S
        (needs overlap=True); later densities and responses are in the
        atomic-orbital basis."""
        hs, ss = H.cstruct(), S.cstruct()
        _check(lib().gq_submatrix_solve_overlap(self.ctx.h, self.graph.h, C.byref(hs),
                                                C.byref(ss), 0, self.h))

    def density(self, kT, n_elec, rho_blocks=None, want_mu=True, mu_guess=None):
        """gq_density; mu_guess (or None) is the warm start.  Returns mu when
        want_mu (which waits for the stream)."""
        if mu_guess is not None and not want_mu:
            raise ValueError("a warm start returns mu: want_mu must be True")
        mu = C.c_double(float("nan") if mu_guess is None else float(mu_guess))
        _check(lib().gq_density(self.ctx.h, self.h, float(kT), float(n_elec),
                                C.byref(mu) if want_mu else None, _ptr(rho_blocks)))
        return mu.value if want_mu else None

    def purify(self, H: DeviceCsr, mu, rho_blocks, max_iter=60, tol=1e-11):
        """gq_purify: zero-temperature core rows 2 Theta(mu - h_i) by McWeeny
        purification into rho_blocks; returns the iterations run.  Raises
        GQError (GQ_ENOCONV) if a subgraph did not converge."""
        s = H.cstruct()
        it = C.c_int32(0)
        _check(lib().gq_purify(self.ctx.h, self.graph.h, C.byref(s), self.h, float(mu),
                               int(max_iter), float(tol), _ptr(rho_blocks), C.byref(it)))
        return it.value

    def response(self, h1, p_blocks, precision=PREC_FP64, mu1_dev=None, want_mu1=True):
        """gq_response.  h1: a [K, N] device tensor of diagonals, or a list of
        K DeviceCsr perturbations (needs general_h1=True)."""
        if isinstance(h1, (list, tuple)):
            K = len(h1)
            arr = (_Csr * K)(*[m.cstruct() for m in h1])
            arg, kind = C.cast(arr, _VP), H1_CSR
        else:
            K = int(h1.shape[0])
            arg, kind = _ptr(h1), H1_DIAG
        host = (C.c_double * K)()
        _check(lib().gq_response(self.ctx.h, self.h, arg, kind, K, int(precision),
                                 _ptr(p_blocks), _ptr(mu1_dev), host if want_mu1 else None))
        return np.array(host[:]) if want_mu1 else None

    def response_static(self, h1, p_blocks, precision=PREC_FP64, mu1_dev=None):
        """gq_response_static: as response, with the per-call buffers in the
        library's static device scratch (no allocation, no host wait)."""
        if isinstance(h1, (list, tuple)):
            K = len(h1)
            arr = (_Csr * K)(*[m.cstruct() for m in h1])
            arg, kind = C.cast(arr, _VP), H1_CSR
        else:
            K = int(h1.shape[0])
            arg, kind = _ptr(h1), H1_DIAG
        _check(lib().gq_response_static(self.ctx.h, self.h, arg, kind, K, int(precision),
                                        _ptr(p_blocks), _ptr(mu1_dev)))

    def export(self):
        n = self.graph.info.sum_n
        eps = np.zeros(n)
        w = np.zeros(n)
        _check(lib().gq_eigs_export(self.ctx.h, self.h, eps.ctypes.data, w.ctypes.data))
        return eps, w

    def vectors(self, i):
        p = _VP()
        n = C.c_int32()
        _check(lib().gq_eigs_vectors(self.h, int(i), C.byref(p), C.byref(n)))
        return p.value, n.value

    def autotune(self, precision=PREC_FP64):
        """Choose the X-kernel launch variant per size bin (gq_autotune); returns the report."""
        buf = C.create_string_buffer(8192)
        _check(lib().gq_autotune(self.ctx.h, self.h, int(precision), buf, len(buf)))
        return buf.value.decode()

    def __del__(self, _rel=_release):
        _rel(self, "gq_eigs_destroy")


class ChargeModel:
    """gq_charge_*: the charge response, the subgraph preconditioner and the
    preconditioned Krylov kernel (Sec. V) on one graph; gamma is the host CSR
    triple of the atom-by-atom charge kernel."""

    def __init__(self, ctx: Context, graph: Graph, gamma, kmax=8):
        import torch
        self.ctx, self.graph = ctx, graph
        keep = []
        gs = _host_csr(*gamma, keep)
        h = _VP()
        _check(lib().gq_charge_create(ctx.h, graph.h, C.byref(gs), int(kmax), C.byref(h)))
        self.h = h
        self.n_atoms = graph.info.n_atoms
        ex = graph.export()
        m = ex["n_core_atoms"].astype(np.int64)
        self.k0_offsets = np.concatenate([[0], np.cumsum(m * m)])
        self.dev = torch.device("cuda", ctx.device)

    def _empty(self, *shape, dtype=None):
        import torch
        return torch.empty(*shape, dtype=dtype or torch.float64, device=self.dev)

    def core(self, blocks):
        """Per-atom core charges of core-row blocks (gq_charge_core)."""
        q = self._empty(self.n_atoms)
        _check(lib().gq_charge_core(self.ctx.h, self.h, _ptr(blocks), _ptr(q)))
        return q

    def response(self, eigs: Eigs, v, precision=PREC_FP64):
        """(q1 [K, n_atoms], mu1 [K]) along the charge vectors v [K, n_atoms]."""
        K = int(v.shape[0])
        q1 = self._empty(K, self.n_atoms)
        mu1 = self._empty(K)
        _check(lib().gq_charge_response(self.ctx.h, self.h, eigs.h, _ptr(v.contiguous()), K,
                                        int(precision), _ptr(q1), _ptr(mu1)))
        return q1, mu1

    def preconditioner(self, eigs: Eigs, alpha):
        """k0 blocks (gq_preconditioner) as one device vector; raises if a
        block is singular."""
        import torch
        k0 = self._empty(int(self.k0_offsets[-1]))
        bad = torch.zeros(1, dtype=torch.int32, device=self.dev)
        _check(lib().gq_preconditioner(self.ctx.h, self.h, eigs.h, float(alpha), _ptr(k0),
                                       _ptr(bad)))
        self.ctx.stream.synchronize()
        if int(bad.item()):
            raise GQError(-3, "gq_preconditioner: a core Jacobian block is singular")
        return k0

    def blocks(self, k0):
        """The k0 vector split into its m_k x m_k blocks (host arrays)."""
        ex = self.graph.export()
        m = ex["n_core_atoms"]
        h = k0.cpu().numpy()
        return [h[self.k0_offsets[s]:self.k0_offsets[s + 1]].reshape(m[s], m[s], order="F")
                for s in range(len(m))]

    def krylov(self, eigs: Eigs, k0, rho_blocks, n, m, omega=1.0, precision=PREC_FP64):
        """gq_krylov_kernel; returns the device tensors ndd, V, F, O, M."""
        import torch
        out = {"ndd": self._empty(self.n_atoms), "V": self._empty(m, self.n_atoms),
               "F": self._empty(m, self.n_atoms), "O": self._empty(m, m), "M": self._empty(m, m)}
        bad = torch.zeros(1, dtype=torch.int32, device=self.dev)
        _check(lib().gq_krylov_kernel(self.ctx.h, self.h, eigs.h, _ptr(k0), _ptr(rho_blocks),
                                      _ptr(n.contiguous()), int(m), float(omega), int(precision),
                                      _ptr(out["ndd"]), _ptr(out["V"]), _ptr(out["F"]),
                                      _ptr(out["O"]), _ptr(out["M"]), _ptr(bad)))
        self.ctx.stream.synchronize()
        out["singular"] = bool(bad.item())
        return out

    def __del__(self, _rel=_release):
        _rel(self, "gq_charge_destroy")


def assemble(ctx: Context, graph: Graph, blocks, vals, K=1):
    _check(lib().gq_assemble(ctx.h, graph.h, _ptr(blocks), int(K), _ptr(vals)))


class Server:
    """Serving runtime (gq_server_*): continuous admission of whole-path
    requests into one device arena, n_slots requests in flight at a time."""

    def __init__(self, device=0, n_slots=4, arena_bytes=64 << 30):
        h = _VP()
        _check(lib().gq_server_create(int(device), int(n_slots), int(arena_bytes), C.byref(h)))
        self.h = h

    def submit(self, system, core_of_atom, tau, rho_prev=None, flags=0, kT=0.01, h1=None,
               precision=PREC_FP64, n_elec=None):
        keep = []
        H = _host_csr(system.h_row_ptr, system.h_col, system.h_val, keep)
        P = _host_csr(*rho_prev, keep) if rho_prev is not None else None
        aop = np.ascontiguousarray(system.atom_orb_ptr, np.int32)
        core = np.ascontiguousarray(core_of_atom, np.int32)
        h1 = np.ascontiguousarray(np.atleast_2d(h1), np.float64)
        req = _Request(system.n_atoms, aop.ctypes.data, C.pointer(H),
                       C.pointer(P) if P is not None else None, core.ctypes.data, float(tau),
                       int(flags), float(kT), float(system.n_elec if n_elec is None else n_elec),
                       h1.shape[0], h1.ctypes.data, int(precision))
        rid = C.c_int64()
        _check(lib().gq_server_submit(self.h, C.byref(req), C.byref(rid)))
        return rid.value

    def wait(self, rid):
        """Blocks until request rid has finished; returns its info as a dict."""
        info = _ReqInfo()
        _check(lib().gq_server_wait(self.h, int(rid), C.byref(info)))
        return {name: getattr(info, name) for name, _ in _ReqInfo._fields_}

    def fetch(self, rid, info, n_orb):
        K, nnz = info["K"], info["nnz"]
        mu1 = np.zeros(K)
        rho = np.zeros(nnz)
        rho1 = np.zeros((K, nnz))
        rp = np.zeros(n_orb + 1, np.int32)
        col = np.zeros(nnz, np.int32)
        _check(lib().gq_server_fetch(self.h, int(rid), mu1.ctypes.data, rho.ctypes.data,
                                     rho1.ctypes.data, rp.ctypes.data, col.ctypes.data))
        return {"mu1": mu1, "rho": rho, "rho1": rho1, "rho_row_ptr": rp, "rho_col": col}

    def release(self, rid):
        _check(lib().gq_server_release(self.h, int(rid)))

    def clock(self):
        return lib().gq_server_clock(self.h)

    def arena_used(self):
        used, size = C.c_int64(), C.c_int64()
        _check(lib().gq_server_arena_used(self.h, C.byref(used), C.byref(size)))
        return used.value, size.value

    def close(self, _rel=_release):
        _rel(self, "gq_server_destroy")

    def __del__(self):
        self.close()
