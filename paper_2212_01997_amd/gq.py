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


# every symbol declared in include/gq.h, with its ctypes signature
_VP = C.c_void_p
_SIGS = {
    "gq_last_error": ([], C.c_char_p),
    "gq_version": ([], C.c_char_p),
    "gq_ctx_create": ([C.c_int32, _VP, C.POINTER(_VP)], C.c_int32),
    "gq_ctx_destroy": ([_VP], None),
    "gq_graph_build": ([C.c_int32, _VP, C.POINTER(_Csr), C.POINTER(_Csr), _VP, C.c_double,
                        C.c_uint32, C.POINTER(_VP)], C.c_int32),
    "gq_graph_query": ([_VP, C.POINTER(_Info)], C.c_int32),
    "gq_graph_export": ([_VP] + [_VP] * 8, C.c_int32),
    "gq_graph_block_offsets": ([_VP, _VP], C.c_int32),
    "gq_graph_destroy": ([_VP], None),
    "gq_eigs_create": ([_VP, _VP, C.c_int32, C.POINTER(_VP)], C.c_int32),
    "gq_eigs_footprint": ([_VP, C.c_int32, C.POINTER(C.c_int64)], C.c_int32),
    "gq_eigs_destroy": ([_VP], None),
    "gq_submatrix_solve": ([_VP, _VP, C.POINTER(_Csr), C.c_uint32, _VP], C.c_int32),
    "gq_density": ([_VP, _VP, C.c_double, C.c_double, _VP, _VP], C.c_int32),
    "gq_response": ([_VP, _VP, _VP, C.c_int32, C.c_uint32, _VP, _VP, _VP], C.c_int32),
    "gq_assemble": ([_VP, _VP, _VP, C.c_int32, _VP], C.c_int32),
    "gq_eigs_export": ([_VP, _VP, _VP, _VP], C.c_int32),
    "gq_eigs_vectors": ([_VP, C.c_int32, C.POINTER(_VP), C.POINTER(C.c_int32)], C.c_int32),
    "gq_ctx_set_profiling": ([_VP, C.c_int32], C.c_int32),
    "gq_ctx_kernel_times": ([_VP, _VP, _VP, _VP, C.c_int32, C.POINTER(C.c_int32)], C.c_int32),
}

_lib = None


def lib():
    """Load libgq.so; raises if it has not been built."""
    global _lib
    if _lib is None:
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


class Context:
    def __init__(self, device=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise GQError(-4, "no GPU visible")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = _VP()
        _check(lib().gq_ctx_create(device, _VP(self.stream.cuda_stream), C.byref(h)))
        self.h = h

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

    def __del__(self):
        if getattr(self, "h", None):
            lib().gq_ctx_destroy(self.h)
            self.h = None


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

    def footprint(self, max_k):
        b = C.c_int64()
        _check(lib().gq_eigs_footprint(self.h, int(max_k), C.byref(b)))
        return b.value

    def __del__(self):
        if getattr(self, "h", None):
            lib().gq_graph_destroy(self.h)
            self.h = None


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

    def __init__(self, ctx: Context, graph: Graph, max_k=1):
        self.ctx, self.graph, self.max_k = ctx, graph, max_k
        h = _VP()
        _check(lib().gq_eigs_create(ctx.h, graph.h, int(max_k), C.byref(h)))
        self.h = h

    def solve(self, H: DeviceCsr):
        s = H.cstruct()
        _check(lib().gq_submatrix_solve(self.ctx.h, self.graph.h, C.byref(s), 0, self.h))

    def density(self, kT, n_elec, rho_blocks=None, want_mu=True):
        mu = C.c_double()
        _check(lib().gq_density(self.ctx.h, self.h, float(kT), float(n_elec),
                                C.byref(mu) if want_mu else None, _ptr(rho_blocks)))
        return mu.value if want_mu else None

    def response(self, h1, p_blocks, precision=PREC_FP64, mu1_dev=None, want_mu1=True):
        K = int(h1.shape[0])
        host = (C.c_double * K)()
        _check(lib().gq_response(self.ctx.h, self.h, _ptr(h1), K, int(precision),
                                 _ptr(p_blocks), _ptr(mu1_dev), host if want_mu1 else None))
        return np.array(host[:]) if want_mu1 else None

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

    def __del__(self):
        if getattr(self, "h", None):
            lib().gq_eigs_destroy(self.h)
            self.h = None


def assemble(ctx: Context, graph: Graph, blocks, vals, K=1):
    _check(lib().gq_assemble(ctx.h, graph.h, _ptr(blocks), int(K), _ptr(vals)))
