"""The whole path on one GPU through the C ABI (marshalling only).

    graph_build -> submatrix_solve -> density -> response -> assemble

Buffers are torch tensors on the context's device; every arithmetic step runs
in libgq's HIP kernels.
"""
from __future__ import annotations

import numpy as np

from . import gq


class GraphPath:
    """Device state of one system on one graph, reusable across perturbations."""

    def __init__(self, ctx: gq.Context, system, core_of_atom, tau, rho_prev=None, flags=0,
                 max_k=1, graph: gq.Graph | None = None, H: gq.DeviceCsr | None = None,
                 general_h1=False, S=None):
        """S: an overlap matrix (host CSR triple) for a non-orthogonal basis, or
        None; with it the densities and responses are atomic-orbital rows."""
        import torch
        self.ctx = ctx
        self.system = system
        self.graph = graph or gq.Graph.for_system(system, core_of_atom, tau, rho_prev, flags)
        self.H = H or gq.DeviceCsr(system.h_row_ptr, system.h_col, system.h_val, ctx.device)
        self.S = None if S is None else gq.DeviceCsr(*S, device=ctx.device)
        self.eigs = gq.Eigs(ctx, self.graph, max_k, general_h1=general_h1, overlap=S is not None)
        nnz = self.graph.info.nnz
        dev = torch.device("cuda", ctx.device)
        self.max_k = max_k
        self.rho_blocks = torch.empty(nnz, dtype=torch.float64, device=dev)
        self.rho = torch.empty(nnz, dtype=torch.float64, device=dev)
        self.p_blocks = torch.empty(max_k * nnz, dtype=torch.float64, device=dev)
        self.rho1 = torch.empty(max_k * nnz, dtype=torch.float64, device=dev)
        self.mu1_dev = torch.empty(max_k, dtype=torch.float64, device=dev)
        # the context may run on a stream of its own: inputs and buffers made on
        # torch's stream are complete before the library's first call
        torch.cuda.synchronize(dev)

    @property
    def nnz(self):
        return self.graph.info.nnz

    def ground_state(self, kT, n_elec=None, want_mu=True, mu_guess=None):
        """submatrix_solve + density (warm-started from mu_guess, if given) +
        assemble(rho)."""
        ne = self.system.n_elec if n_elec is None else n_elec
        if self.S is None:
            self.eigs.solve(self.H)
        else:
            self.eigs.solve_overlap(self.H, self.S)
        mu = self.eigs.density(kT, ne, self.rho_blocks, want_mu=want_mu, mu_guess=mu_guess)
        gq.assemble(self.ctx, self.graph, self.rho_blocks, self.rho, 1)
        return mu

    def purified_state(self, mu, max_iter=60, tol=1e-11):
        """Zero-temperature density by recursive expansion (purify +
        assemble(rho)) at the given mu; returns the iterations run.  The
        eigenbasis is overwritten: ground_state again before a response."""
        it = self.eigs.purify(self.H, mu, self.rho_blocks, max_iter=max_iter, tol=tol)
        gq.assemble(self.ctx, self.graph, self.rho_blocks, self.rho, 1)
        return it

    def respond(self, h1, precision=gq.PREC_FP64, want_mu1=True):
        """response + assemble(rho1) for K perturbations: a [K, N] tensor of
        diagonals or a list of K DeviceCsr matrices."""
        K = len(h1) if isinstance(h1, (list, tuple)) else int(h1.shape[0])
        mu1 = self.eigs.response(h1, self.p_blocks[:K * self.nnz], precision,
                                 mu1_dev=self.mu1_dev[:K], want_mu1=want_mu1)
        gq.assemble(self.ctx, self.graph, self.p_blocks[:K * self.nnz], self.rho1[:K * self.nnz], K)
        return mu1

    def sync(self):
        """Wait for the work enqueued on the context's stream."""
        self.ctx.stream.synchronize()

    def rho1_view(self, K):
        return self.rho1[:K * self.nnz].view(K, self.nnz)


def bootstrap_prev(ctx, system, core_of_atom, kT):
    """Previous-step density for the graph estimate: one pass of the path on
    the graph of every nonzero of H.  Returns the host CSR triple."""
    p = GraphPath(ctx, system, core_of_atom, 0.0)
    p.ground_state(kT, want_mu=False)
    p.sync()
    ex = p.graph.export()
    vals = p.rho.cpu().numpy()
    return ex["rho_row_ptr"], ex["rho_col"], vals


def collected_rows(graph_export):
    rp = graph_export["rho_row_ptr"]
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))
