"""gq_response_static (the response entry point that allocates nothing, its
per-call buffers in the library's static device scratch) against gq_response,
through the C ABI: two calls in a row, the second on a smaller input, then a
system whose perturbations run in several chunks, the general (CSR) kind, and
the size limit.  The two entry points share every kernel, so the results must
agree bit for bit."""
import sys

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

pytestmark = pytest.mark.gpu

KT = 0.01


def _say(msg):
    print(f"[gpu-no-alloc] {msg}", flush=True)
    sys.stdout.flush()


def _pair(ctx, s, core, tau, prev, flags, h1, precision=0, general=False):
    """(gq_response, gq_response_static) outputs on one eigenbasis."""
    import torch
    from paper_2212_01997_amd.path import GraphPath
    K = len(h1) if isinstance(h1, list) else int(h1.shape[0])
    p = GraphPath(ctx, s, core, tau, prev, flags, max_k=K, general_h1=general)
    p.ground_state(KT)
    nnz = p.nnz
    ref_p = torch.empty(K * nnz, dtype=torch.float64, device="cuda")
    ref_m = torch.empty(K, dtype=torch.float64, device="cuda")
    p.eigs.response(h1, ref_p, precision, mu1_dev=ref_m, want_mu1=False)
    out_p = torch.full((K * nnz,), float("nan"), dtype=torch.float64, device="cuda")
    out_m = torch.full((K,), float("nan"), dtype=torch.float64, device="cuda")
    p.eigs.response_static(h1, out_p, precision, mu1_dev=out_m)
    torch.cuda.synchronize()
    return (ref_p.cpu().numpy(), ref_m.cpu().numpy()), (out_p.cpu().numpy(), out_m.cpu().numpy()), p


def _same(ref, out):
    assert np.array_equal(ref[1], out[1]), (ref[1], out[1])
    assert np.array_equal(ref[0], out[0]), float(np.nanmax(np.abs(ref[0] - out[0])))


@pytest.fixture(scope="module")
def ctx():
    from paper_2212_01997_amd import gq
    return gq.Context(0)


def test_two_calls_second_smaller(ctx, oracle_lib):
    import torch
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    h1 = torch.as_tensor(I.h1_diagonal(s, 3, seed=62), device="cuda")
    _say("water60 K=3 fp64")
    ref, out, _ = _pair(ctx, s, core, 0.07, prev, 1, h1)
    _same(ref, out)
    s1 = I.water32_system()
    c1 = I.single_atom_cores(s1)
    prev1 = O.bootstrap_prev(s1, c1, KT)
    h1b = torch.as_tensor(I.h1_diagonal(s1, 1, seed=1002), device="cuda")
    _say("water32 K=1 fp64 (smaller, after the larger)")
    ref, out, _ = _pair(ctx, s1, c1, 0.07, prev1, 1, h1b)
    _same(ref, out)
    _say("water32 K=1 split32")
    ref, out, _ = _pair(ctx, s1, c1, 0.07, prev1, 1, h1b, precision=1)
    _same(ref, out)


def test_general_kind(ctx, oracle_lib):
    from paper_2212_01997_amd import gq
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    mats = [gq.DeviceCsr(*m) for m in I.h1_on_pattern(s, 2, seed=63)]
    _say("water60 K=2 CSR")
    ref, out, _ = _pair(ctx, s, core, 0.07, prev, 1, mats, general=True)
    _same(ref, out)


def test_chunked_water1000(ctx):
    """The 1,000-water system: one perturbation's buffers fill most of the
    scratch, so K = 2 runs as two chunks of one."""
    import torch
    from paper_2212_01997_amd.path import bootstrap_prev
    s = I.water1000_system()
    core = I.spatial_cores(s, 8)
    prev = bootstrap_prev(ctx, s, core, KT)
    h1 = torch.as_tensor(I.h1_diagonal(s, 2, seed=2002), device="cuda")
    _say("water1000 K=2 (chunked)")
    ref, out, _ = _pair(ctx, s, core, 0.07, prev, 1, h1)
    _same(ref, out)


def test_size_limit(ctx):
    """34 subgraphs of 1,020 orbitals: sum n^2 = 3.5e7 doubles is beyond the
    scratch, and the call says so."""
    import torch
    from paper_2212_01997_amd import gq
    from paper_2212_01997_amd.path import GraphPath
    s = I.water_system(170, 17.2, seed=171)
    core = (np.arange(s.n_atoms) // 15).astype(np.int32)
    p = GraphPath(ctx, s, core, 0.0, None, 2, max_k=1)
    p.ground_state(KT, want_mu=False)
    h1 = torch.zeros((1, s.n_orb), dtype=torch.float64, device="cuda")
    with pytest.raises(gq.GQError, match="static scratch holds"):
        p.eigs.response_static(h1, p.p_blocks)
    torch.cuda.synchronize()
