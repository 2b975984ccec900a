"""The batched form of the path: size-binned X launches (every launch variant
gives bit-identical results), the autotuner, K perturbations per launch, and
HIP-graph capture of a whole step (every replay equal to the eager result).

Parity bar as in test_gpu_parity: rho, rho1, mu1 within 1e-10 of the oracle
on the FP64 path, rho1 and mu1 within 1e-6 on the split-FP32 path.
"""
import sys

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

pytestmark = pytest.mark.gpu

KT = 0.01


def _say(msg):
    print(f"[gpu-batching] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2212_01997_amd import gq
    return gq.Context(0)


@pytest.fixture(scope="module")
def water60(oracle_lib):
    O = oracle_lib
    s = I.water_system(60, 12.2, seed=61)
    core = I.spatial_cores(s, 8)
    prev = O.bootstrap_prev(s, core, KT)
    h1 = I.h1_diagonal(s, 3, seed=62)
    g = O.graph_build(s, core, 0.07, rho_prev=prev, flags=O.PATHS2)
    r = O.solve_pool(s, g, KT, h1)
    return s, core, prev, h1, r


def _path(ctx, s, core, prev, K, tau=0.07, flags=1):
    from paper_2212_01997_amd.path import GraphPath
    return GraphPath(ctx, s, core, tau, prev, flags, max_k=K)


def test_launch_variants_bit_identical(ctx):
    """1,000 waters (subgraphs of 153..383 orbitals: three size bins): every
    tile shape and grid of the X kernel gives the same bits, FP64 and split."""
    import torch
    from paper_2212_01997_amd.path import bootstrap_prev
    s = I.water1000_system()
    core = I.spatial_cores(s, 8)
    prev = bootstrap_prev(ctx, s, core, KT)
    K = 2
    p = _path(ctx, s, core, prev, K)
    h1 = torch.as_tensor(I.h1_diagonal(s, K, seed=2002), device="cuda")
    p.ground_state(KT)
    for precision in (0, 1):
        ref = None
        for variant in range(4):
            for b in range(5):
                p.graph.set_launch(precision, b, variant)
            mu1 = p.respond(h1, precision=precision)
            out = p.rho1_view(K).cpu().numpy().copy()
            _say(f"precision {precision} variant {variant}: mu1 {mu1}")
            if ref is None:
                ref = (out, mu1)
            else:
                assert np.array_equal(out, ref[0]) and np.array_equal(mu1, ref[1]), (precision, variant)
    for b in range(5):
        p.graph.set_launch(0, b, 0)
        p.graph.set_launch(1, b, 0)


def test_autotune_then_parity(ctx, water60):
    import torch
    s, core, prev, h1, r = water60
    K = h1.shape[0]
    p = _path(ctx, s, core, prev, K)
    p.ground_state(KT)
    for precision, tol in ((0, 1e-10), (1, 1e-6)):
        report = p.eigs.autotune(precision)
        _say(report)
        assert "->" in report
        mu1 = p.respond(torch.as_tensor(h1, device="cuda"), precision=precision)
        assert np.abs(mu1 - r.mu1).max() <= tol
        assert np.abs(p.rho1_view(K).cpu().numpy() - r.rho1).max() <= tol
    assert np.abs(p.rho.cpu().numpy() - r.rho).max() <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_capture_replay(water60, precision):
    """Ground state + K responses + assemble recorded once and replayed three
    times, with other eager work in between: every replay gives the eager bits."""
    import torch
    from paper_2212_01997_amd import gq
    s, core, prev, h1, r = water60
    K = h1.shape[0]
    side = torch.cuda.Stream()
    cx = gq.Context(0, stream=side)
    p = _path(cx, s, core, prev, K)
    h1d = torch.as_tensor(h1, device="cuda")
    h1b = torch.as_tensor(I.h1_diagonal(s, K, seed=99), device="cuda")
    torch.cuda.synchronize()

    def step(h):
        p.ground_state(KT, want_mu=False)
        p.respond(h, precision=precision, want_mu1=False)

    step(h1d)
    side.synchronize()
    ref_rho = p.rho.clone()
    ref_rho1 = p.rho1_view(K).clone()
    ref_mu1 = p.mu1_dev[:K].clone()
    torch.cuda.synchronize()
    tol = 1e-10 if precision == 0 else 1e-6
    assert np.abs(ref_rho1.cpu().numpy() - r.rho1).max() <= tol

    cx.capture_begin()
    with pytest.raises(gq.GQError, match="capturing"):
        p.eigs.density(KT, s.n_elec, p.rho_blocks, want_mu=True)
    step(h1d)
    x = cx.capture_end()
    for rep in range(3):
        p.rho.zero_()
        p.rho1.zero_()
        p.mu1_dev.zero_()
        torch.cuda.synchronize()
        x.launch()
        side.synchronize()
        assert torch.equal(p.rho, ref_rho), rep
        assert torch.equal(p.rho1_view(K), ref_rho1), rep
        assert torch.equal(p.mu1_dev[:K], ref_mu1), rep
        step(h1b)  # eager work with another perturbation between replays
        side.synchronize()
        assert not torch.equal(p.rho1_view(K), ref_rho1)
    del x


def test_grouped_perturbations_equal_single(ctx, water60):
    """K = 4 perturbations in one call (three per workgroup in the X kernel,
    the last one alone) give, bit for bit, what four K = 1 calls give, on the
    FP64 and the split-FP32 path."""
    import torch
    s, core, prev, h1, r = water60
    assert h1.shape[0] == 3
    h1 = np.concatenate([h1, (0.5 * h1[0] + h1[2])[None]])
    K = h1.shape[0]
    p = _path(ctx, s, core, prev, K)
    p.ground_state(KT)
    h1d = torch.as_tensor(h1, device="cuda")
    for precision in (0, 1):
        mu1_all = p.respond(h1d, precision=precision)
        all_rho1 = p.rho1_view(K).cpu().numpy().copy()
        for q in range(K):
            mu1_q = p.respond(h1d[q:q + 1].contiguous(), precision=precision)
            one = p.rho1_view(1).cpu().numpy()
            _say(f"precision {precision} q {q}: mu1 {mu1_q[0]!r} vs {mu1_all[q]!r}")
            assert np.array_equal(one[0], all_rho1[q]), (precision, q)
            assert mu1_q[0] == mu1_all[q], (precision, q)
