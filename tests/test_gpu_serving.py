"""The serving runtime (gq_server_*): results through the server equal the
oracle; each request gives the same result alone and in a mix of concurrent
requests; admission follows the arena footprint.
"""
import sys

import numpy as np
import pytest

from paper_2212_01997_amd import inputs as I

pytestmark = pytest.mark.gpu

KT = 0.01


def _say(msg):
    print(f"[gpu-serving] {msg}", flush=True)
    sys.stdout.flush()


def _requests(ctx):
    """Six systems of different kinds and sizes, each with its own K."""
    from paper_2212_01997_amd.path import bootstrap_prev
    specs = [("water", 60, 12.2, 1), ("chain", 900, 180, 3), ("water", 200, 18.3, 2),
             ("water", 100, 14.6, 4), ("chain", 1500, 300, 2), ("water", 400, 23.0, 1)]
    out = []
    for i, (kind, a, b, K) in enumerate(specs):
        if kind == "water":
            s = I.water_system(a, b, seed=700 + i)
        else:
            s = I.chain_water_system(a, b, seed=700 + i)
        core = I.spatial_cores(s, 8)
        prev = bootstrap_prev(ctx, s, core, KT)
        h1 = I.h1_diagonal(s, K, seed=800 + i)
        out.append((s, core, prev, h1))
    return out


@pytest.fixture(scope="module")
def ctx():
    from paper_2212_01997_amd import gq
    return gq.Context(0)


def test_server_matches_oracle(oracle_lib):
    from paper_2212_01997_amd import gq
    O = oracle_lib
    s = I.water32_system()
    core = I.single_atom_cores(s)
    prev = O.bootstrap_prev(s, core, KT)
    h1 = I.h1_diagonal(s, 2, seed=1002)
    g = O.graph_build(s, core, 0.07, rho_prev=prev, flags=O.PATHS2)
    r = O.solve(s, g, KT, h1)
    srv = gq.Server(0, n_slots=2, arena_bytes=1 << 30)
    try:
        for precision, tol in ((0, 1e-10), (1, 1e-6)):
            rid = srv.submit(s, core, 0.07, prev, gq.PATHS2, KT, h1, precision)
            info = srv.wait(rid)
            res = srv.fetch(rid, info, s.n_orb)
            srv.release(rid)
            assert np.array_equal(res["rho_row_ptr"], g.rho_row_ptr)
            assert np.array_equal(res["rho_col"], g.rho_col)
            assert abs(info["mu"] - r.mu) <= 1e-12
            assert np.abs(res["rho"] - r.rho).max() <= 1e-10
            assert np.abs(res["mu1"] - r.mu1).max() <= tol
            assert np.abs(res["rho1"] - r.rho1).max() <= tol
    finally:
        srv.close()


def test_alone_equals_mix(ctx):
    """Each request alone on an idle server, then all six submitted at once to
    four slots: every result is the same (bit for bit, so within any
    tolerance), FP64 and split-FP32."""
    from paper_2212_01997_amd import gq
    reqs = _requests(ctx)
    for precision in (0, 1):
        alone = []
        srv = gq.Server(0, n_slots=1, arena_bytes=8 << 30)
        try:
            for s, core, prev, h1 in reqs:
                rid = srv.submit(s, core, 0.07, prev, gq.PATHS2, KT, h1, precision)
                info = srv.wait(rid)
                alone.append((info, srv.fetch(rid, info, s.n_orb)))
                srv.release(rid)
        finally:
            srv.close()
        srv = gq.Server(0, n_slots=4, arena_bytes=8 << 30)
        try:
            ids = [srv.submit(s, core, 0.07, prev, gq.PATHS2, KT, h1, precision)
                   for s, core, prev, h1 in reqs]
            mix = []
            for rid, (s, *_rest) in zip(ids, reqs):
                info = srv.wait(rid)
                mix.append((info, srv.fetch(rid, info, s.n_orb)))
            admits = sorted(info["t_admit"] for info, _ in mix)
            dones = sorted(info["t_done"] for info, _ in mix)
            _say(f"precision {precision}: admitted {admits}, done {dones}")
            # overlap: some request was admitted before another one finished
            assert any(info_a["t_admit"] < info_b["t_done"] and info_b["t_admit"] < info_a["t_done"]
                       for i, (info_a, _) in enumerate(mix) for info_b, _ in mix[i + 1:])
        finally:
            srv.close()
        for (ia, ra), (im, rm) in zip(alone, mix):
            assert ia["mu"] == im["mu"]
            for key in ("mu1", "rho", "rho1", "rho_col"):
                assert np.array_equal(ra[key], rm[key]), key
            tol = 1e-10 if precision == 0 else 1e-6
            assert np.abs(ra["rho1"] - rm["rho1"]).max() <= tol


def test_admission_by_footprint(ctx):
    """An arena that holds about one request at a time still serves them all
    (in turn); a request larger than the arena fails with GQ_ENOMEM."""
    from paper_2212_01997_amd import gq
    all_reqs = _requests(ctx)
    reqs = all_reqs[:4]
    graphs = [gq.Graph.for_system(s, core, 0.07, prev, gq.PATHS2) for s, core, prev, _ in reqs]
    fps = [g.footprint(h1.shape[0]) for g, (_s, _c, _p, h1) in zip(graphs, reqs)]
    arena = int(max(fps) * 1.6)
    big_s, big_core, big_prev, _ = all_reqs[4]
    big_h1 = I.h1_diagonal(big_s, 8, seed=5)
    big_g = gq.Graph.for_system(big_s, big_core, 0.07, big_prev, gq.PATHS2)
    assert big_g.footprint(8) > arena
    srv = gq.Server(0, n_slots=4, arena_bytes=arena)
    try:
        ids = [srv.submit(s, core, 0.07, prev, gq.PATHS2, KT, h1)
               for s, core, prev, h1 in reqs]
        infos = [srv.wait(rid) for rid in ids]
        for info in infos:
            assert info["status"] == 0 and info["footprint"] <= arena
        # at no time did the admitted requests exceed the arena
        events = sorted([(i["t_admit"], i["footprint"]) for i in infos] +
                        [(i["t_done"], -i["footprint"]) for i in infos])
        live = 0
        for _, d in events:
            live += d
            assert live <= arena
        rid = srv.submit(big_s, big_core, 0.07, big_prev, gq.PATHS2, KT, big_h1)
        with pytest.raises(gq.GQError, match="arena"):
            srv.wait(rid)
    finally:
        srv.close()
