#!/usr/bin/env python3
"""Benchmark of the graph-based density + canonical response path on one MI355X.

A step is one pass of the whole path over the 1,000-water system (3,000 atoms,
6,000 orbitals, 8-atom spatial cores, graph = paths of two of the thresholded
previous density and Hamiltonian at tau = 0.07, kT = 0.01 Ha):
gather + FP64 eigensolve of every subgraph, shared mu, density core rows,
mu-response rows, divided differences, the response to one diagonal H1 with
its canonical mu1, and the collect of rho and rho1.  The graph estimate is
built on the host from the previous-step density before the timed region and
timed on its own (graph_build_ms).

Prints one JSON line.  Options: --steps K --warmup W --gpus N (1 only)
--no-cpu-baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "response solves/s, mixed & served vs FP64 at ‖Δρ1‖≤1e-6; p50/p99 latency"
KT = 0.01
TAU = 0.07
PEAK_FP64 = 78.6e12     # MI355X FP64 (vector = MFMA), FLOP/s
PEAK_HBM = 8.0e12       # B/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_work(sizes, cores):
    """Algorithmic flops of each kernel per step (sum over subgraphs)."""
    n = sizes.astype(float)
    c = cores.astype(float)
    return {
        "k_tridiag": (4.0 / 3.0 * n ** 3).sum(),
        "k_formq": (4.0 / 3.0 * n ** 3).sum(),
        "k_ql": (6.0 * n ** 3).sum(),
        "k_density_rows": (4.0 * c * n ** 2).sum(),
        "k_xy": (n ** 3 + n ** 2).sum(),
        "k_rows": (4.0 * c * n ** 2).sum(),
        "eigensolve_9n3": (9.0 * n ** 3).sum(),
    }


def tridiag_bytes(sizes):
    """Algorithmic HBM bytes of k_tridiag per step (Sec. II.D eigensolve,
    one-stage Householder reduction): for every column c the symmetric product
    reads the trailing matrix (rows and columns > c) once, and every panel of
    16 reflectors reads and writes the trailing matrix once in its rank-2x16
    update; 8 bytes per FP64 element."""
    total = 0.0
    for n in sizes.astype(int):
        m = n - 1
        symv = m * (m + 1) * (2 * m + 1) / 6.0 - 1.0 if n >= 3 else 0.0  # sum_{c<=n-3} (n-c-1)^2
        upd = 0.0
        k0 = 0
        while k0 + 2 < n:
            t0 = k0 + min(16, n - 2 - k0)
            upd += 2.0 * (n - t0) ** 2
            k0 += 16
        total += 8.0 * (symv + upd)
    return total


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel factor), or None
    when the kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic_water1000.txt")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("{"):
                rec = json.loads(line)
    if not rec or kernel not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][kernel]
    src = os.path.join(ROOT, "paper_2212_01997_amd", "csrc", k["source"])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != k["sha256_16"]:
            return None
    return k["bytes_per_launch"]


def cpu_baseline(system, core, h1, budget_s=12.0):
    """The oracle as it stands, single-threaded, on a size-stratified sample of
    subgraphs of its own graph (its own bootstrap density); extrapolated to the
    whole step by sum n^3."""
    import numpy as np
    from oracle import oracle as O
    prev = O.bootstrap_prev(system, core, KT, pool=True)
    g = O.graph_build(system, core, TAU, rho_prev=prev, flags=O.PATHS2)
    sizes = g.sizes()
    H = O.Csr(system.h_row_ptr, system.h_col, system.h_val)
    # size-stratified order: quantiles first, then the rest, until the budget is spent
    order = np.argsort(sizes)
    first = [int(order[min(len(order) - 1, int(f * len(order)))])
             for f in (0.5, 0.95, 0.05, 0.75, 0.25, 0.99, 0.01, 0.6, 0.4, 0.85, 0.15)]
    rest = [int(x) for x in np.random.default_rng(0).permutation(g.n_sub)]
    picks = list(dict.fromkeys(first + rest))
    t_used, n3_used, done = 0.0, 0.0, 0
    mu = -0.22
    for s in picks:
        t0 = time.perf_counter()
        orbs = g.orbs(s)
        c = int(g.n_core_orbs[s])
        e, z = O.eigh(O.gather(H, orbs))
        O.core_rows(z, e, c, mu, KT)
        O.mu_response_rows(z, e, c, mu, KT)
        dF = O.divided_differences(e, mu, KT)
        O.lambda_response_rows(z, dF, np.diag(h1[0, orbs]), c)
        t_used += time.perf_counter() - t0
        n3_used += float(len(orbs)) ** 3
        done += 1
        if t_used > budget_s and done >= 3:
            break
    total = t_used / n3_used * float((sizes.astype(float) ** 3).sum())
    return {
        "value": 1.0 / total,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{done} of {g.n_sub} subgraphs (size-stratified, n {int(min(sizes[p] for p in picks[:done]))}"
                   f"..{int(max(sizes[p] for p in picks[:done]))}), single thread, {t_used:.1f} s of"
                   f" gather + eigensolve + density rows + response rows; whole-step time"
                   f" extrapolated by sum n^3 to {total:.1f} s"),
    }


# ------------------------------------------------------------ the three forms
def _time_ms(fn, sync, reps=3):
    """Best of `reps` wall-clock runs of fn, bracketed by `sync`."""
    best = 1e30
    for _ in range(reps):
        sync()
        t0 = time.perf_counter()
        fn()
        sync()
        best = min(best, time.perf_counter() - t0)
    return best * 1e3


def _golden3():
    path = os.path.join(ROOT, "tests", "golden", "config3_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _digest(a):
    import hashlib
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a, np.int32).tobytes()).hexdigest()[:16]


def form_batched_and_mixed(ctx, side):
    """Config 3 (30,000-atom chain in water, K = 6 perturbations per
    eigenbasis): the plain batched FP64 path against the autotuned,
    size-binned, graph-captured one; then the split-FP32 congruences at
    kT = 0.003, 0.01, 0.03 with their errors against the FP64 path (whole
    system) and against the stored oracle values (sampled positions)."""
    import numpy as np
    import torch
    from paper_2212_01997_amd import gq, inputs as I
    from paper_2212_01997_amd.path import GraphPath, bootstrap_prev
    K = 6
    log("config 3: generating the 30,000-atom system")
    s = I.config_system(3)
    core = I.spatial_cores(s, 8)
    prev = bootstrap_prev(ctx, s, core, KT)
    graph = gq.Graph.for_system(s, core, TAU, prev, gq.PATHS2)
    info = graph.info
    path = GraphPath(ctx, s, core, TAU, graph=graph, max_k=K)
    h1 = torch.as_tensor(I.h1_diagonal(s, K, seed=3002), device="cuda")
    torch.cuda.synchronize()
    sync = side.synchronize
    out = {"workload": "config 3: 30,000 atoms (6,000-atom C/N/O/S chain in water), 72,000 "
                       "orbitals, 8-atom cores, paths of two at tau 0.07, K = 6 diagonal H1",
           "n_sub": info.n_sub, "n_min": info.min_n, "n_max": info.max_n, "nnz": info.nnz}
    # plain: default launch variant, eager launches
    for b in range(5):
        graph.set_launch(0, b, 0)
        graph.set_launch(1, b, 0)
    path.ground_state(KT, want_mu=False)
    g_ms = _time_ms(lambda: path.ground_state(KT, want_mu=False), sync)
    r_ms = _time_ms(lambda: path.respond(h1, want_mu1=False), sync)
    out["plain"] = {"ground_state_ms": g_ms, "response_ms_K6": r_ms,
                    "response_solves_per_s": K * 1e3 / r_ms,
                    "step_ms": g_ms + r_ms, "step_solves_per_s": K * 1e3 / (g_ms + r_ms)}
    # the congruence kernel at K = 6 (two perturbations per workgroup), timed
    # with the library's hipEvent pairs on its own stream
    ctx.set_profiling(True)
    for _ in range(3):
        path.respond(h1, want_mu1=False)
    sync()
    kt = ctx.kernel_times()
    ctx.set_profiling(False)
    if "k_xy" in kt:
        n3 = np.diff(graph.export()["sub_orb_ptr"]).astype(float)
        flops = K * float((n3 ** 3 + n3 ** 2).sum())
        xy_ms = kt["k_xy"][1] / kt["k_xy"][0]
        out["congruence_roofline_K6"] = {
            "bound": "mfma", "kernel": "k_xy", "achieved": flops / (xy_ms * 1e-3) / 1e12,
            "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
            "frac": flops / (xy_ms * 1e-3) / PEAK_FP64,
            "algorithmic_flops_per_launch": flops, "launch_ms": xy_ms}
    # batched: autotuned bins + one captured graph per step
    report = path.eigs.autotune(gq.PREC_FP64)
    ctx.capture_begin()
    path.respond(h1, want_mu1=False)
    x_resp = ctx.capture_end()
    ctx.capture_begin()
    path.ground_state(KT, want_mu=False)
    path.respond(h1, want_mu1=False)
    x_step = ctx.capture_end()
    rb_ms = _time_ms(x_resp.launch, sync)
    sb_ms = _time_ms(x_step.launch, sync)
    out["batched"] = {"response_ms_K6": rb_ms, "response_solves_per_s": K * 1e3 / rb_ms,
                      "step_ms": sb_ms, "step_solves_per_s": K * 1e3 / sb_ms,
                      "speedup_response_vs_plain": r_ms / rb_ms,
                      "speedup_step_vs_plain": (g_ms + r_ms) / sb_ms,
                      "autotune": [ln for ln in report.splitlines() if "->" in ln]}
    del x_resp, x_step
    # mixed precision at three temperatures
    gold = _golden3()
    ex = graph.export()
    gold_ok = gold is not None and all(
        gold["graph"][k] == _digest(ex[k]) for k in ("sub_orb_ptr", "sub_orbs", "rho_row_ptr", "rho_col"))
    path.eigs.autotune(gq.PREC_SPLIT32)
    mixed = []
    for kT in (0.003, 0.01, 0.03):
        mu = path.ground_state(kT)
        path.sync()
        mu1_64 = path.respond(h1)
        path.sync()
        rho = path.rho.clone()
        rho1_64 = path.rho1_view(K).clone()
        t64 = _time_ms(lambda: path.respond(h1, want_mu1=False), sync)
        mu1_32 = path.respond(h1, precision=gq.PREC_SPLIT32)
        path.sync()
        rho1_32 = path.rho1_view(K).clone()
        t32 = _time_ms(lambda: path.respond(h1, precision=gq.PREC_SPLIT32, want_mu1=False), sync)
        row = {"kT": kT, "fp64_response_ms_K6": t64, "split32_response_ms_K6": t32,
               "speedup": t64 / t32,
               "split32_vs_fp64_path": {"rho1": float((rho1_32 - rho1_64).abs().max()),
                                        "mu1": float(np.abs(mu1_32 - mu1_64).max())}}
        if gold_ok:
            g = gold["kT"][repr(kT)]
            idx = torch.as_tensor(np.array(gold["idx"]), device="cuda")
            r_or = np.array(g["rho1"])
            row["vs_oracle_sampled"] = {
                "positions": len(gold["idx"]),
                "mu": abs(mu - g["mu"]),
                "rho": float(np.abs(rho[idx].cpu().numpy() - np.array(g["rho"])).max()),
                "fp64": {"rho1": float(np.abs(rho1_64[:, idx].cpu().numpy() - r_or).max()),
                         "mu1": float(np.abs(mu1_64 - np.array(g["mu1"])).max())},
                "split32": {"rho1": float(np.abs(rho1_32[:, idx].cpu().numpy() - r_or).max()),
                            "mu1": float(np.abs(mu1_32 - np.array(g["mu1"])).max())}}
        mixed.append(row)
        log(f"mixed kT={kT}: fp64 {t64:.2f} ms, split32 {t32:.2f} ms, "
            f"|drho1| {row['split32_vs_fp64_path']['rho1']:.2e}")
    out["mixed"] = mixed
    out["oracle_values"] = ("stored oracle values at 4,096 sampled positions (tests/golden)"
                            if gold_ok else "not compared (stored oracle values missing or for another graph)")
    return out


def form_served(ctx, side, n_slots=4):
    """Config 5: a Poisson trace (20 requests/s, 200 requests, 500..20,000
    atoms, K = 1..8) served by the runtime, against the same trace run one
    request after another on the plain path (FIFO, same arrival times)."""
    import threading
    import numpy as np
    import torch
    from paper_2212_01997_amd import gq, inputs as I
    from paper_2212_01997_amd.path import GraphPath, bootstrap_prev
    tr = I.serving_trace()
    systems = []
    for k, spec in enumerate(tr.pool):
        systems.append(I.pool_system(*spec))
        log(f"config 5: pool system {k + 1}/{len(tr.pool)}: {spec[0]}, {systems[-1].n_atoms} atoms")
    cores = [I.spatial_cores(s, 8) for s in systems]
    prevs = [bootstrap_prev(ctx, s, c, KT) for s, c in zip(systems, cores)]
    h1s = [I.h1_diagonal(systems[i], int(k), seed=int(sd))
           for i, k, sd in zip(tr.system, tr.K, tr.h1_seed)]
    n = len(tr.arrival)
    solves = int(tr.K.sum())
    # sequential plain path
    log("config 5: sequential plain path")
    lat_seq = np.zeros(n)
    t0 = time.perf_counter()
    for j in range(n):
        now = time.perf_counter() - t0
        if now < tr.arrival[j]:
            time.sleep(tr.arrival[j] - now)
        i = int(tr.system[j])
        p = GraphPath(ctx, systems[i], cores[i], TAU, prevs[i], gq.PATHS2, max_k=int(tr.K[j]))
        p.ground_state(KT, want_mu=False)
        p.respond(torch.as_tensor(h1s[j], device="cuda"), want_mu1=False)
        side.synchronize()
        rho1 = p.rho1.cpu()  # results to the host, as the server returns them
        del rho1
        lat_seq[j] = time.perf_counter() - t0 - tr.arrival[j]
        del p
        if (j + 1) % 50 == 0:
            log(f"config 5: sequential {j + 1}/{n}")
    span_seq = time.perf_counter() - t0
    torch.cuda.empty_cache()
    # served
    log("config 5: served")
    srv = gq.Server(0, n_slots=n_slots, arena_bytes=96 << 30)
    ids = [None] * n
    start = srv.clock()

    def feeder():
        for j in range(n):
            now = srv.clock() - start
            if now < tr.arrival[j]:
                time.sleep(tr.arrival[j] - now)
            i = int(tr.system[j])
            ids[j] = srv.submit(systems[i], cores[i], TAU, prevs[i], gq.PATHS2, KT, h1s[j])

    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    log("config 5: all requests submitted")
    infos = [srv.wait(rid) for rid in ids]
    log("config 5: all requests served")
    lat_srv = np.array([inf["t_done"] - (start + tr.arrival[j]) for j, inf in enumerate(infos)])
    span_srv = max(inf["t_done"] for inf in infos) - start
    srv.close()
    return {"workload": f"config 5: {n} requests, Poisson 20/s, {len(tr.pool)} seeded pool systems "
                        f"of 500..20,000 atoms (log-uniform; water or chain-in-water), K = 1..8 "
                        f"({solves} solves), kT 0.01, paths of two at tau 0.07",
            "served": {"slots": n_slots, "p50_ms": float(np.percentile(lat_srv, 50) * 1e3),
                       "p99_ms": float(np.percentile(lat_srv, 99) * 1e3),
                       "solves_per_s": solves / span_srv, "makespan_s": span_srv},
            "sequential_plain": {"p50_ms": float(np.percentile(lat_seq, 50) * 1e3),
                                 "p99_ms": float(np.percentile(lat_seq, 99) * 1e3),
                                 "solves_per_s": solves / span_seq, "makespan_s": span_seq}}



def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched (config 3), mixed (config 4) and served (config 5) forms")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one device copy of 256 MiB (reference for byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU path "
              "(the multi-GPU sharding is described, not run).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2212_01997_amd import gq, inputs as I
    from paper_2212_01997_amd.path import GraphPath, bootstrap_prev

    log("building the 1,000-water system")
    system = I.config_system(2)
    core = I.spatial_cores(system, 8)
    h1_host = I.h1_diagonal(system, 1, seed=2002)
    side = torch.cuda.Stream()  # a stream of its own, so that whole steps can be captured
    ctx = gq.Context(0, stream=side)
    log("previous-step density on the Hamiltonian graph")
    prev = bootstrap_prev(ctx, system, core, KT)
    gb = []
    for _ in range(3):
        t0 = time.perf_counter()
        graph = gq.Graph.for_system(system, core, TAU, prev, gq.PATHS2)
        gb.append((time.perf_counter() - t0) * 1e3)
    info = graph.info
    ex = graph.export()
    sizes = np.diff(ex["sub_orb_ptr"])
    cores_n = ex["n_core_orbs"]
    log(f"graph: {info.n_sub} subgraphs, n {info.min_n}..{info.max_n}, nnz {info.nnz}")
    path = GraphPath(ctx, system, core, TAU, graph=graph, max_k=1)
    h1 = torch.as_tensor(h1_host, device="cuda")

    def step():
        path.ground_state(KT, want_mu=False)
        path.respond(h1, want_mu1=False)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms:.3f} ms/step")

    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 268435456 bytes read, 268435456 bytes written")

    # per-kernel durations, measured with hipEvents on the library stream
    ctx.set_profiling(True)
    nprof = max(2, min(5, args.steps))
    for _ in range(nprof):
        step()
    kt = ctx.kernel_times()
    ctx.set_profiling(False)
    per_step = {k: v[1] / nprof for k, v in kt.items()}
    per_launch = {k: v[1] / v[0] for k, v in kt.items()}
    work = algorithmic_work(sizes, cores_n)
    dominant = max(per_step, key=per_step.get)
    # work per step over the kernel's summed launch durations per step, which
    # is work per launch over the average launch duration when the launches
    # share the work evenly (the eigensolve launches k_tridiag once per size
    # class, on two streams, so their durations overlap and this understates)
    launches_per_step = kt[dominant][0] / nprof
    flops = work.get(dominant, 0.0) / launches_per_step
    launch_s = per_launch[dominant] * 1e-3
    achieved = flops / launch_s if flops else 0.0
    if dominant == "k_tridiag":
        # BLAS-2 bound: the symmetric product streams the trailing matrix once
        # per column, so the roofline is HBM with the algorithm's own bytes
        nbytes = tridiag_bytes(sizes) / launches_per_step
        roofline = {"bound": "hbm", "kernel": dominant, "achieved": nbytes / launch_s / 1e9,
                    "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": nbytes / launch_s / PEAK_HBM,
                    "traffic": measured_traffic(dominant),
                    "algorithmic_bytes_per_launch": nbytes,
                    "algorithmic_flops_per_launch": flops, "achieved_tflops": achieved / 1e12,
                    "launch_ms": per_launch[dominant], "launches_per_step": launches_per_step}
    else:
        bound = "alu" if dominant in ("k_dc_prep", "k_dc_leaves") else "mfma"
        roofline = {"bound": bound, "kernel": dominant, "achieved": achieved / 1e12,
                    "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
                    "traffic": measured_traffic(dominant),
                    "algorithmic_flops_per_launch": flops, "launch_ms": per_launch[dominant],
                    "launches_per_step": launches_per_step}
    xy_flops = work["k_xy"]
    xy_ms = per_launch.get("k_xy", 0.0)
    roofline_congruence = None
    if xy_ms:
        a = xy_flops / (xy_ms * 1e-3)
        roofline_congruence = {"bound": "mfma", "kernel": "k_xy", "achieved": a / 1e12,
                               "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": a / PEAK_FP64,
                               "traffic": measured_traffic("k_xy"),
                               "algorithmic_flops_per_launch": xy_flops, "launch_ms": xy_ms}
    phases = {k: round(v, 4) for k, v in sorted(per_step.items(), key=lambda x: -x[1])}
    eig_ms = sum(v for k, v in per_step.items() if k in ("k_gather", "k_tridiag") or k.startswith(("k_dc", "k_back")))
    resp_ms = sum(per_step.get(k, 0) for k in ("k_xy", "k_rows", "k_mu1_combine"))
    dens_ms = sum(per_step.get(k, 0) for k in ("k_mu", "k_density_rows", "k_divided_differences"))
    line = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "1,000 waters (3,000 atoms, 6,000 orbitals, 31 A box, seed 2001); "
                        "8-atom Morton cores; graph = paths of two of thr(rho_prev) u thr(H), "
                        "tau 0.07; kT 0.01 Ha; one diagonal H1 per solve",
            "n_sub": info.n_sub, "n_min": info.min_n, "n_max": info.max_n,
            "n_mean": float(sizes.mean()), "nnz": info.nnz, "K": 1,
            "precision": "fp64",
        },
        "phase_ms": {"eigensolve": eig_ms, "density": dens_ms, "response": resp_ms,
                     "assemble": per_step.get("k_assemble", 0.0),
                     "graph_build_host": float(np.median(gb)),
                     "note": "device phases are summed kernel durations; the eigensolve's two "
                             "streams overlap, so its sum exceeds its share of ms_per_step"},
        "kernel_ms_per_step": phases,
        "elements_per_s": info.nnz * 1000.0 / ms,
        "response_only_solves_per_s": 1000.0 / resp_ms if resp_ms else None,
        "roofline": roofline,
        "roofline_congruence": roofline_congruence,
    }
    if not args.no_forms:
        forms = {}
        forms["batched_and_mixed"] = form_batched_and_mixed(ctx, side)
        torch.cuda.empty_cache()
        forms["served"] = form_served(ctx, side)
        line["forms"] = forms
    if not args.no_cpu_baseline:
        log("oracle CPU baseline on a sample of subgraphs")
        from oracle import oracle as O
        O.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
        line["cpu_baseline"] = cpu_baseline(system, core, h1_host)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
