"""Benchmark: exact-BC TEPS (|S| * m / s) of Brandes++ and plain Brandes on one MI355X.

A step is one full Brandes++ pass over the workload: bc_partition_sk (P', frontiers,
Dijkstra_SK, skeleton assembly) then bc_brandes_pp_dev (Brandes_SK, then Centrality:
in the resident kernel, or for groups of 4 to 64 sources or many table rows in two
kernels of its own after it; scores written to a device tensor). The graph is resident on the
device before timing starts. Plain GPU Brandes on the same graph and targets is timed
the same way and reported beside it, with the CPU oracle on a bounded sample.

The default workload is pareto_100k: 100,000 nodes in 500 planted communities of
Pareto(2) sizes, mean degree 8, 85% intra-community edges, weights 1..4, 2,000 random
targets (Sec. 7's workload shape: random targets, community-structured graphs).

Prints one JSON line. Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                                             [--workload pareto_100k]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# source file of each kernel kind: measured HBM traffic is reported only while the
# kernel's source is the one the counters were taken on
KERNEL_SOURCES = {
    "resident": "paper_1406_4173_amd/csrc/resident.hip",
    "select": "paper_1406_4173_amd/csrc/engine.hip",
    "settle": "paper_1406_4173_amd/csrc/engine.hip",
    "push": "paper_1406_4173_amd/csrc/engine.hip",
    "backward": "paper_1406_4173_amd/csrc/engine.hip",
    # (the resident path's Centrality: the transpose and the interior sweep of split groups)
    "centrality": "paper_1406_4173_amd/csrc/resident.hip",
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs summarised in profiles/hbm_traffic.json (each counter scaled by its
    reading for a plain device copy of known size), or None when there is no entry or
    the kernel's source has changed since the counters were taken."""
    import hashlib

    try:
        with open(TRAFFIC_FILE) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return None
    ent = table.get(workload, {}).get(kernel)
    src = KERNEL_SOURCES.get(kernel)
    if not ent or not src:
        return None
    with open(os.path.join(ROOT, src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if sha != ent.get("source_sha256"):
        return None
    return float(ent["fetch_bytes_per_launch"]) + float(ent["write_bytes_per_launch"])


def roofline_entry(workload, kernel, kp, timing=None):
    """Roofline of one kernel kind from its profiler totals: algorithmic bytes per
    launch over the launch's average HIP-event duration, against the HBM peak; beside it
    the measured HBM traffic (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled) and its own
    fraction of the peak. `bound` comes from those counters: "hbm" when the measured
    traffic runs at half the peak or more, else "latency" (neither HBM nor ALU throughput
    is near its peak: the kernel waits on L2 and LDS round trips), or null without
    counters for the current source."""
    launches = max(kp["launches"], 1)
    avg_s = kp["ms"] * 1e-3 / launches
    alg = kp["alg_bytes"] / launches
    achieved = alg / avg_s / 1e9 if avg_s > 0 else 0.0
    traffic = measured_traffic(workload, kernel)
    mfrac = traffic / avg_s / 1e9 / PEAK_HBM_GBS if traffic and avg_s > 0 else None
    bound = None if mfrac is None else ("hbm" if mfrac >= 0.5 else "latency")
    r = {"kernel": kernel, "bound": bound, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
         "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "measured_frac": mfrac,
         "launches": kp["launches"], "avg_launch_us": avg_s * 1e6, "alg_bytes_per_launch": alg}
    if timing:
        r["timing"] = timing
    return r


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    # a process's first calls include a one-off stall of several ms (once, somewhere in
    # the first dozen calls, whatever the call pattern): warm up past it
    ap.add_argument("--warmup", type=int, default=15)
    ap.add_argument("--workload", default="pareto_100k",
                    choices=["planted_1k", "sbm_10k", "pareto_100k", "smallcut_100k", "batch_256", "p1_sweep",
                             "serve_64", "lp_pareto_100k", "pp_all_planted_1k"])
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="measured window of the serving workload (after a 2 s warm-up)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean query arrivals per second")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain Brandes line")
    ap.add_argument("--only-plain", action="store_true",
                    help="time plain Brandes alone (a profiling run of the plain pass; prints no line)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time budget of the oracle sample")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (a known-size "
                         "kernel that scales profiler byte counters)")
    return ap.parse_args()


def timed(fn, steps, warmup, sync):
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def cpu_baseline(g, budget_s):
    """The oracle as it stands, on the first sources of S, timed on the host: half the
    budget single-threaded, half on all host threads (up to 16), each thread one oracle
    call on a contiguous chunk of the sample (the C oracle keeps no global state and
    releases the GIL). TEPS over each sample; value is the all-threads rate."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    L = oracle.lib()
    S = np.asarray(g.S, np.int32)
    probe = S[: max(2, min(S.size, 20))]
    t0 = time.perf_counter()
    oracle.bc(g, probe, L=L)
    per_src = max((time.perf_counter() - t0) / probe.size, 1e-6)
    ns1 = int(max(2, min(S.size, 0.5 * budget_s / per_src)))
    t0 = time.perf_counter()
    oracle.bc(g, S[:ns1], L=L)
    dt1 = time.perf_counter() - t0
    v1 = ns1 * g.m / dt1
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(16, avail, S.size // 2))
    nsp = int(max(2 * cores, min(S.size, 0.5 * budget_s / per_src * cores)))
    chunks = np.array_split(S[:nsp], cores)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        list(ex.map(lambda c: oracle.bc(g, c, L=L), chunks))
    dtp = time.perf_counter() - t0
    return {
        "value": nsp * g.m / dtp,
        "unit": "TEPS",
        "cores": cores,
        "kind": "oracle",
        "value_1core": v1,
        "sample": (f"{cores} host threads on the first {nsp} of {S.size} targets of the same graph, "
                   f"a contiguous chunk each ({dtp:.1f} s); one thread on the first {ns1} ({dt1:.1f} s)"),
    }


def calibration_copy(args):
    """One plain device copy of --copy-mib MiB: a kernel of known traffic whose
    profiler byte counters scale the others'."""
    import torch

    if args.copy_mib:
        a = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b


def bench_batch(args):
    """256 independent graphs in one device run; TEPS = sum over graphs of |S_g| m_g / s.
    The batch entry point returns host arrays, so this rate includes the copy of all
    scores to the host. Each pass replays its captured HIP graph; a graph holds no
    per-launch events, so the roofline's kernel durations come from HIP events on eager
    runs of the same launches (same kernels, groups and launch records), taken right
    after the timed replays."""
    import torch

    from paper_1406_4173_amd import bcpp, inputs

    gs = inputs.batch_256()
    B = bcpp.Batch(gs)
    sync = torch.cuda.synchronize
    calibration_copy(args)
    units = float(sum(len(g.S) * g.m for g in gs))
    t_pp = timed(lambda: B.run(pp=True), args.steps, args.warmup, sync)
    t_plain = timed(lambda: B.run(pp=False), args.steps, args.warmup, sync)
    bcpp.profile_enable(True)
    B.run(pp=True, graph=False)
    sync()
    bcpp.profile_reset()
    t_eager = timed(lambda: B.run(pp=True, graph=False), args.steps, 0, sync)
    prof = bcpp.profile_read()
    bcpp.profile_enable(False)
    kern = max((k for k in prof if k != "other"), key=lambda k: prof[k]["ms"])
    kp = prof[kern]
    res = {
        "metric": "exact-BC TEPS (|S|*m/s), Brandes++ batched, 1 GPU",
        "value": units / t_pp, "unit": "TEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_pp * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32/u64/f64", "data": "synthetic",
        "config": {"workload": "batch_256", "graphs": len(gs), "n": int(sum(g.n for g in gs)),
                   "m": int(sum(g.m for g in gs)), "targets": int(sum(len(g.S) for g in gs))},
        "roofline": roofline_entry("batch_256", kern, kp, "HIP events on eager runs of the replayed launches"),
        "kernels_ms_per_step": {k: v["ms"] / args.steps for k, v in prof.items()},
        "eager_ms_per_step": t_eager * 1e3,
        "plain": {"value": units / t_plain, "unit": "TEPS", "ms_per_step": t_plain * 1e3},
        "pp_over_plain": t_plain / t_pp,
    }
    print(json.dumps(res), flush=True)


def bench_p1_sweep(args):
    """Small-cut sweep (100,000 nodes in 5,000 communities of 20, mean degree 8, weights
    1..4, |S| = 200) over the fraction of intra-community edges: per fraction, Brandes++
    (partition included) and plain Brandes timed the same way as the single-graph
    workloads, and the skeleton's size. The smaller the cut, the smaller the skeleton
    and the larger Brandes++'s lead. value = Brandes++ TEPS at the smallest cut."""
    import numpy as np
    import torch

    from paper_1406_4173_amd import bcpp, inputs

    dev = torch.device("cuda:0")
    sync = torch.cuda.synchronize
    rows = []
    for f in inputs.P1_INTRA:
        g = inputs.p1_graph(f)
        G = bcpp.Graph(g, stream=torch.cuda.current_stream(dev))
        S_dev = torch.tensor(g.S, dtype=torch.int32, device=dev)
        out = torch.empty(g.n, dtype=torch.float64, device=dev)
        part = np.ascontiguousarray(g.part, np.int32)
        S_host = np.ascontiguousarray(g.S, np.int32)
        state = {}

        def pp_step():
            sk = bcpp.partition_sk(G, part, g.k, S_host)
            bcpp.brandes_pp_dev(G, sk, out)
            state["sk"] = sk

        t_pp = timed(pp_step, args.steps, args.warmup, sync)
        t_plain = timed(lambda: bcpp.brandes_plain_dev(G, S_dev, out), args.steps, args.warmup, sync)
        st = state["sk"].stats()
        units = float(len(g.S) * g.m)
        rows.append({"intra": f, "m": int(g.m), "pp_ms": t_pp * 1e3, "plain_ms": t_plain * 1e3,
                     "pp_teps": units / t_pp, "plain_teps": units / t_plain, "pp_over_plain": t_plain / t_pp,
                     "skeleton_nodes": st["n_sk"], "skeleton_arcs": st["r_arcs"] + st["clique_arcs"],
                     "table_nnz": st["table_nnz"]})
        print(f"p1 intra {f}: Brandes++ {t_pp*1e3:.2f} ms, plain {t_plain*1e3:.2f} ms", file=sys.stderr,
              flush=True)
    last = rows[-1]
    res = {
        "metric": "exact-BC TEPS (|S|*m/s), Brandes++ vs plain Brandes over a small-cut sweep, 1 GPU",
        "value": last["pp_teps"], "unit": "TEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": last["pp_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32/u64/f64", "data": "synthetic",
        "config": {"workload": "p1_sweep", "n": 100000, "communities": 5000, "targets": 200,
                   "intra": list(inputs.P1_INTRA)},
        "sweep": rows,
    }
    print(json.dumps(res), flush=True)


def bench_lp(args):
    """The device partitioner (bc_partition_lp, size-constrained label propagation) on
    pareto_100k, and Brandes++ over its partition beside Brandes++ over the planted one
    and plain Brandes (same targets, timed the same way as the single-graph workloads;
    the partition is made once per graph, so its time is reported apart from the
    step). Scores do not depend on the partition (Sec. 5); its cut decides the
    skeleton's size. value = Brandes++ TEPS over the device partition."""
    import numpy as np
    import torch

    from paper_1406_4173_amd import bcpp, inputs

    dev = torch.device("cuda:0")
    sync = torch.cuda.synchronize
    g = inputs.pareto_100k()
    G = bcpp.Graph(g, stream=torch.cuda.current_stream(dev))
    S_dev = torch.tensor(g.S, dtype=torch.int32, device=dev)
    S_host = np.ascontiguousarray(g.S, np.int32)
    out = torch.empty(g.n, dtype=torch.float64, device=dev)
    cap, rounds, seed = 0, 48, 5
    res_lp = {}

    def lp():
        res_lp["p"] = bcpp.partition_lp(G, cap, rounds, seed)

    t_lp = timed(lp, max(args.steps // 2, 1), 1, sync)
    lp_part, lp_k = res_lp["p"]
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    col = np.asarray(g.col)
    rows = {}
    for name, part, k in (("device", lp_part, lp_k), ("planted", np.ascontiguousarray(g.part, np.int32), g.k)):
        state = {}

        def pp_step(part=part, k=k, state=state):
            sk = bcpp.partition_sk(G, part, k, S_host)
            bcpp.brandes_pp_dev(G, sk, out)
            state["sk"] = sk

        t = timed(pp_step, args.steps, args.warmup, sync)
        st = state["sk"].stats()
        rows[name] = {"parts": int(k), "cut": float(np.mean(part[src] != part[col])), "pp_ms": t * 1e3,
                      "skeleton_nodes": st["n_sk"], "skeleton_arcs": st["r_arcs"] + st["clique_arcs"],
                      "table_nnz": st["table_nnz"]}
    t_plain = timed(lambda: bcpp.brandes_plain_dev(G, S_dev, out), args.steps, args.warmup, sync)
    units = float(len(g.S) * g.m)
    d = rows["device"]
    res = {
        "metric": "exact-BC TEPS (|S|*m/s), Brandes++ over the device partition, 1 GPU",
        "value": units / (d["pp_ms"] * 1e-3), "unit": "TEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": d["pp_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32/u64/f64", "data": "synthetic",
        "config": {"workload": "lp_pareto_100k", "n": g.n, "m": int(g.m), "targets": int(len(g.S)),
                   "max_part": cap, "rounds": rounds, "seed": seed},
        "partition_ms": t_lp * 1e3, "partitions": rows, "plain_ms": t_plain * 1e3,
    }
    print(json.dumps(res), flush=True)


def bench_pp_all(args):
    """Brandes++All (bc_brandes_pp_all, Sec. 6, Alg. 3) on planted_1k: all-pairs scores
    through one skeleton per ordered pair of its 8 parts (64 skeleton builds and
    Brandes_SK + Centrality passes), beside plain Brandes and Brandes++ with S = V on the
    same graph. value = Brandes++All TEPS (n * m / s)."""
    import numpy as np
    import torch

    from paper_1406_4173_amd import bcpp, inputs

    dev = torch.device("cuda:0")
    sync = torch.cuda.synchronize
    g = inputs.planted_1k()
    G = bcpp.Graph(g, stream=torch.cuda.current_stream(dev))
    part = np.ascontiguousarray(g.part, np.int32)
    S_host = np.arange(g.n, dtype=np.int32)
    S_dev = torch.tensor(S_host, device=dev)
    out = torch.empty(g.n, dtype=torch.float64, device=dev)
    t_all = timed(lambda: bcpp.brandes_pp_all(G, part, g.k), args.steps, min(args.warmup, 3), sync)

    def pp_step():
        bcpp.brandes_pp_dev(G, bcpp.partition_sk(G, part, g.k, S_host), out)

    t_pp = timed(pp_step, args.steps, args.warmup, sync)
    t_plain = timed(lambda: bcpp.brandes_plain_dev(G, S_dev, out), args.steps, args.warmup, sync)
    units = float(g.n * g.m)
    res = {
        "metric": "exact-BC TEPS (n*m/s), Brandes++All on 1 GPU",
        "value": units / t_all, "unit": "TEPS", "n_gpus": 1, "steps": args.steps, "warmup": min(args.warmup, 3),
        "ms_per_step": t_all * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32/u64/f64", "data": "synthetic",
        "config": {"workload": "pp_all_planted_1k", "n": g.n, "m": int(g.m), "parts": int(g.k),
                   "skeletons": int(g.k) ** 2},
        "pp_ms": t_pp * 1e3, "plain_ms": t_plain * 1e3,
    }
    print(json.dumps(res), flush=True)


def bench_serve(args):
    """Open-loop Poisson stream of Brandes++ queries over 64 resident graphs; TEPS =
    sum of |S| m over the queries submitted in the measured window, divided by the time
    from the window's start to the last of them finishing; p50/p99 are their
    submit-to-result latencies."""
    import numpy as np

    from paper_1406_4173_amd import bcpp, inputs

    warm = 2.0
    pool = inputs.serving_pool()
    stream = inputs.serving_stream([g.n for g in pool], rate=args.serve_rate,
                                   seconds=warm + args.serve_seconds)
    srv = bcpp.Server(96 << 30, max_inflight=64)
    gids = [srv.add_graph(g) for g in pool]
    # a seeded 1% (at least 20) of the measured window's queries, kept for the oracle
    measured = [i for i, q in enumerate(stream) if q[0] >= warm]
    ns_check = min(len(measured), max(20, -(-len(measured) // 100)))
    check = set(np.random.default_rng(1406).choice(measured, ns_check, replace=False).tolist())
    kept = {}
    t0 = time.perf_counter()
    out = {}
    lat, units_done, last_done = [], 0.0, 0.0
    failed = 0
    reasons = {}
    i = 0
    next_report = 5.0
    while i < len(stream) or out:
        now = time.perf_counter() - t0
        while i < len(stream) and stream[i][0] <= now:
            ts, gi, S = stream[i]
            t = srv.submit(gids[gi], S)
            if t is None:  # queue full: retry on the next pass
                break
            out[t] = (ts, pool[gi].n, float(len(S)) * pool[gi].m, i)
            i += 1
        for t in list(out):
            ts, n, units, qi = out[t]
            try:
                r = srv.poll(t, n)
            except bcpp.BcError as e:
                failed += 1
                reasons[str(e)[:80]] = reasons.get(str(e)[:80], 0) + 1
                del out[t]
                continue
            if r is None:
                continue
            tdone = time.perf_counter() - t0
            del out[t]
            if qi in check:
                kept[qi] = r
            if ts >= warm:
                lat.append((tdone - ts) * 1e3)
                units_done += units
                last_done = max(last_done, tdone)
        if now >= next_report:
            print(f"serve: t={now:.0f}s submitted {i}/{len(stream)} outstanding {len(out)}",
                  file=sys.stderr, flush=True)
            next_report += 5.0
        time.sleep(0.0005)
    st = srv.stats()
    srv.close()
    # outside the measured window: the sample against the oracle (within 1e-9)
    import concurrent.futures as cf

    import oracle

    L = oracle.lib()
    done_check = sorted(kept)

    def rel_err(qi):
        ts, gi, S = stream[qi]
        want = oracle.bc(pool[gi], S, L=L)
        got = kept[qi]
        err = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
        err[want == 0] = 0
        return float(err.max(initial=0.0)) if np.array_equal(got == 0, want == 0) else float("inf")

    with cf.ThreadPoolExecutor(16) as ex:
        errs = list(ex.map(rel_err, done_check))
    oracle_check = {"sample": len(check), "checked": len(done_check),
                    "mismatches": int(sum(e > 1e-9 for e in errs)),
                    "max_rel_err": max(errs, default=0.0), "tolerance": 1e-9,
                    "how": "seeded 1% (at least 20) of the measured window's queries, CPU oracle"}
    lat = np.array(lat) if lat else np.zeros(1)
    window = max(last_done - warm, 1e-9)
    res = {
        "metric": "exact-BC TEPS (|S|*m/s), Brandes++ served, 1 GPU; p50/p99 query ms",
        "value": units_done / window, "unit": "TEPS", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": window * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32/u64/f64", "data": "synthetic",
        "config": {"workload": "serve_64", "graphs": len(pool), "rate_per_s": args.serve_rate,
                   "measured_s": args.serve_seconds, "queries": int(len(lat)),
                   "failed": int(failed), "failures": reasons},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "server": st, "oracle_check": oracle_check,
    }
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards "
              "by source batches across GPUs by design but only the one-GPU kernel is built",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch_256":
        return bench_batch(args)
    if args.workload == "serve_64":
        return bench_serve(args)
    if args.workload == "p1_sweep":
        return bench_p1_sweep(args)
    if args.workload == "lp_pareto_100k":
        return bench_lp(args)
    if args.workload == "pp_all_planted_1k":
        return bench_pp_all(args)
    import numpy as np
    import torch

    from paper_1406_4173_amd import bcpp, inputs

    g = inputs.CONFIGS[args.workload]()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    G = bcpp.Graph(g, stream=stream)
    S_dev = torch.tensor(g.S, dtype=torch.int32, device=dev)
    out = torch.empty(g.n, dtype=torch.float64, device=dev)
    part = np.ascontiguousarray(g.part, np.int32)
    S_host = np.ascontiguousarray(g.S, np.int32)
    sync = torch.cuda.synchronize
    state = {}

    def pp_step():
        sk = bcpp.partition_sk(G, part, g.k, S_host)
        bcpp.brandes_pp_dev(G, sk, out)
        state["sk"] = sk

    def plain_step():
        bcpp.brandes_plain_dev(G, S_dev, out)

    calibration_copy(args)
    if args.only_plain:
        t_plain = timed(plain_step, args.steps, args.warmup, sync)
        print(f"plain Brandes on {args.workload}: {t_plain * 1e3:.3f} ms per step", file=sys.stderr, flush=True)
        return

    # timed Brandes++ steps, kernels timed with HIP events on the library's stream
    bcpp.profile_enable(True)
    for _ in range(args.warmup):
        pp_step()
    sync()
    bcpp.profile_reset()
    t_pp = timed(pp_step, args.steps, 0, sync)
    prof = bcpp.profile_read()
    bcpp.profile_enable(False)
    sk_stats = state["sk"].stats()

    units = float(len(g.S)) * g.m
    res = {
        "metric": "exact-BC TEPS (|S|*m/s), Brandes++ on 1 GPU",
        "value": units / t_pp,
        "unit": "TEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_pp * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64/f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "n": g.n,
            "m": g.m,
            "targets": int(len(g.S)),
            "parts": int(g.k),
            "weights": "unit" if g.w is None else f"1..{int(g.w.max())}",
            "skeleton_nodes": sk_stats["n_sk"],
            "skeleton_arcs": sk_stats["r_arcs"] + sk_stats["clique_arcs"],
            "table_nnz": sk_stats["table_nnz"],
            "dijkstra_sk_sources": sk_stats["dsk_sources"],
        },
    }
    # roofline of the dominant kernel (most time over the timed steps), and of every
    # kernel kind that ran, each with its share of the step
    kern = max((k for k in prof if k not in ("other",)), key=lambda k: prof[k]["ms"])
    res["roofline"] = roofline_entry(args.workload, kern, prof[kern])
    res["kernels"] = {k: dict(roofline_entry(args.workload, k, v), ms_per_step=v["ms"] / args.steps)
                      for k, v in prof.items() if v["launches"] > 0 and k in ("resident", "dijkstra_sk", "centrality")}
    res["kernels_ms_per_step"] = {k: v["ms"] / args.steps for k, v in prof.items()}
    # where a Brandes++ step goes: the partition call (P', frontiers, Dijkstra_SK,
    # assembly; host work included) and the Brandes_SK + Centrality call, timed apart
    sk_keep = state["sk"]
    t_part = timed(lambda: bcpp.partition_sk(G, part, g.k, S_host), args.steps, 2, sync)
    t_bsk = timed(lambda: bcpp.brandes_pp_dev(G, sk_keep, out), args.steps, 2, sync)
    res["pp_breakdown_ms"] = {
        "partition_sk": t_part * 1e3,
        "brandes_sk_centrality": t_bsk * 1e3,
        "dijkstra_sk_kernel": prof["dijkstra_sk"]["ms"] / args.steps,
        "brandes_sk_kernel": prof["resident"]["ms"] / args.steps,
        "centrality_kernels": prof["centrality"]["ms"] / args.steps,
    }
    if not args.no_plain:
        t_plain = timed(plain_step, args.steps, args.warmup, sync)
        res["plain"] = {"value": units / t_plain, "unit": "TEPS", "ms_per_step": t_plain * 1e3}
        # the plain pass's roofline: the same steps again with the kernels' HIP events and
        # byte counters on (after the timed steps, which ran without them)
        bcpp.profile_enable(True)
        bcpp.profile_reset()
        for _ in range(args.steps):
            plain_step()
        sync()
        pk = bcpp.profile_read()["resident"]
        bcpp.profile_enable(False)
        if pk["ms"] > 0 and pk["launches"] > 0:
            res["plain"]["roofline"] = roofline_entry(
                args.workload + ":plain", "resident", pk,
                "HIP events on a profiled pass of the same steps after the timed ones")
        res["pp_over_plain"] = t_plain / t_pp
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
