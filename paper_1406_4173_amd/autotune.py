"""Autotuner of the resident kernel's launch shapes; writes csrc/tuned.h.

Usage (on a machine with the GPU): python -m paper_1406_4173_amd.autotune [--out PATH]
[--pairs SMALL:MID,...] [--divs DIV,...] [--dense SHIFT,...], then rebuild (python -m
paper_1406_4173_amd.build_lib). The options narrow the grids below ("all" = no limit);
a single --dense value is kept without timing.

Four values are tuned, all fixed per build so that a graph gets the same launch shape
alone, inside a batch or in the server (results then agree bit for bit):

* threads per workgroup by node range (256 up to tuned_small_range, 512 up to
  tuned_mid_range, 1024 above) and sources per group, ceil(|S| / div). The two
  interact: the divisor sets how many groups a launch has and so how many a compute
  unit holds, which decides whether wide or narrow workgroups fill it. They are
  therefore chosen together, from a grid of threshold pairs and divisors, each timed
  on the workloads they serve: the 10,000-node stochastic block model and the
  1,000-node planted partition (plain Brandes and Brandes++), and the 256-graph batch
  (both passes). The grid point with the smallest total time is kept (a sum of
  times relative to each workload's best would let the sub-millisecond 1,000-node
  runs outweigh the batch);
* the launch shape of Dijkstra_SK groups, which run up to 64 sources of one part one
  after another in a launch that lasts as long as its longest group: their own
  thread-class thresholds and a work budget per group (a large part's sources are
  dealt to more groups), timed on pareto_100k, smallcut_100k and the 256-graph batch
  (Brandes++);
* the dense-step threshold of bucket frontiers (ranges whose state lives in device
  memory; a step with more than range >> shift bucket bits scans the range): shifts 1
  to 6, and 63 (scan nearly always), timed the same way on the two 100,000-node graphs.

Every timing is the best of a few runs of a call through the Python binding, with the
choice under test set through the BCPP_TUNE_* overrides the library reads at each
launch; batches are rebuilt per grid point, since a batch captures its plain pass once.
"""
from __future__ import annotations

import argparse
import math
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BIG = 1 << 40


def _time(fn, sync, reps=3):
    fn()
    sync()
    best = math.inf
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        sync()
        best = min(best, time.perf_counter() - t0)
    return best


def _clear():
    for k in ("BCPP_TUNE_SMALL", "BCPP_TUNE_MID", "BCPP_TUNE_SPG_DIV", "BCPP_TUNE_DENSE_SHIFT",
              "BCPP_TUNE_DSK_SMALL", "BCPP_TUNE_DSK_MID", "BCPP_TUNE_DSK_WORK"):
        os.environ.pop(k, None)


SHAPE_PAIRS = [(BIG, BIG), (6500, BIG), (4000, 6500), (2500, 6500), (2500, 4000), (1500, 6500), (1500, 4000),
               (1000, 6500), (1000, 4000), (500, 4000), (0, 6500), (0, 4000), (0, 0)]
SHAPE_DIVS = (256, 1024)


def sweep_shapes(bcpp, inputs, torch, log, pairs=SHAPE_PAIRS, divs=SHAPE_DIVS):
    singles = []
    for name in ("sbm_10k", "planted_1k"):
        g = getattr(inputs, name)()
        G = bcpp.Graph(g)
        S = torch.tensor(g.S, dtype=torch.int32, device="cuda")
        out = torch.empty(g.n, dtype=torch.float64, device="cuda")
        singles.append((name + " plain", lambda G=G, S=S, out=out: bcpp.brandes_plain_dev(G, S, out)))
        singles.append((name + " pp", lambda G=G, g=g: bcpp.brandes_pp(G, bcpp.partition_sk(G, g.part, g.k, g.S))))
    gs = inputs.batch_256()
    names = [n for n, _ in singles] + ["batch_256 plain", "batch_256 pp"]
    rows = {}
    for small, mid in pairs:
        for div in divs:
            os.environ["BCPP_TUNE_SMALL"] = str(small)
            os.environ["BCPP_TUNE_MID"] = str(mid)
            os.environ["BCPP_TUNE_SPG_DIV"] = str(div)
            t = [_time(f, torch.cuda.synchronize, reps=2) for _, f in singles]
            B = bcpp.Batch(gs)
            t.append(_time(lambda: B.run(pp=False), torch.cuda.synchronize, reps=2))
            t.append(_time(lambda: B.run(pp=True), torch.cuda.synchronize, reps=2))
            del B
            rows[(small, mid, div)] = t
            show = lambda v: "all" if v >= BIG else str(v)
            log.append(f"256 to {show(small):>4s} 512 to {show(mid):>4s} div {div:4d}: " + "  ".join(
                f"{nm} {x*1e3:7.2f}" for nm, x in zip(names, t)))
            print(log[-1], flush=True)
    _clear()
    return min(rows, key=lambda k: sum(rows[k]))


DSK_PAIRS = [(2000, 5000), (1000, 2000), (500, 1000), (250, 1000), (500, 2000)]
DSK_WORK = (0, 400000, 200000, 100000)


def sweep_dsk(bcpp, inputs, torch, log, pairs=DSK_PAIRS, works=DSK_WORK):
    """Dijkstra_SK launch shapes: thread-class thresholds and the per-group work budget,
    timed on whole Brandes++ steps (the other steps do not depend on them)."""
    work = []
    for name in ("pareto_100k", "smallcut_100k"):
        g = getattr(inputs, name)()
        G = bcpp.Graph(g)
        work.append((name + " pp", lambda G=G, g=g: bcpp.brandes_pp(G, bcpp.partition_sk(G, g.part, g.k, g.S))))
    gs = inputs.batch_256()
    rows = {}
    for small, mid in pairs:
        for wk in works:
            os.environ["BCPP_TUNE_DSK_SMALL"] = str(small)
            os.environ["BCPP_TUNE_DSK_MID"] = str(mid)
            os.environ["BCPP_TUNE_DSK_WORK"] = str(wk)
            t = [_time(f, torch.cuda.synchronize, reps=3) for _, f in work]
            B = bcpp.Batch(gs)
            t.append(_time(lambda: B.run(pp=True), torch.cuda.synchronize, reps=2))
            del B
            rows[(small, mid, wk)] = t
            log.append(f"Dijkstra_SK 256 to {small:4d} 512 to {mid:4d} work {wk:6d}: " + "  ".join(
                f"{nm} {x*1e3:7.2f}" for nm, x in zip([n for n, _ in work] + ["batch_256 pp"], t)))
            print(log[-1], flush=True)
    for k in ("BCPP_TUNE_DSK_SMALL", "BCPP_TUNE_DSK_MID", "BCPP_TUNE_DSK_WORK"):
        os.environ.pop(k, None)
    return min(rows, key=lambda k: sum(rows[k]))


def sweep_dense(bcpp, inputs, torch, log, shifts=(1, 2, 3, 4, 6, 63)):
    """Bucket steps with more than range >> shift bits scan the range instead; the
    shift only moves time (both visits queue the same nodes in the same order)."""
    work = []
    for name in ("smallcut_100k", "pareto_100k"):
        g = getattr(inputs, name)()
        G = bcpp.Graph(g)
        S = torch.tensor(g.S, dtype=torch.int32, device="cuda")
        out = torch.empty(g.n, dtype=torch.float64, device="cuda")
        work.append((name + " plain", lambda G=G, S=S, out=out: bcpp.brandes_plain_dev(G, S, out)))
        work.append((name + " pp", lambda G=G, g=g: bcpp.brandes_pp(G, bcpp.partition_sk(G, g.part, g.k, g.S))))
    rows = {}
    for shift in shifts:
        os.environ["BCPP_TUNE_DENSE_SHIFT"] = str(shift)
        rows[shift] = [_time(f, torch.cuda.synchronize, reps=2) for _, f in work]
        log.append(f"dense shift {shift:2d}: " + "  ".join(
            f"{name} {t*1e3:8.3f} ms" for (name, _), t in zip(work, rows[shift])))
        print(log[-1], flush=True)
    _clear()
    return min(rows, key=lambda k: sum(rows[k]))


def write_header(path, small, mid, div, dense, log, dsk=(2000, 5000, 0)):
    lines = [
        "// Launch shapes of the resident kernel. Written by paper_1406_4173_amd/autotune.py from",
        "// timings on one MI355X; edit by re-running it, not by hand.",
        "//",
        "// Node ranges up to tuned_small_range run with 256 threads per workgroup, up to",
        "// tuned_mid_range with 512, larger ones with 1024. A group holds",
        "// ceil(|S| / tuned_spg_div) sources (1..64). A bucket step of a range of n nodes",
        "// with more than n >> tuned_dense_shift bits scans the range instead.",
        "// Dijkstra_SK groups (forward only, integer results, so any launch shape gives the same",
        "// bits) have their own thresholds, tuned_dsk_small_range and tuned_dsk_mid_range, and",
        "// hold max(8, tuned_dsk_group_work / w) of their part's sources, at most 64, where w is",
        "// the part's nodes plus arcs (0: always 64). The count depends on the part alone, so a",
        "// part is split the same way in every build that holds it.",
        "//",
        "// Timings of the sweep (ms, best of 2 after a warm-up run):",
    ]
    lines += [f"//   {ln}" for ln in log]
    lines += [
        "#pragma once",
        "#include <cstdint>",
        "",
        "namespace bcpp {",
        f"constexpr int64_t tuned_small_range = {small};",
        f"constexpr int64_t tuned_mid_range = {mid};",
        f"constexpr int64_t tuned_spg_div = {div};",
        f"constexpr int64_t tuned_dense_shift = {dense};",
        f"constexpr int64_t tuned_dsk_small_range = {dsk[0]};",
        f"constexpr int64_t tuned_dsk_mid_range = {dsk[1]};",
        f"constexpr int64_t tuned_dsk_group_work = {dsk[2]};",
        "}  // namespace bcpp",
        "",
    ]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "tuned.h"))
    ap.add_argument("--pairs", default=None, help="SMALL:MID,... (\"all\" = no limit)")
    ap.add_argument("--divs", default=None, help="DIV,...")
    ap.add_argument("--dense", default=None, help="SHIFT,... (one value: kept untimed)")
    ap.add_argument("--dsk-pairs", default=None, help="Dijkstra_SK SMALL:MID,...")
    ap.add_argument("--dsk-work", default=None, help="Dijkstra_SK per-group work budgets, 0 = none")
    args = ap.parse_args()
    lim = lambda v: BIG if v == "all" else int(v)
    pairs = ([tuple(lim(x) for x in p.split(":")) for p in args.pairs.split(",")] if args.pairs
             else SHAPE_PAIRS)
    divs = tuple(int(x) for x in args.divs.split(",")) if args.divs else SHAPE_DIVS
    shifts = tuple(int(x) for x in args.dense.split(",")) if args.dense else (1, 2, 3, 4, 6, 63)
    import torch

    from paper_1406_4173_amd import bcpp, inputs

    bcpp.lib()
    _clear()
    log = []
    small, mid, div = sweep_shapes(bcpp, inputs, torch, log, pairs, divs)
    os.environ["BCPP_TUNE_SMALL"] = str(small)
    os.environ["BCPP_TUNE_MID"] = str(mid)
    os.environ["BCPP_TUNE_SPG_DIV"] = str(div)
    dense = shifts[0] if len(shifts) == 1 else sweep_dense(bcpp, inputs, torch, log, shifts)
    os.environ["BCPP_TUNE_DENSE_SHIFT"] = str(dense)
    dpairs = ([tuple(int(x) for x in p.split(":")) for p in args.dsk_pairs.split(",")] if args.dsk_pairs
              else DSK_PAIRS)
    dwork = tuple(int(x) for x in args.dsk_work.split(",")) if args.dsk_work else DSK_WORK
    dsk = sweep_dsk(bcpp, inputs, torch, log, dpairs, dwork)
    log.append(f"chosen: small range {small}, mid range {mid}, sources-per-group divisor {div}, "
               f"dense shift {dense}, Dijkstra_SK small {dsk[0]} mid {dsk[1]} work {dsk[2]}")
    print(log[-1], flush=True)
    write_header(args.out, small, mid, div, dense, log, dsk)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
