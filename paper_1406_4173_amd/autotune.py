"""Autotuner of the resident kernel's launch shapes; writes csrc/tuned.h.

Usage (on a machine with the GPU): python -m paper_1406_4173_amd.autotune [--out PATH]
then rebuild (python -m paper_1406_4173_amd.build_lib).

Three choices are tuned, all fixed per build so that a graph gets the same launch
shape alone, inside a batch or in the server (results then agree bit for bit):

* threads per workgroup by node range: every graph of a sweep over community graphs
  of 500 to 12,000 nodes (unit and integer weights) is timed with 256, 512 and 1024
  threads per workgroup (through the BCPP_TUNE_SMALL / BCPP_TUNE_MID overrides); the
  range thresholds are placed between the sizes where the best choice changes;
* sources per group, ceil(|S| / div): div in {256, 512, 1024, 2048, 4096} timed on the
  10,000-node stochastic block model (S = V) and the 256-graph batch, and the div with
  the smallest sum of times relative to each workload's best is kept;
* the dense-step threshold of bucket frontiers (a step with more than range >> shift
  bucket bits scans the range): shifts 1 to 6, and 63 (scan nearly always), timed the
  same way on three 10,000 to 100,000-node graphs and the batch's Brandes++ pass.

The timed call is plain target-set Brandes on the device (bc_brandes_plain_dev, or a
batch run); the sweep uses the library only through its Python binding.
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


def _force_threads(T):
    """Environment overrides that put every LDS range into the class of T threads."""
    if T == 256:
        os.environ["BCPP_TUNE_SMALL"] = str(BIG)
        os.environ["BCPP_TUNE_MID"] = str(BIG)
    elif T == 512:
        os.environ["BCPP_TUNE_SMALL"] = "1"
        os.environ["BCPP_TUNE_MID"] = str(BIG)
    else:
        os.environ["BCPP_TUNE_SMALL"] = "1"
        os.environ["BCPP_TUNE_MID"] = "1"


def _clear():
    for k in ("BCPP_TUNE_SMALL", "BCPP_TUNE_MID", "BCPP_TUNE_SPG_DIV", "BCPP_TUNE_DENSE_SHIFT"):
        os.environ.pop(k, None)


def sweep_threads(bcpp, inputs, torch, log):
    sizes = [500, 1500, 3000, 5000, 8000, 12000]
    best = {}
    for n in sizes:
        for wmax in (None, 10):
            rng = inputs.rng_for(inputs.SEED_BASE + 77, n, 0 if wmax is None else 1)
            g = inputs._community_graph(rng, n, max(4, n // 250), 10.0, 0.9, wmax, f"tune{n}")
            G = bcpp.Graph(g)
            ns = min(n, 1024)
            S = torch.tensor(np.sort(rng.choice(n, ns, replace=False)).astype(np.int32), device="cuda")
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            row = {}
            for T in (256, 512, 1024):
                _force_threads(T)
                row[T] = _time(lambda: bcpp.brandes_plain_dev(G, S, out), torch.cuda.synchronize)
            _clear()
            key = (n, "unit" if wmax is None else f"1..{wmax}")
            best[key] = row
            log.append(f"n={n:6d} w={key[1]:5s} " + "  ".join(f"T={T}: {row[T]*1e3:8.3f} ms" for T in row))
            print(log[-1], flush=True)
    # per size: the thread count with the smallest summed time over the weight kinds
    choice = {}
    for n in sizes:
        tot = {T: sum(best[k][T] for k in best if k[0] == n) for T in (256, 512, 1024)}
        choice[n] = min(tot, key=tot.get)
    # thresholds: the largest size still won by 256 (then 512), placed half way to
    # the next size; a class never won gets an empty range
    small = 0
    mid = 0
    for i, n in enumerate(sizes):
        nxt = sizes[i + 1] if i + 1 < len(sizes) else n * 2
        if choice[n] == 256:
            small = (n + nxt) // 2
        if choice[n] in (256, 512):
            mid = (n + nxt) // 2
    mid = max(mid, small)
    return small, mid, choice


def sweep_spg(bcpp, inputs, torch, log):
    g = inputs.sbm_10k()
    G = bcpp.Graph(g)
    S = torch.tensor(g.S, dtype=torch.int32, device="cuda")
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    gs = inputs.batch_256()
    B = bcpp.Batch(gs)
    rows = {}
    for div in (256, 512, 1024, 2048, 4096):
        os.environ["BCPP_TUNE_SPG_DIV"] = str(div)
        a = _time(lambda: bcpp.brandes_plain_dev(G, S, out), torch.cuda.synchronize)
        b = _time(lambda: B.run(pp=False), torch.cuda.synchronize, reps=2)
        rows[div] = (a, b)
        log.append(f"div={div:5d} sbm_10k plain {a*1e3:8.3f} ms  batch_256 plain {b*1e3:8.3f} ms")
        print(log[-1], flush=True)
    _clear()
    ba = min(r[0] for r in rows.values())
    bb = min(r[1] for r in rows.values())
    return min(rows, key=lambda d: rows[d][0] / ba + rows[d][1] / bb)


def sweep_dense(bcpp, inputs, torch, log):
    """Bucket steps with more than range >> shift bits scan the range instead; the
    shift only moves time (both visits queue the same nodes in the same order)."""
    work = []
    for name in ("sbm_10k", "smallcut_100k", "pareto_100k"):
        g = getattr(inputs, name)()
        G = bcpp.Graph(g)
        S = torch.tensor(g.S, dtype=torch.int32, device="cuda")
        out = torch.empty(g.n, dtype=torch.float64, device="cuda")
        work.append((name + " plain", lambda G=G, S=S, out=out: bcpp.brandes_plain_dev(G, S, out)))
    gs = inputs.batch_256()
    work.append(("batch_256 pp", lambda: bcpp.Batch(gs).run(pp=True)))
    rows = {}
    for shift in (1, 2, 3, 4, 6, 63):
        os.environ["BCPP_TUNE_DENSE_SHIFT"] = str(shift)
        rows[shift] = [_time(f, torch.cuda.synchronize, reps=2) for _, f in work]
        log.append(f"dense shift {shift:2d}: " + "  ".join(
            f"{name} {t*1e3:8.3f} ms" for (name, _), t in zip(work, rows[shift])))
        print(log[-1], flush=True)
    _clear()
    best = [min(r[i] for r in rows.values()) for i in range(len(work))]
    return min(rows, key=lambda k: sum(t / b for t, b in zip(rows[k], best)))


def write_header(path, small, mid, div, dense, log):
    lines = [
        "// Launch shapes of the resident kernel. Written by paper_1406_4173_amd/autotune.py from",
        "// timings on one MI355X; edit by re-running it, not by hand.",
        "//",
        "// Node ranges up to tuned_small_range run with 256 threads per workgroup, up to",
        "// tuned_mid_range with 512, larger ones with 1024. A group holds",
        "// ceil(|S| / tuned_spg_div) sources (1..64). A bucket step of a range of n nodes",
        "// with more than n >> tuned_dense_shift bits scans the range instead.",
        "//",
        "// Timings of the sweep (best of 3, plain target-set Brandes on the device):",
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
        "}  // namespace bcpp",
        "",
    ]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "csrc", "tuned.h"))
    args = ap.parse_args()
    import torch

    from paper_1406_4173_amd import bcpp, inputs

    bcpp.lib()
    _clear()
    log = []
    small, mid, choice = sweep_threads(bcpp, inputs, torch, log)
    log.append("best threads per size: " + ", ".join(f"{n}: {t}" for n, t in choice.items()))
    div = sweep_spg(bcpp, inputs, torch, log)
    os.environ["BCPP_TUNE_SPG_DIV"] = str(div)
    dense = sweep_dense(bcpp, inputs, torch, log)
    log.append(f"chosen: small range {small}, mid range {mid}, sources-per-group divisor {div}, "
               f"dense shift {dense}")
    print(log[-1], flush=True)
    write_header(args.out, small, mid, div, dense, log)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
