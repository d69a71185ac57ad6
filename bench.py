"""Benchmark: GCMC trial moves/s and pair evaluations/s on one MI355X.

Workload (default): the two-phase slab, box a x a x 4a with a liquid slab at
reduced density 0.8 inside vapour at 0.02, N ~ 1,500,000, rc = 2.5, T* = 0.85,
mu* = -3, the 1/3-1/3-1/3 move mix; one step = one persistent launch of
200,000 moves of the chain.  Inputs are seeded synthetic configurations
(random sequential addition with overlap rejection), resident in HBM before the
timed region starts.

Prints one JSON line: moves/s (value), pair evaluations/s, the roofline of the
chain kernel (algorithmic bytes per launch / average launch time, against the
8 TB/s HBM peak), the batched-boxes throughput, and the CPU oracle timed on a
bounded sample of the same chain on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GCMC trial moves/sec + LJ pair evals/sec at 1M particles; % HBM peak; batched vs single"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def alg_bytes(stats, nstencil):
    """Algorithmic HBM bytes of a chain launch: per gathered stencil its cell
    counters (4 B each), per candidate its coordinates and id (24 + 4 B), per
    displacement/deletion the picked particle's record (32 B), per accepted move
    the commit writes (one 32 B record and one 32 B cell entry, counters)."""
    att = [int(v) for v in stats["attempts"]]
    acc = [int(v) for v in stats["accepts"]]
    return (int(stats["stencils"]) * nstencil * 4 + int(stats["candidates"]) * 28 + (att[0] + att[2]) * 32
            + sum(acc) * 72)


def workload_by_name(name):
    from paper_1408_3764_amd import workloads
    return {"slab": workloads.slab, "large": workloads.large, "small": workloads.small}[name]()


def run_cpu_baseline(wb, budget_s, max_moves):
    """The oracle chain (all-pairs, one thread) on the first moves of the same chain."""
    import oracle
    p = oracle.make_params(wb.L, wb.rc, beta=wb.beta, mu=wb.mu, lambda3=wb.lambda3, max_disp=wb.max_disp,
                           p_disp=wb.p_disp)
    t = time.perf_counter()
    oracle.chain(wb.pos, 10, p, seed=wb.seed, max_n=wb.n + 20)
    per = max((time.perf_counter() - t) / 10, 1e-7)
    n = int(max(20, min(max_moves, budget_s / per)))
    t = time.perf_counter()
    _, _, olog = oracle.chain(wb.pos, n, p, seed=wb.seed, max_n=wb.n + n + 1)
    dt = time.perf_counter() - t
    return n, dt, olog


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="slab", choices=["slab", "large", "small"])
    ap.add_argument("--moves-per-step", type=int, default=0, help="0: the workload's move count")
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-allpairs", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (the chain of one box is a "
              "dependent sequence; see the sharding notes in DESIGN.md). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1408_3764_amd import tune
    from paper_1408_3764_amd.box import Batch, Box

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = time.perf_counter()
    wb = workload_by_name(args.workload)
    log("workload %s: N=%d generated in %.1fs" % (wb.name, wb.n, time.perf_counter() - t))
    mps = args.moves_per_step or wb.n_moves
    total_moves = mps * (args.steps + args.warmup)
    box = Box.from_workload(wb, max_n=wb.n + total_moves + 1)
    info = box.info()
    nst = info["span"][0] * info["span"][1] * info["span"][2]
    if args.waves and args.rows:
        box.set_launch(args.waves, args.rows)
        shape = (args.waves, args.rows)
    else:
        shape = tune.chain_shape(box)
        box.set_launch(*shape)
    U0 = box.total_energy()
    log("box: cells %s cap %d stencil %d, launch %dx%d, U0=%.6f" % (info["cell_m"], info["cell_cap"], nst,
                                                                     shape[0], shape[1], U0["U_pair"]))
    stream = torch.cuda.current_stream()
    ctr = 0
    for w in range(args.warmup):
        box.step(mps, counter0=ctr)
        ctr += mps
    torch.cuda.synchronize()
    evs = []
    stats_all = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st, _ = box.step(mps, counter0=ctr)
        e1.record(stream)
        ctr += mps
        evs.append((e0, e1))
        stats_all.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    for st in stats_all:
        if int(st["error"]) != 0:
            raise SystemExit("chain error %d at move %d" % (int(st["error"]), int(st["error_move"])))
    launch_ms = [a.elapsed_time(b) for a, b in evs]
    moves = mps * args.steps
    pair_evals = sum(int(s["pair_evals"]) for s in stats_all)
    incut = sum(int(s["in_cutoff"]) for s in stats_all)
    cand = sum(int(s["candidates"]) for s in stats_all)
    bytes_per_launch = sum(alg_bytes(s, nst) for s in stats_all) / args.steps
    avg_launch_s = sum(launch_ms) / len(launch_ms) / 1e3
    achieved = bytes_per_launch / avg_launch_s / 1e9
    log("timed %d x %d moves: %.3fs wall, launch avg %.2f ms, %.0f moves/s, %.3g pair evals/s" %
        (args.steps, mps, wall, 1e3 * avg_launch_s, moves / wall, pair_evals / wall))
    acc = np.sum([s["accepts"] for s in stats_all], axis=0)
    att = np.sum([s["attempts"] for s in stats_all], axis=0)

    out = {
        "metric": METRIC,
        "value": moves / wall,
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random sequential addition, overlap rejection at 0.8 sigma)",
        "config": {"workload": wb.name, "n": wb.n, "moves_per_step": mps, "rc": wb.rc, "T": 1.0 / wb.beta,
                   "mu": wb.mu, "cells": info["cell_m"], "cell_cap": info["cell_cap"], "stencil_cells": nst,
                   "launch": {"waves": shape[0], "rows": shape[1]}},
        "pair_evals_per_s": pair_evals / wall,
        "in_cutoff_pairs_per_s": incut / wall,
        "candidates_per_move": cand / moves,
        "acceptance": {"displace": float(acc[0] / max(att[0], 1)), "insert": float(acc[1] / max(att[1], 1)),
                       "delete": float(acc[2] / max(att[2], 1))},
        "us_per_move": 1e6 * wall / moves,
        "roofline": {"bound": "hbm", "kernel": "k_chain", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": bytes_per_launch, "avg_launch_ms": 1e3 * avg_launch_s},
    }

    if not args.no_allpairs and args.workload != "slab":
        # the no-cell-list path of the paper, same chain, a bounded number of moves
        ab = Box.from_workload(wb, max_n=wb.n + 2001)
        ab.step(50, counter0=0, all_pairs=True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        sa, _ = ab.step(1000, counter0=50, all_pairs=True)
        torch.cuda.synchronize()
        da = time.perf_counter() - ta
        out["allpairs"] = {"moves_per_s": 1000 / da, "pair_evals_per_s": int(sa["pair_evals"]) / da,
                           "moves": 1000}
        ab.close()

    if not args.no_batched:
        from paper_1408_3764_amd import workloads
        tb = time.perf_counter()
        wbs = workloads.batched()
        log("batched: %d boxes, N total %d, generated in %.1fs" % (len(wbs), sum(w.n for w in wbs),
                                                                 time.perf_counter() - tb))
        boxes = [Box.from_workload(w, max_n=w.n + 2101, box_id=k) for k, w in enumerate(wbs)]
        bshape = tune.batch_shape(boxes)
        for b in boxes:
            b.set_launch(*bshape)
        bt = Batch(boxes)
        bt.step(100, counter0=0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        tb = time.perf_counter()
        e0.record(stream)
        bst = bt.step(1000, counter0=100)
        e1.record(stream)
        torch.cuda.synchronize()
        db = time.perf_counter() - tb
        bmoves = 1000 * len(boxes)
        out["batched"] = {"boxes": len(boxes), "moves_per_box": 1000, "moves_per_s": bmoves / db,
                          "pair_evals_per_s": float(np.sum(bst["pair_evals"])) / db,
                          "launch_ms": e0.elapsed_time(e1), "launch": {"waves": bshape[0], "rows": bshape[1]},
                          "errors": int(np.count_nonzero(bst["error"]))}
        bt.close()
        for b in boxes:
            b.close()

    if not args.no_cpu:
        n_cpu, dt, olog = run_cpu_baseline(wb, args.cpu_budget, 20000)
        # the same moves on the GPU, for a parity check of the timed chain
        pb = Box.from_workload(wb, max_n=wb.n + n_cpu + 1)
        pb.set_launch(*shape)
        _, glog = pb.step(n_cpu, counter0=0, log=True)
        same = bool(np.array_equal(glog["type"], olog["type"]) and np.array_equal(glog["accepted"], olog["accepted"])
                    and np.array_equal(glog["index"], olog["index"]))
        out["cpu_baseline"] = {"value": n_cpu / dt, "unit": "moves/s", "cores": 1, "kind": "oracle",
                               "sample": "first %d moves of the same chain from the same initial configuration "
                                         "(all-pairs FP64 oracle, one thread, %.1fs)" % (n_cpu, dt),
                               "gpu_chain_matches_on_sample": same}
        pb.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
