"""Benchmark: GCMC trial moves/s and pair evaluations/s on one MI355X.

Workload (default): the two-phase slab, box a x a x 4a with a liquid slab at
reduced density 0.8 inside vapour at 0.02, N = 1,500,000, rc = 2.5, T* = 0.85,
mu* = -3, the 1/3-1/3-1/3 move mix; one step = one persistent launch of
200,000 moves of the chain, always from the initial 1.5M-particle
configuration: before every step (outside its timed region) the box is put
back into that state with the same move counter, so every timed step is the
same 200,000 moves from N = 1,500,000 (the slab is not stationary at this
state point: left running, it loses particles).  Inputs are seeded synthetic
configurations (random sequential addition with overlap rejection), resident
in HBM before the timed region starts.

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


def resident_alg_bytes(n_start, n_end, ncells):
    """Algorithmic HBM bytes of a launch that holds the box in LDS: the records
    read once (32 B each), records and cell entries written back at the end
    (32 + 32 B each), and the cell counters cleared and counted (4 + 4 B each);
    the moves themselves read and write only LDS."""
    return n_start * 32 + n_end * 64 + ncells * 8


# Sources each chain kernel is compiled from: a traffic record taken with
# rocprofv3 counters is used only while these files are unchanged.
KERNEL_SOURCES = {
    "k_chain": ["chain.hip", "trial.h", "gcmc_internal.h"],
    "k_chain_spec": ["spec.hip", "spec_eval.h", "trial.h", "gcmc_internal.h"],
    "k_chain_async": ["async.hip", "spec_eval.h", "trial.h", "gcmc_internal.h"],
}


def kernel_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1408_3764_amd", "csrc")
    for f in KERNEL_SOURCES[kernel] + ["../../include/gcmc.h"]:
        with open(os.path.normpath(os.path.join(csrc, f)), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, shape, workload, moves_per_launch):
    """HBM bytes per launch from the committed counter summaries under profiles/:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the same kernel, launch shape
    and workload, each scaled by what the counter reads for a copy of known size,
    per move times the moves of this launch; also the ratio of the measured bytes
    to the algorithmic bytes of the profiled launch.  None when no record matches
    or the kernel's sources changed since."""
    import glob
    import re
    want = kernel_source_hash(kernel)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for m in re.finditer(r"<!-- traffic (\{.*?\}) -->", fh.read()):
                r = json.loads(m.group(1))
                if (r["kernel"] == kernel and tuple(r["launch"]) == tuple(shape) and r["workload"] == workload
                        and r["source_hash"] == want):
                    measured = (r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"]) * 1024.0
                    return (measured * moves_per_launch / r["moves_per_launch"], os.path.relpath(path, ROOT),
                            measured / r["alg_bytes"])
    return None, None, None


def stencil_candidates(count, span):
    """Sum over cells c of count[c] x (particles in the stencil of c): the pair
    distances a full-stencil total-energy pass evaluates (self pairs included)."""
    import numpy as np
    tot = np.zeros_like(count, dtype=np.int64)
    sx, sy, sz = span     # stencil cells per axis (2k + 1, or the whole axis)
    for dz in range(-(sz // 2), sz - sz // 2):
        for dy in range(-(sy // 2), sy - sy // 2):
            for dx in range(-(sx // 2), sx - sx // 2):
                tot += np.roll(count, (dz, dy, dx), axis=(0, 1, 2))
    return int((count.astype(np.int64) * tot).sum())


def extra_configs(Box, tune, stream):
    """The small box's 1,000-move chain and the binary mixture's forward and
    backward passes (the parity workloads, timed with HIP events)."""
    import numpy as np
    import torch
    from paper_1408_3764_amd import workloads
    res = {}
    sw = workloads.small()
    sb = Box.from_workload(sw, max_n=sw.n + 12_000)
    sb.set_launch(*tune.chain_shape(sb))
    sb.step(1000, counter0=0)
    torch.cuda.synchronize()
    times = []
    for k in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sb.step(1000, counter0=1000 * (k + 1))
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    res["small"] = {"workload": sw.name, "moves_per_launch": 1000, "launch_ms_median": float(np.median(times)),
                    "moves_per_s": 1000 / (float(np.median(times)) / 1e3)}
    sb.close()
    log("small box: %.0f moves/s (median of 5 launches of 1,000 moves)" % res["small"]["moves_per_s"])
    mw = workloads.mixture()
    mb = Box.from_workload(mw)
    info = mb.info()
    _, count, _ = mb.cells()
    m = info["cell_m"]
    # distances a full-stencil pass evaluates (self pairs included): the backward pass; the
    # forward and virial passes take each pair once
    pairs = stencil_candidates(count.reshape(m[2], m[1], m[0]), info["span"])
    whole_axis = any(int(info["span"][a]) >= int(m[a]) for a in range(3))   # then the full stencil runs
    half = pairs if whole_axis else (pairs - mw.n) // 2
    mb.total_energy_device()
    mb.backward_device(mw.n)
    torch.cuda.synchronize()
    from paper_1408_3764_amd import _lib
    vout = torch.empty(2, dtype=torch.float64, device="cuda")
    fw, bw, vw = [], [], []
    for k in range(5):
        e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        e0.record(stream)
        mb.total_energy_device()
        e1.record(stream)
        mb.backward_device(mw.n)
        e2.record(stream)
        _lib.gcmc_virial(mb.handle, vout, mb.stream)
        e3.record(stream)
        torch.cuda.synchronize()
        fw.append(e0.elapsed_time(e1))
        bw.append(e1.elapsed_time(e2))
        vw.append(e2.elapsed_time(e3))
    f, b, v = float(np.median(fw)), float(np.median(bw)), float(np.median(vw))
    res["mixture"] = {"workload": mw.name, "n": mw.n, "forward_ms_median": f, "backward_ms_median": b,
                      "virial_ms_median": v, "pair_distances": pairs, "pair_distances_forward": half,
                      "pair_distances_per_s_forward": half / (f / 1e3),
                      "pair_distances_per_s_backward": pairs / (b / 1e3)}
    mb.close()
    log("mixture N=%d: forward %.3f ms, backward %.3f ms, virial %.3f ms, %.3g pair distances per backward pass, "
        "%.3g per forward or virial pass" % (mw.n, f, b, v, pairs, half))
    return res


def cell_size_sweep():
    """Traditional cells (side >= rc) against microcells of about rc/2 and rc/3
    (Sec. 3.3), whose stencils of 2k+1 cells per axis drop the cells beyond the
    cutoff, on the small, large and slab workloads: for each cell size and each
    launch shape that applies, moves/s of one chain (median of 3 launches after
    a warmup launch) and the candidates read per move."""
    import numpy as np
    import torch
    from paper_1408_3764_amd import tune
    from paper_1408_3764_amd.box import Box
    from paper_1408_3764_amd._lib import COUNTER_CONTINUE
    stream = torch.cuda.current_stream()
    out = {}
    for name, mps in (("small", 1000), ("large", 10_000), ("slab", 10_000)):
        wb = workload_by_name(name)
        base = None
        rows = []
        for f in (1, 2, 3):
            kw = {} if f == 1 else {"cell_m": [f * m for m in base]}
            b = Box.from_workload(wb, max_n=wb.n + 20 * mps + 1000, **kw)
            info = b.info()
            base = base or info["cell_m"]
            shapes = ([(8, 0)] if tune.spec_supported(b) else []) + [(4, 4), (8, 2), (8, 4), (8, -2)]
            for shape in shapes:
                b.set_launch(*shape)
                b.step(mps, counter0=COUNTER_CONTINUE)
                torch.cuda.synchronize()
                ts, cand = [], 0
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    st, _ = b.step(mps, counter0=COUNTER_CONTINUE)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    if int(st["error"]) != 0:
                        raise SystemExit("chain error %d in the cell sweep" % int(st["error"]))
                    ts.append(e0.elapsed_time(e1))
                    cand += int(st["candidates"])
                med = float(np.median(ts))
                r = {"cell_m": info["cell_m"], "cell_side": [float(wb.L[a] / info["cell_m"][a]) for a in range(3)],
                     "stencil_cells": info["n_stencil"], "stencil_block": int(np.prod(info["span"])),
                     "cell_cap": info["cell_cap"], "launch": list(shape), "moves_per_s": mps / (med / 1e3),
                     "candidates_per_move": cand / (3 * mps)}
                rows.append(r)
                log("%s cells %s (stencil %d of %d) launch %dx%d: %.0f moves/s, %.1f candidates/move" %
                    (name, info["cell_m"], r["stencil_cells"], r["stencil_block"], shape[0], shape[1],
                     r["moves_per_s"], r["candidates_per_move"]))
            b.close()
        out[wb.name] = rows
    return out


def paper_studies(sizes, cutoffs):
    """The paper's size and cutoff studies (Sec. 4) on this GPU: moves/s of one
    chain against N (density 0.67, rc = 2.5) and against the cutoff (87,296
    particles in 128K sigma^3, rc = 2.5 ... 4.25), for the chain without a cell
    list (all pairs), with traditional cells (the per-move kernel and, where it
    applies, the speculative kernel; boxes of at most 2,048 particles also held
    in LDS) and with microcells of about rc/2 (the
    per-move kernel, the paper's one-cell-per-thread mapping and the
    speculative kernel)."""
    import numpy as np
    import torch
    from paper_1408_3764_amd import tune, workloads
    from paper_1408_3764_amd.box import Box
    from paper_1408_3764_amd._lib import COUNTER_CONTINUE
    stream = torch.cuda.current_stream()

    def rate(b, moves, all_pairs=False):
        b.step(max(moves // 4, 1), counter0=COUNTER_CONTINUE, all_pairs=all_pairs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st, _ = b.step(moves, counter0=COUNTER_CONTINUE, all_pairs=all_pairs)
        e1.record(stream)
        torch.cuda.synchronize()
        if int(st["error"]) != 0:
            raise SystemExit("chain error %d in the paper studies" % int(st["error"]))
        return moves / (e0.elapsed_time(e1) / 1e3), int(st["candidates"]) / moves

    def one(wb, moves):
        r = {"n": wb.n, "rc": wb.rc}
        b = Box.from_workload(wb, max_n=wb.n + 4 * moves + 1000)
        r["cells"] = b.info()["cell_m"]
        r["all_pairs"] = rate(b, max(moves // 8, 500), all_pairs=True)[0]
        best = None
        for shape in ((4, 4), (8, 4)):
            b.set_launch(*shape)
            v, c = rate(b, moves)
            if best is None or v > best[0]:
                best = (v, c, shape)
        r["cells_per_move"], r["cells_candidates_per_move"], r["cells_per_move_launch"] = best[0], best[1], best[2]
        r["cells_speculative"] = None
        if tune.spec_supported(b):
            b.set_launch(8, 0)
            r["cells_speculative"] = rate(b, moves)[0]
        # a box small enough to hold in LDS
        r["held_in_lds"] = None
        if wb.n <= tune.RESIDENT_CAP and tune.resident_supported(b):
            b.set_launch(8, -3)
            r["held_in_lds"] = rate(b, moves)[0]
        base = r["cells"]
        b.close()
        b = Box.from_workload(wb, max_n=wb.n + 4 * moves + 1000, cell_m=[2 * m for m in base])
        r["microcells"] = b.info()["cell_m"]
        r["microcell_stencil"] = b.info()["n_stencil"]
        best = None
        for shape in ((4, 4), (8, 4)):
            b.set_launch(*shape)
            v, c = rate(b, moves)
            if best is None or v > best[0]:
                best = (v, c, shape)
        r["microcells_per_move"], r["microcell_candidates_per_move"] = best[0], best[1]
        # the paper's microcell mapping (one stencil cell per thread) and the speculative kernel
        b.set_launch(8, -2)
        r["microcells_paper_mapping"] = rate(b, moves)[0]
        r["microcells_speculative"] = None
        if tune.spec_supported(b):
            b.set_launch(8, 0)
            r["microcells_speculative"] = rate(b, moves)[0]
        b.close()
        log("%s: all pairs %.0f, cells %.0f (%dx%d)%s%s, microcells %.0f (paper mapping %.0f%s) moves/s" % (
            wb.name, r["all_pairs"], r["cells_per_move"], best[2][0], best[2][1],
            "" if r["cells_speculative"] is None else ", speculative %.0f" % r["cells_speculative"],
            "" if r["held_in_lds"] is None else ", held in LDS %.0f" % r["held_in_lds"],
            r["microcells_per_move"], r["microcells_paper_mapping"],
            "" if r["microcells_speculative"] is None else ", speculative %.0f" % r["microcells_speculative"]))
        return r

    out = {"size_study": [], "cutoff_study": []}
    for n in sizes:
        out["size_study"].append(one(workloads.paper_size(n), 20_000))
    for wb in workloads.paper_cutoff(cutoffs):
        out["cutoff_study"].append(one(wb, 20_000))
    return out


def workload_by_name(name):
    from paper_1408_3764_amd import workloads
    return {"slab": workloads.slab, "large": workloads.large, "small": workloads.small}[name]()


def host_cores():
    """CPU cores this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def run_cpu_baseline(wb, budget_s, max_moves, **mode):
    """The oracle chain on the first moves of the same chain from the same
    configuration, sized to about budget_s of CPU time (a 10-move probe sets the
    sample size).  mode: the oracle's chain variant (threads=T: all pairs over
    T threads; mode="cells": its cell list); default the plain all-pairs loop."""
    import oracle
    p = oracle.make_params(wb.L, wb.rc, beta=wb.beta, mu=wb.mu, lambda3=wb.lambda3, max_disp=wb.max_disp,
                           p_disp=wb.p_disp)
    probe = 10 if mode.get("mode") != "cells" else 2000
    t = time.perf_counter()
    oracle.chain(wb.pos, probe, p, seed=wb.seed, max_n=wb.n + probe + 1, **mode)
    per = max((time.perf_counter() - t) / probe, 1e-7)
    n = int(max(20, min(max_moves, budget_s / per)))
    t = time.perf_counter()
    _, _, olog = oracle.chain(wb.pos, n, p, seed=wb.seed, max_n=wb.n + n + 1, **mode)
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
    ap.add_argument("--rows", type=int, default=0, help="with --waves: rows per wavefront; 0 = speculative rounds, -1 = pipelined kernel")
    ap.add_argument("--cpu-budget", type=float, default=10.0, help="seconds of oracle time per CPU mode")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the small-box chain and the mixture forward/backward")
    ap.add_argument("--no-allpairs", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="heuristic launch shape instead of timing them")
    ap.add_argument("--cell-sweep", action="store_true",
                    help="only compare traditional cells with pruned microcells on the small, large and slab boxes")
    ap.add_argument("--paper-studies", action="store_true",
                    help="only run the paper's size and cutoff studies (all pairs, cells, microcells)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (reference for the traffic counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "launches": 3}))
        return
    if args.paper_studies:
        print(json.dumps(paper_studies([2 ** 9, 2 ** 12, 2 ** 15, 2 ** 18, 2 ** 20],
                                        [2.5, 3.0, 3.5, 4.0, 4.25])))
        return
    if args.cell_sweep:
        print(json.dumps({"cell_sweep": cell_size_sweep()}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path here (one box's chain is a "
              "dependent sequence; independent boxes would shard by box). Use --gpus 1.", file=sys.stderr)
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
    total_moves = mps * (args.steps + args.warmup) + 40_000   # + the moves the tuner runs
    cell_m = None
    tuning = None
    if args.waves:
        box = Box.from_workload(wb, max_n=wb.n + total_moves + 1)
        box.set_launch(args.waves, args.rows)
        shape = (args.waves, args.rows)
    elif args.no_tune:
        box = Box.from_workload(wb, max_n=wb.n + total_moves + 1)
        shape = tune.chain_shape(box)
        box.set_launch(*shape)
    else:
        # cell size (the paper's cells, or twice as many per axis) and launch shape, every
        # candidate timed on its own box (the chain continues on the device counter)
        box, cell_m, shape, tuning = tune.autotune_cells(
            lambda cm: Box.from_workload(wb, max_n=wb.n + total_moves + 1, cell_m=cm))
        log("tuned cells %s, launch %dx%d: %s" % (box.info()["cell_m"], shape[0], shape[1],
                                                   {k: round(v * 1e3, 2) for k, v in tuning.items()}))
    info = box.info()
    nst = info["n_stencil"]
    U0 = box.total_energy()
    box.virial()
    log("box: cells %s cap %d stencil %d, launch %dx%d, U0=%.6f" % (info["cell_m"], info["cell_cap"], nst,
                                                                     shape[0], shape[1], U0["U_pair"]))
    from paper_1408_3764_amd import _lib
    from paper_1408_3764_amd._lib import COUNTER_CONTINUE, STATS_DTYPE
    stream = torch.cuda.current_stream()
    # the state every step starts from: the initial configuration, its energy and virial,
    # move counter c0 (the tuner leaves the box there)
    snap = box.snapshot()
    c0, n0 = snap[4]["counter"], snap[4]["n"]
    st_dev = torch.zeros(STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    for w in range(args.warmup):
        box.restore(snap)
        _lib.gcmc_step(box.handle, mps, c0, st_dev, None, box.stream)
    torch.cuda.synchronize()
    evs, walls, stats_all = [], [], []
    for k in range(args.steps):
        box.restore(snap)            # outside the timed region: N = n0 again, same counters
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        _lib.gcmc_step(box.handle, mps, c0, st_dev, None, box.stream)
        e1.record(stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        evs.append((e0, e1))
        stats_all.append(np.frombuffer(st_dev.cpu().numpy().tobytes(), dtype=STATS_DTYPE)[0].copy())
        log("step %d: N %d -> %d, %.2f ms, %.1f candidates/move" % (
            k, n0, int(stats_all[-1]["n"]), 1e3 * walls[-1], int(stats_all[-1]["candidates"]) / mps))
    wall = sum(walls)
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
    kname = {0: "k_chain_spec", -1: "k_chain_async"}.get(shape[1], "k_chain")
    traffic, traffic_src, traffic_ratio = measured_traffic(kname, shape, wb.name, mps)
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
        "config": {"workload": wb.name, "n": n0, "moves_per_step": mps, "rc": wb.rc, "T": 1.0 / wb.beta,
                   "mu": wb.mu, "cells": info["cell_m"], "cell_cap": info["cell_cap"], "stencil_cells": nst,
                   "launch": {"waves": shape[0], "rows": shape[1]},
                   "every_step_starts_from": "the initial configuration (N = %d, move counter %d)" % (n0, c0)},
        "n_start_per_step": [n0] * args.steps,
        "n_end_per_step": [int(s["n"]) for s in stats_all],
        "averages_last_step": {"n": float(stats_all[-1]["avg_n"]), "u": float(stats_all[-1]["avg_u"]),
                               "p": float(stats_all[-1]["avg_p"])},
        "pair_evals_per_s": pair_evals / wall,
        "in_cutoff_pairs_per_s": incut / wall,
        "candidates_per_move": cand / moves,
        "acceptance": {"displace": float(acc[0] / max(att[0], 1)), "insert": float(acc[1] / max(att[1], 1)),
                       "delete": float(acc[2] / max(att[2], 1))},
        "us_per_move": 1e6 * wall / moves,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": traffic_src, "traffic_over_alg_bytes": traffic_ratio,
                     "alg_bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": 1e3 * avg_launch_s},
    }

    # the cell-list build of the same box (binning, Sec. 3.2.1): counters cleared, every particle
    # claims a slot of its cell, cells ordered by particle id; algorithmic bytes per build: each
    # record read (32 B) and written into its cell (32 B) with its back-pointer (8 B), and the
    # counters cleared and incremented (8 B per cell)
    n_now = box.n
    box.cell_build()
    torch.cuda.synchronize()
    bts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        box.cell_build()
        e1.record(stream)
        torch.cuda.synchronize()
        bts.append(e0.elapsed_time(e1))
    b_ms = float(np.median(bts))
    b_bytes = 72.0 * n_now + 8.0 * info["n_cells"]
    out["cell_build"] = {"n": n_now, "cells": info["n_cells"], "ms_median": b_ms,
                         "particles_per_s": n_now / (b_ms / 1e3),
                         "roofline": {"bound": "hbm", "alg_bytes": b_bytes,
                                      "achieved": b_bytes / (b_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": b_bytes / (b_ms / 1e3) / 1e9 / HBM_PEAK_GBS}}
    log("cell-list build of %d particles in %d cells: %.3f ms" % (n_now, info["n_cells"], b_ms))

    if not args.no_allpairs:
        # the paper's comparison of its cell list with the no-cell-list GPU code, on the
        # 262,144-particle box (rc = 3.0): the same chain through both paths
        lw = wb if args.workload == "large" else workload_by_name("large")
        cb = Box.from_workload(lw, max_n=lw.n + 30001)
        cb.set_launch(*tune.chain_shape(cb))
        cb.step(1000, counter0=0)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        sc, _ = cb.step(20000, counter0=1000)
        torch.cuda.synchronize()
        dc = time.perf_counter() - tc
        cb.close()
        ab = Box.from_workload(lw, max_n=lw.n + 2001)
        ab.step(50, counter0=0, all_pairs=True)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        sa, _ = ab.step(1000, counter0=50, all_pairs=True)
        torch.cuda.synchronize()
        da = time.perf_counter() - ta
        ab.close()
        out["cell_vs_allpairs"] = {"workload": lw.name,
                                   "cell_list": {"moves_per_s": 20000 / dc, "pair_evals_per_s": int(sc["pair_evals"]) / dc},
                                   "all_pairs": {"moves_per_s": 1000 / da, "pair_evals_per_s": int(sa["pair_evals"]) / da},
                                   "speedup": (20000 / dc) / (1000 / da)}
        log("cell list vs all pairs at N=%d: %.0f vs %.0f moves/s" % (lw.n, 20000 / dc, 1000 / da))

    if not args.no_batched:
        from paper_1408_3764_amd import workloads
        tb = time.perf_counter()
        wbs = workloads.batched()
        log("batched: %d boxes, N total %d, generated in %.1fs" % (len(wbs), sum(w.n for w in wbs),
                                                                 time.perf_counter() - tb))
        boxes = [Box.from_workload(w, max_n=w.n + 3001, box_id=k) for k, w in enumerate(wbs)]
        bt = Batch(boxes)
        # launch shapes per box (uniform, or the largest boxes wider), each rule timed on identical
        # work; the boxes are left in their starting state with the fastest rule applied
        brule, btimes = tune.autotune_batch(bt, boxes, n_moves=300)
        bshape = tune.rule_name(brule)
        log("batched tuning (s per 300 moves/box): %s" % {k: round(v, 4) for k, v in btimes.items()})
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        tb = time.perf_counter()
        e0.record(stream)
        bst = bt.step(1000, counter0=COUNTER_CONTINUE)
        e1.record(stream)
        torch.cuda.synchronize()
        db = time.perf_counter() - tb
        bmoves = 1000 * len(boxes)
        binfo = [b.info() for b in boxes]
        b_alg = float(sum(resident_alg_bytes(wbs[k].n, int(bst[k]["n"]), binfo[k]["n_cells"])
                          if boxes[k].launch[1] == -3 else alg_bytes(bst[k], binfo[k]["n_stencil"])
                          for k in range(len(boxes))))
        shape_counts = {}
        for b in boxes:
            key = "%dx%d" % b.launch
            shape_counts[key] = shape_counts.get(key, 0) + 1
        b_ms = e0.elapsed_time(e1)
        out["batched"] = {"boxes": len(boxes), "moves_per_box": 1000, "moves_per_s": bmoves / db,
                          "pair_evals_per_s": float(np.sum(bst["pair_evals"])) / db,
                          "launch_ms": b_ms, "launch_rule": bshape, "launch_shapes": shape_counts,
                          "rule_timings_300_moves_s": btimes,
                          "errors": int(np.count_nonzero(bst["error"])),
                          "roofline": {"bound": "hbm", "alg_bytes_per_launch": b_alg,
                                       "achieved": b_alg / (b_ms / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": b_alg / (b_ms / 1e3) / 1e9 / HBM_PEAK_GBS}}
        # the same 1,000 moves per box as ten 100-move launches captured in one HIP graph
        # (device-side move counters), replayed once to warm up and once timed
        from paper_1408_3764_amd import _lib
        from paper_1408_3764_amd._lib import STATS_DTYPE
        gs = torch.cuda.Stream()
        gst = torch.zeros(len(boxes) * STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gs):
            for _ in range(10):
                _lib.gcmc_batch_step(bt.handle, 100, COUNTER_CONTINUE, gst, gs)
        graph.replay()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record()
        graph.replay()
        g1.record()
        torch.cuda.synchronize()
        g_ms = g0.elapsed_time(g1)
        gstats = np.frombuffer(gst.cpu().numpy().tobytes(), dtype=STATS_DTYPE)
        out["batched"]["graph"] = {"launches": 10, "moves_per_launch": 100, "replay_ms": g_ms,
                                   "moves_per_s": bmoves / (g_ms / 1e3),
                                   "errors": int(np.count_nonzero(gstats["error"]))}
        # one more 1,000-move launch on the chains as they now stand (3,000 moves past the initial
        # configurations: the densest boxes have lost a fifth or more of their particles), for
        # comparison with timings taken on continued chains
        c0e, c1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        c0e.record(stream)
        cst = bt.step(1000, counter0=COUNTER_CONTINUE)
        c1e.record(stream)
        torch.cuda.synchronize()
        out["batched"]["continued"] = {"moves_before": 3000, "launch_ms": c0e.elapsed_time(c1e),
                                       "n_total_before": int(sum(int(v) for v in gstats["n"])),
                                       "errors": int(np.count_nonzero(cst["error"]))}
        log("batched: one launch of 1,000 moves/box %.3f ms; graph of 10 x 100 moves/box %.3f ms; a further "
            "1,000-move launch on the continued chains %.3f ms" % (b_ms, g_ms, c0e.elapsed_time(c1e)))
        bt.close()
        for b in boxes:
            b.close()

    if not args.no_extra:
        out.update(extra_configs(Box, tune, stream))

    if not args.no_cpu:
        cores = host_cores()
        n_cpu, dt, olog = run_cpu_baseline(wb, args.cpu_budget, 20000)
        # the same moves on the GPU, for a parity check of the timed chain
        pb = Box.from_workload(wb, max_n=wb.n + n_cpu + 1, cell_m=cell_m)
        pb.set_launch(*shape)
        _, glog = pb.step(n_cpu, counter0=0, log=True)
        same = bool(np.array_equal(glog["type"], olog["type"]) and np.array_equal(glog["accepted"], olog["accepted"])
                    and np.array_equal(glog["index"], olog["index"]))
        pb.close()
        n_mt, dt_mt, _ = run_cpu_baseline(wb, args.cpu_budget, 20000, threads=cores)
        n_cl, dt_cl, _ = run_cpu_baseline(wb, args.cpu_budget, mps, mode="cells")
        out["cpu_baseline"] = {
            "value": n_cpu / dt, "unit": "moves/s", "cores": 1, "kind": "oracle", "host_cores": cores,
            "sample": "first %d moves of the same chain from the same initial configuration "
                      "(all-pairs FP64 oracle, one thread, %.1fs)" % (n_cpu, dt),
            "gpu_chain_matches_on_sample": same,
            "modes": {
                "all_pairs_1_thread": {"value": n_cpu / dt, "unit": "moves/s", "cores": 1, "moves": n_cpu,
                                       "seconds": dt},
                "all_pairs_all_cores": {"value": n_mt / dt_mt, "unit": "moves/s", "cores": cores, "moves": n_mt,
                                        "seconds": dt_mt,
                                        "note": "each position's sums split into contiguous particle ranges, "
                                                "one per thread, partials added in range order"},
                "cell_list_1_thread": {"value": n_cl / dt_cl, "unit": "moves/s", "cores": 1, "moves": n_cl,
                                       "seconds": dt_cl,
                                       "note": "the oracle's host cell list (linked cells on the paper's grid, "
                                               "27-cell stencils), the best CPU algorithm here; the first %d "
                                               "moves of the timed step" % n_cl},
            },
            "gpu_vs_cpu_cell_list": (moves / wall) / (n_cl / dt_cl),
        }
        log("CPU oracle: %.1f moves/s (1 thread, all pairs), %.1f (%d threads), %.0f (cell list, 1 thread)" % (
            n_cpu / dt, n_mt / dt_mt, cores, n_cl / dt_cl))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
