"""Launch-shape and cell-size selection for the move kernels.

The move kernel's shape is (waves per workgroup, candidate slots per lane per
pass).  A move's candidate slots are (stencil cells) x G, G = the power of two
at or above the fullest cell, doubled when a displacement leaves its cell; one
pass of W waves x R rows covers 64 W R slots, so the heuristic picks the
smallest workgroup that covers a cross-cell displacement in one pass (one
memory round trip), and :func:`autotune_chain` measures the candidates on a
copy of the box and caches the winner per workload shape.
"""
from __future__ import annotations

import json
import os
import time

SHAPES = [(1, 8), (2, 8), (4, 2), (4, 4), (4, 8), (8, 2), (8, 4)]
# rows = 0: the speculative kernel, W consecutive moves evaluated at once and
# committed in order (one species, stencils of at most 512 cells)
SPEC_SHAPES = [(2, 0), (4, 0), (8, 0), (16, 0)]
# rows = -1: the pipelined kernel, one committer and waves - 1 evaluator wavefronts
# (the same limits, plus at most 1024 cells per axis)
ASYNC_SHAPES = [(4, -1), (8, -1)]
# rows = -2: the paper's microcell mapping, one stencil cell per thread (any grid)
PAPER_SHAPES = [(4, -2), (8, -2)]
# rows = -3: the box held in LDS, every move evaluated against all other particles (one species;
# particles past RESIDENT_CAP are read from global memory, so it is offered to small boxes)
RESIDENT_SHAPES = [(4, -3), (8, -3)]
RESIDENT_CAP = 2048
SPEC_OWN = 8192   # flattened candidates the 32-cell path of the speculative kernel can hold
SPEC_MAX_STENCIL = 512   # stencil cells the speculative kernel takes (microcell path above 32)
CACHE_ENV = "GCMC_TUNE_CACHE"


def _slots(box):
    info = box.info()
    cell_of, count, _ = box.cells()
    maxc = int(count.max()) if len(count) else 1
    g = 1
    while g < maxc:
        g *= 2
    nst = info["n_stencil"]
    return nst * g


def spec_supported(box):
    info = box.info()
    return info["n_species"] == 1 and info["n_stencil"] <= SPEC_MAX_STENCIL


def resident_supported(box):
    return box.info()["n_species"] == 1


def async_supported(box):
    info = box.info()
    nst = info["n_stencil"]
    return (info["n_species"] == 1 and nst <= 32 and 2 * nst * info["cell_cap"] <= SPEC_OWN
            and max(info["cell_m"]) <= 1024)


def chain_shape(box):
    """The speculative kernel with eight wavefronts where it applies; otherwise
    the smallest per-move shape whose one pass covers the two stencils of a
    cross-cell displacement."""
    if spec_supported(box):
        return (8, 0)
    need = 2 * _slots(box)
    best = None
    for w, r in SHAPES:
        cover = 64 * w * r
        if cover >= need:
            key = (w * r, w)          # fewest slots per pass, then fewest waves
            if best is None or key < best[0]:
                best = (key, (w, r))
    return best[1] if best else (8, 4)


def batch_shape(boxes):
    """Batched boxes: one workgroup per box, a single wave when the stencil fits it."""
    need = max(_slots(b) for b in boxes[:8])
    for w, r in ((1, 8), (2, 8), (4, 4), (4, 8), (8, 4)):
        if 64 * w * r >= need:
            return (w, r)
    return (8, 4)


BATCH_RULES = [("uniform", (2, 0)), ("uniform", (4, 0)), ("uniform", (8, 0)), ("uniform", (4, 4)),
               ("split", 0.25, (8, 0), (4, 0)), ("split", 0.25, (8, 0), (2, 0)), ("split", 0.5, (4, 0), (2, 0)),
               ("cost", 0.125, (8, 0), (2, 0)), ("cost", 0.25, (8, 0), (2, 0)), ("cost", 0.125, (8, 0), (4, 0)),
               ("cost", 0.25, (4, 0), (2, 0)),
               ("lds", ((1024, (4, -3)),), ("uniform", (4, 0))), ("lds", ((1536, (4, -3)),), ("uniform", (4, 0))),
               ("lds", ((768, (4, -3)), (1536, (8, -3))), ("uniform", (4, 0))),
               ("lds", ((1024, (4, -3)), (2048, (8, -3))), ("uniform", (4, 0))),
               ("lds", ((768, (4, -3)), (1536, (8, -3))), ("split", 0.25, (8, 0), (4, 0)))]


def move_cost(box):
    """Candidates a move of the box reads, about: the particles in one stencil
    (the whole box when the stencil covers it)."""
    info = box.info()
    return box.n * min(1.0, info["n_stencil"] / max(1, info["n_cells"]))


def apply_batch_rule(boxes, rule):
    """Set every box's launch shape by a rule: ("uniform", shape); ("split",
    f, big, small): the fraction f of the boxes with the most particles take
    `big`, the others `small`; ("cost", f, big, small): the same, ranked by the
    candidates a move reads (move_cost); ("lds", ((n_1, shape_1), (n_2,
    shape_2), ...), rule): a box of at most n_1 particles held in LDS with
    shape_1, else of at most n_2 with shape_2, ..., the others by `rule`.
    A shape the box cannot take falls back to the per-move 4x4."""
    if rule[0] == "lds":
        _, tiers, inner = rule
        shapes = apply_batch_rule(boxes, inner)
        for k, b in enumerate(boxes):
            if not resident_supported(b):
                continue
            n = b.n
            for nmax, rshape in tiers:
                if n <= nmax:
                    b.set_launch(*rshape)
                    shapes[k] = rshape
                    break
        return shapes
    if rule[0] == "uniform":
        shapes = [rule[1]] * len(boxes)
    else:
        _, f, big, small = rule
        ns = [b.n for b in boxes] if rule[0] == "split" else [move_cost(b) for b in boxes]
        order = sorted(range(len(boxes)), key=lambda k: -ns[k])
        top = set(order[:max(1, int(round(f * len(boxes))))])
        shapes = [big if k in top else small for k in range(len(boxes))]
    for b, sh in zip(boxes, shapes):
        if sh[1] == 0 and not spec_supported(b):
            sh = (4, 4)
        b.set_launch(*sh)
    return shapes


def rule_name(rule):
    if rule[0] == "lds":
        return "lds" + ",".join("%d:%dx%d" % (n, sh[0], sh[1]) for n, sh in rule[1]) + "+" + rule_name(rule[2])
    if rule[0] == "uniform":
        return "%dx%d" % rule[1]
    return "%s%g:%dx%d/%dx%d" % ("top" if rule[0] == "split" else "cost", rule[1], rule[2][0], rule[2][1], rule[3][0],
                                 rule[3][1])


def _timed_launch(launch):
    """GPU time (s) of launch() on the current stream, from HIP events around it."""
    import torch
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def autotune_batch(batch, boxes, n_moves=300, rules=None):
    """Launch shapes of a batch: every rule of BATCH_RULES timed on identical
    work (each box's snapshot restored before the warm-up and before the timed
    launch, which continue each box's own counter; the launch timed with HIP
    events); the fastest rule is left applied and the boxes back in their
    starting state.  Returns (rule, timings keyed by rule_name)."""
    import numpy as np
    import torch
    from . import _lib
    from ._lib import COUNTER_CONTINUE, STATS_DTYPE
    rules = rules or BATCH_RULES
    snaps = [b.snapshot() for b in boxes]
    st = torch.zeros(len(boxes) * STATS_DTYPE.itemsize, dtype=torch.uint8, device=boxes[0].device)
    timings, best = {}, None
    for rule in rules:
        apply_batch_rule(boxes, rule)
        for b, sn in zip(boxes, snaps):
            b.restore(sn)
        batch.step(min(50, n_moves), counter0=COUNTER_CONTINUE)
        for b, sn in zip(boxes, snaps):
            b.restore(sn)
        torch.cuda.synchronize()
        dt = _timed_launch(lambda s: _lib.gcmc_batch_step(batch.handle, n_moves, COUNTER_CONTINUE, st, s))
        stats = np.frombuffer(st.cpu().numpy().tobytes(), dtype=STATS_DTYPE)
        if int((stats["error"] != 0).sum()):
            raise RuntimeError("chain error while tuning the batch")
        timings[rule_name(rule)] = dt
        if best is None or dt < best[0]:
            best = (dt, rule)
    apply_batch_rule(boxes, best[1])
    for b, sn in zip(boxes, snaps):
        b.restore(sn)
    torch.cuda.synchronize()
    return best[1], timings


def _cache_path():
    return os.environ.get(CACHE_ENV, "")


def autotune_live(box, n_moves=3000, shapes=None):
    """Time each launch shape on the box itself and leave the fastest set.
    Every shape runs identical work: the box's state is snapshotted first and
    put back before each shape's warm-up and before its timed launch, so each
    timing covers the same n_moves moves (same counters) from the same
    configuration; afterwards the box is back in that state.  Returns (shape,
    timings)."""
    import numpy as np
    import torch
    from . import _lib
    from ._lib import STATS_DTYPE
    if shapes is None:
        shapes = SHAPES + (SPEC_SHAPES if spec_supported(box) else []) + (ASYNC_SHAPES if async_supported(box) else [])
        if box.n <= RESIDENT_CAP and resident_supported(box):
            shapes = shapes + RESIDENT_SHAPES
    snap = box.snapshot()
    c0 = snap[4]["counter"]
    st_dev = torch.zeros(STATS_DTYPE.itemsize, dtype=torch.uint8, device=box.device)
    timings = {}
    best = None
    for w, r in shapes:
        box.set_launch(w, r)
        box.restore(snap)
        box.step(min(300, n_moves), counter0=c0)
        box.restore(snap)
        torch.cuda.synchronize()
        dt = _timed_launch(lambda s: _lib.gcmc_step(box.handle, n_moves, c0, st_dev, None, s))
        st = np.frombuffer(st_dev.cpu().numpy().tobytes(), dtype=STATS_DTYPE)[0]
        if int(st["error"]) != 0:
            raise RuntimeError("chain error %d while tuning" % int(st["error"]))
        timings["%dx%d" % (w, r)] = dt
        if best is None or dt < best[0]:
            best = (dt, (w, r))
    box.restore(snap)
    box.set_launch(*best[1])
    return best[1], timings


def autotune_cells(make_box, factors=(1, 2), n_moves=3000):
    """Cell size and launch shape together.  make_box(cell_m) builds the box:
    cell_m None gives the paper's cells (side >= rc, 27-cell stencils); factor
    f > 1 asks for f times as many cells per axis (microcells, whose stencils
    drop the cells beyond the cutoff).  Every launch shape that applies is
    timed on each box with autotune_live (identical work for every shape, the
    box left in its starting state); the fastest box is returned open with its
    shape set and the others are closed.  Returns (box, cell_m or None, shape, timings keyed
    "MxMxM/WxR")."""
    best = None
    base = None
    timings = {}
    for f in factors:
        cm = None if f == 1 else [f * m for m in base]
        b = make_box(cm)
        info = b.info()
        if base is None:
            base = info["cell_m"]
        shape, t = autotune_live(b, n_moves=n_moves)
        grid = "x".join(str(m) for m in info["cell_m"])
        for k, v in t.items():
            timings["%s/%s" % (grid, k)] = v
        dt = t["%dx%d" % shape]
        if best is None or dt < best[0]:
            if best is not None:
                best[1].close()
            best = (dt, b, cm, shape)
        else:
            b.close()
    best[1].set_launch(*best[3])
    return best[1], best[2], best[3], timings


def autotune_chain(make_box, n_moves=2000, shapes=SHAPES, key=None):
    """Time each launch shape on a fresh box from make_box() and return the fastest.
    Every shape runs the same chain (counter-based draws), so the comparison is
    between identical work.  The result is cached in $GCMC_TUNE_CACHE (JSON) under key."""
    import torch
    path = _cache_path()
    if key and path and os.path.exists(path):
        try:
            c = json.load(open(path))
            if key in c:
                return tuple(c[key]), {}
        except (OSError, ValueError):
            pass
    best = None
    timings = {}
    for w, r in shapes:
        b = make_box()
        b.set_launch(w, r)
        b.step(200, counter0=0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        b.step(n_moves, counter0=200)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        timings["%dx%d" % (w, r)] = dt
        if best is None or dt < best[0]:
            best = (dt, (w, r))
        b.close()
    if key and path:
        try:
            c = json.load(open(path)) if os.path.exists(path) else {}
        except (OSError, ValueError):
            c = {}
        c[key] = list(best[1])
        with open(path, "w") as f:
            json.dump(c, f)
    return best[1], timings
