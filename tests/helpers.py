"""Shared comparison rules of the parity tests.

Tolerances (energy deltas, gradients) follow the readings fixed for this
build: a difference of sums is compared against the sum of the magnitudes of
its terms, since a relative test on a near-zero difference is meaningless.
"""
import math

import numpy as np

DU_REL = 1e-10          # per-move energy (and virial) deltas
GRAD_REL = 1e-7         # gradients


def du_close(got, ref, sumabs, rel=DU_REL):
    return abs(got - ref) <= rel * max(abs(ref), sumabs) + 1e-300


def assert_du(got, ref, sumabs, what="", rel=DU_REL):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    sumabs = np.asarray(sumabs, dtype=np.float64)
    lim = rel * np.maximum(np.abs(ref), sumabs)
    bad = ~(np.abs(got - ref) <= lim)
    bad &= ~(np.isinf(got) & np.isinf(ref) & (np.sign(got) == np.sign(ref)))
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise AssertionError("%s: %d mismatches, first at %d: gpu=%r oracle=%r scale=%r" %
                             (what, int(bad.sum()), i, got[i], ref[i], max(abs(ref[i]), sumabs[i])))


def near_tie(o, beta):
    """The oracle's decision at log record o lies within the tie band
    |ln A - arg| <= 10 beta tol_dU (GPU and glibc exp/log may differ by an ulp,
    and the sums' order differs)."""
    tol = DU_REL * max(abs(o["dU_pair"]), o["sumabs"])
    lnA = math.log(o["a"]) if o["a"] > 0 else -math.inf
    return abs(lnA - o["arg"]) <= 10 * beta * tol + 1e-12


def compare_chain_logs(glog, olog, beta, what="chain"):
    """Move-by-move comparison.  Returns the number of moves compared; a
    different accept decision is allowed only at a near-tie, where the
    comparison stops (the caller resyncs, see chain_parity)."""
    n = len(olog)
    assert len(glog) >= n
    has_w = "dW_pair" in glog.dtype.names and "wsumabs" in olog.dtype.names
    for m in range(n):
        g, o = glog[m], olog[m]
        assert int(g["type"]) == int(o["type"]), (what, m, "type")
        assert int(g["index"]) == int(o["index"]), (what, m, "index", int(g["index"]), int(o["index"]))
        assert int(g["flags"]) == int(o["flags"]), (what, m, "flags")
        if int(o["flags"]) & 1:
            assert int(g["accepted"]) == 0
            continue
        assert (g["x"], g["y"], g["z"]) == (o["x"], o["y"], o["z"]), (what, m, "trial position")
        tol = DU_REL * max(abs(o["dU_pair"]), o["sumabs"])
        if not (math.isinf(o["dU_pair"]) and math.isinf(g["dU_pair"])):
            assert abs(g["dU_pair"] - o["dU_pair"]) <= tol + 1e-300, (what, m, g["dU_pair"], o["dU_pair"], tol)
            if has_w:
                tw = DU_REL * max(abs(o["dW_pair"]), o["wsumabs"])
                assert abs(g["dW_pair"] - o["dW_pair"]) <= tw + 1e-300, (what, m, "dW", g["dW_pair"], o["dW_pair"])
        assert abs(g["dU_tail"] - o["dU_tail"]) <= 1e-12 * max(1.0, abs(o["dU_tail"])), (what, m, "tail")
        if int(g["accepted"]) != int(o["accepted"]):
            assert near_tie(o, beta), (what, m, "accept decision differs away from a tie")
            return m
    return n


def chain_parity(box, orc, start, p, seed, n_moves, beta, max_n, what="chain", U0=None, W0=None, max_ties=3):
    """Run n_moves of the GPU chain from `start` (box freshly created from it,
    counter 0) and of the oracle chain, and compare them move by move.  At a
    near-tie whose decisions differ, the tie is recorded, the oracle's state
    after that move is imported into the box and both continue from there
    (the resync reading of near-ties).  Returns a dict: the oracle's final
    positions, energy and log ("opos", "oU", "olog"), the tie moves ("ties"),
    and the box's statistics of its last step ("stats"); fails on any
    difference away from a tie."""
    if U0 is None:
        t0 = orc.total_energy(start, p)
        U0 = t0["U_pair"] + t0["U_tail"]
    opos, oU, olog = orc.chain(start, n_moves, p, seed=seed, max_n=max_n, U0=U0)
    ties = []
    m0 = 0
    while True:
        stats, glog = box.step(n_moves - m0, counter0=m0, log=True)
        k = compare_chain_logs(glog, olog[m0:], beta, what)
        if k == n_moves - m0:
            return {"opos": opos, "oU": oU, "olog": olog, "ties": ties, "stats": stats}
        m = m0 + k
        ties.append(m)
        assert len(ties) <= max_ties, (what, "too many near-ties", ties)
        # the oracle's state after move m, into the box; continue at move m + 1
        spos, sU, slog = orc.chain(start, m + 1, p, seed=seed, max_n=max_n, U0=U0)
        n = len(spos)
        tail = orc.tail_energy([n], p)
        ck = {"n": n, "u_pair": sU - tail, "w_pair": 0.0, "counter": m + 1, "moves": 0, "attempts": [0, 0, 0],
              "accepts": [0, 0, 0], "sum_n": 0.0, "sum_n2": 0.0, "sum_u": 0.0, "sum_w": 0.0, "error": 0,
              "error_move": -1}
        box.import_state(spos, ck)
        m0 = m + 1
