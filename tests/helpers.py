"""Shared comparison rules of the parity tests.

Tolerances (energy deltas, gradients) follow the readings fixed for this
build: a difference of sums is compared against the sum of the magnitudes of
its terms, since a relative test on a near-zero difference is meaningless.
"""
import math

import numpy as np

DU_REL = 1e-10          # per-move energy deltas
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


def compare_chain_logs(glog, olog, beta, what="chain"):
    """Move-by-move comparison.  Returns the number of moves compared; a
    different accept decision is allowed only at a near-tie (|ln A - arg| within
    10 beta of the energy tolerance), after which the chains may differ."""
    n = len(olog)
    assert len(glog) >= n
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
        assert abs(g["dU_tail"] - o["dU_tail"]) <= 1e-12 * max(1.0, abs(o["dU_tail"])), (what, m, "tail")
        if int(g["accepted"]) != int(o["accepted"]):
            lnA = math.log(o["a"]) if o["a"] > 0 else -math.inf
            near = abs(lnA - o["arg"]) <= 10 * beta * tol + 1e-12
            assert near, (what, m, "accept decision differs away from a tie")
            return m
    return n
