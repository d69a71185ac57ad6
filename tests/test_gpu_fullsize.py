"""Parity at the full sizes of the five workloads, in the launch shapes the
benchmark uses, on outputs the oracle can compute one by one (a sample of
moves, of particles, of boxes), plus properties that hold at any size.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1408_3764_amd import tune, workloads
from tests.helpers import DU_REL, assert_du, chain_parity, compare_chain_logs

pytestmark = pytest.mark.gpu


def _params(wb):
    return oracle.make_params(wb.L, wb.rc, eps=wb.eps, sigma=wb.sigma, beta=wb.beta, mu=wb.mu, lambda3=wb.lambda3,
                              max_disp=wb.max_disp, p_disp=wb.p_disp)


def _box(wb, **kw):
    from paper_1408_3764_amd.box import Box
    return Box.from_workload(wb, **kw)


@pytest.fixture(scope="module")
def large():
    return workloads.large()


@pytest.fixture(scope="module")
def slab():
    return workloads.slab()


@pytest.fixture(scope="module")
def mixture():
    return workloads.mixture()


def _chain_check(wb, n_moves, shape=None):
    """n_moves of the chain from the workload's configuration, move for move
    against the oracle (a near-tie resyncs from the oracle's state), then the
    final configuration bit for bit."""
    p = _params(wb)
    b = _box(wb, max_n=wb.n + n_moves + 1)
    b.set_launch(*(shape or tune.chain_shape(b)))
    r = chain_parity(b, oracle, wb.pos, p, wb.seed, n_moves, wb.beta, wb.n + n_moves + 1, wb.name, U0=0.0)
    gpos, _ = b.particles()
    assert np.array_equal(gpos, r["opos"])
    return b, r


@pytest.mark.parametrize("shape", [None, (4, 4), (16, 0), (8, -1)])
def test_large_chain_matches_oracle(large, shape):
    """N=262,144, rc=3.0: 300 moves, bit-exact decisions (per-move and speculative kernels)."""
    _chain_check(large, 300, shape)


def test_large_deltas_cell_and_allpairs(large):
    from paper_1408_3764_amd.box import make_moves
    p = _params(large)
    rng = np.random.default_rng(11)
    m = 120
    types = rng.integers(0, 3, m)
    idx = rng.integers(0, large.n, m)
    pts = np.mod(large.pos[idx] + rng.uniform(-0.3, 0.3, (m, 3)), large.L)
    pts = np.where(types[:, None] == 1, rng.random((m, 3)) * large.L, pts)
    mv = make_moves(types, idx, pts)
    b = _box(large, max_n=large.n + 10)
    gc, tc = b.delta_energy(mv)
    ga, ta = b.delta_energy(mv, all_pairs=True)
    ref, scale = [], []
    for k in range(m):
        t, i = int(types[k]), int(idx[k])
        if t == 0:
            a = oracle.position_energy(large.pos, p, pts[k], exclude=i)
            c = oracle.position_energy(large.pos, p, large.pos[i], exclude=i)
            ref.append(a[0] - c[0]); scale.append(a[1] + c[1])
        elif t == 1:
            a = oracle.position_energy(large.pos, p, pts[k])
            ref.append(a[0]); scale.append(a[1])
        else:
            c = oracle.position_energy(large.pos, p, large.pos[i], exclude=i)
            ref.append(-c[0]); scale.append(c[1])
    assert_du(gc, ref, scale, "large, cell list")
    assert_du(ga, ref, scale, "large, all pairs")


def test_large_allpairs_chain(large):
    p = _params(large)
    b = _box(large, max_n=large.n + 101)
    _, glog = b.step(100, counter0=0, log=True, all_pairs=True)
    _, _, olog = oracle.chain(large.pos, 100, p, seed=large.seed, max_n=large.n + 101)
    assert compare_chain_logs(glog, olog, large.beta, "large all-pairs chain") == 100


def test_large_total_energy_sampled(large):
    p = _params(large)
    b = _box(large)
    cell = b.total_energy(per_particle=True)
    ap = b.total_energy(all_pairs=True)
    # the cell list and the all-pairs kernel agree on U (1e-10 of the magnitude sum)
    scale = 0.5 * np.abs(cell["e"]).sum()
    assert abs(cell["U_pair"] - ap["U_pair"]) <= 1e-10 * scale
    assert cell["U_pair"] == pytest.approx(0.5 * math.fsum(cell["e"]), rel=1e-12)
    rng = np.random.default_rng(4)
    for i in rng.choice(large.n, 150, replace=False):
        e, s = oracle.position_energy(large.pos, p, large.pos[i], exclude=i)
        assert abs(cell["e"][i] - e) <= 1e-10 * s
    assert cell["U_tail"] == pytest.approx(oracle.tail_energy([large.n], p), rel=1e-13)


@pytest.mark.parametrize("shape", [None, (4, 4), (16, 0), (8, -1)])
def test_slab_chain_matches_oracle(slab, shape):
    """The 1.5M-particle slab: 150 moves, bit-exact decisions (per-move and speculative kernels)."""
    _chain_check(slab, 150, shape)


@pytest.mark.parametrize("bshape", [None, (4, 0)])
def test_batched_sample_matches_oracle(bshape):
    """512 boxes advanced together in one launch (the per-move heuristic shape, and the
    speculative 4x0 the benchmark's tuner picks); every 16th box, the largest and the
    smallest checked against the oracle's chain (final configuration, acceptances)."""
    from paper_1408_3764_amd.box import Batch, Box
    wbs = workloads.batched()
    boxes = [Box.from_workload(w, max_n=w.n + 1001, box_id=k) for k, w in enumerate(wbs)]
    shape = bshape or tune.batch_shape(boxes)
    for b in boxes:
        b.set_launch(*shape)
    bt = Batch(boxes)
    stats = bt.step(1000, counter0=0)
    assert np.all(stats["error"] == 0) and np.all(stats["moves_done"] == 1000)
    ns = np.array([w.n for w in wbs])
    pick = sorted({int(np.argmax(ns)), int(np.argmin(ns)), 511} | set(range(0, 512, 16)))
    for k in pick:
        w = wbs[k]
        p = _params(w)
        opos, _, olog = oracle.chain(w.pos, 1000, p, seed=w.seed, box=k, max_n=w.n + 1001)
        gpos, _ = boxes[k].particles()
        assert np.array_equal(gpos, opos), k
        assert [int(v) for v in stats[k]["accepts"]] == [
            int(((olog["type"] == t) & (olog["accepted"] == 1)).sum()) for t in range(3)]
    bt.close()


def test_mixture_forward_backward(mixture):
    """Binary mixture, N=262,144: energy and gradients on sampled particles,
    Newton's third law, eps-homogeneity and finite differences of the parameters."""
    w = mixture
    p = _params(w)
    b = _box(w)
    fw = b.total_energy(per_particle=True)
    bw = b.backward()
    rng = np.random.default_rng(8)
    # the configured 4,096-particle subsample: the oracle's analytic gradient, and e_i on a quarter of it
    sample = rng.choice(w.n, 4096, replace=False)
    for q, i in enumerate(sample):
        if q % 4 == 0:
            e, s = oracle.position_energy(w.pos, p, w.pos[i], exclude=i, species=w.species,
                                          point_species=int(w.species[i]))
            assert abs(fw["e"][i] - e) <= 1e-10 * s
        g = oracle.particle_gradient(w.pos, i, p, species=w.species)
        assert np.allclose(bw["grad"][i], g, rtol=1e-7, atol=1e-7 * max(1.0, np.abs(g).max())), i
    G = bw["grad"]
    assert np.abs(G.sum(axis=0)).max() <= 1e-9 * np.abs(G).sum()
    U = fw["U_pair"] + fw["U_tail"]
    assert (w.eps * bw["d_eps"]).sum() == pytest.approx(U, rel=1e-10)
    # central differences of U in each unique parameter (the tables stay symmetric)
    h = 1e-6
    for (a, c) in ((0, 0), (0, 1), (1, 1)):
        E = np.zeros((2, 2)); E[a, c] = E[c, a] = 1.0
        vals = []
        for sgn in (+1, -1):
            b.set_params(w.eps + sgn * h * E, w.sigma)
            t = b.total_energy()
            vals.append(t["U_pair"] + t["U_tail"])
        fd_e = (vals[0] - vals[1]) / (2 * h)
        vals = []
        for sgn in (+1, -1):
            b.set_params(w.eps, w.sigma + sgn * h * E)
            t = b.total_energy()
            vals.append(t["U_pair"] + t["U_tail"])
        fd_s = (vals[0] - vals[1]) / (2 * h)
        b.set_params(w.eps, w.sigma)
        want_e = bw["d_eps"][a, c] + (bw["d_eps"][c, a] if a != c else 0.0)
        want_s = bw["d_sigma"][a, c] + (bw["d_sigma"][c, a] if a != c else 0.0)
        assert fd_e == pytest.approx(want_e, rel=1e-7)
        assert fd_s == pytest.approx(want_s, rel=1e-6)


def test_mixture_position_fd(mixture):
    """dU/dr_i against central differences of the energy (h = 1e-6) on the
    configured 4,096-particle subsample, skipping particles with a neighbour
    within 10 h of the cutoff (the truncation makes U jump there).  The
    differences come from the GPU's energy changes of displacements by +-h;
    at a sample of those points they are also checked against the oracle's."""
    from paper_1408_3764_amd.box import make_moves
    w = mixture
    p = _params(w)
    b = _box(w)
    g = b.backward(params=False)["grad"]
    h = 1e-6
    rng = np.random.default_rng(21)
    sample = rng.choice(w.n, 4096, replace=False)
    keep = []
    for i in sample:
        d = w.pos - w.pos[i]
        d -= w.L * np.round(d / w.L)
        r = np.sqrt((d * d).sum(axis=1))
        if not np.any(np.abs(r - w.rc) < 10 * h):
            keep.append(int(i))
    assert len(keep) >= 4000
    pts, idx = [], []
    for i in keep:
        for a in range(3):
            for sgn in (+1, -1):
                q = w.pos[i].copy()
                q[a] += sgn * h
                pts.append(np.mod(q, w.L))
                idx.append(i)
    mv = make_moves([0] * len(idx), idx, pts)
    dp, _ = b.delta_energy(mv)
    fd = ((dp[0::2] - dp[1::2]) / (2 * h)).reshape(-1, 3)
    for k, i in enumerate(keep):
        assert np.allclose(fd[k], g[i], rtol=1e-7, atol=1e-6), (i, fd[k], g[i])
    for k in range(0, len(keep), 256):
        i = keep[k]
        for j in range(6):
            s_i = int(w.species[i])
            en = oracle.position_energy(w.pos, p, pts[6 * k + j], exclude=i, species=w.species, point_species=s_i)
            eo = oracle.position_energy(w.pos, p, w.pos[i], exclude=i, species=w.species, point_species=s_i)
            assert abs(dp[6 * k + j] - (en[0] - eo[0])) <= DU_REL * (en[1] + eo[1])


def test_autograd_function():
    from paper_1408_3764_amd.autograd import lj_energy
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    w = workloads.random_box(300, 11.0, rc=3.0, seed=17, species_counts=[150, 150], eps=eps, sigma=sig)
    b = _box(w)
    pos = torch.tensor(w.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    E = torch.tensor(eps, dtype=torch.float64, device="cuda", requires_grad=True)
    S = torch.tensor(sig, dtype=torch.float64, device="cuda", requires_grad=True)
    U = lj_energy(pos, E, S, b)
    U.backward()
    p = _params(w)
    t = oracle.total_energy(w.pos, p, species=w.species)
    assert float(U.detach()) == pytest.approx(t["U_pair"] + t["U_tail"], rel=1e-11)
    g, de, ds = oracle.gradients(w.pos, p, species=w.species)
    assert np.allclose(pos.grad.cpu().numpy(), g, rtol=1e-7, atol=1e-9 * np.abs(g).max())
    assert np.allclose(E.grad.cpu().numpy(), de, rtol=1e-7)
    assert np.allclose(S.grad.cpu().numpy(), ds, rtol=1e-7)
    # a second forward at moved positions and changed parameters
    pos2 = torch.tensor(np.mod(w.pos + 0.01, w.L), dtype=torch.float64, device="cuda", requires_grad=True)
    U2 = lj_energy(pos2, E * 1.1, S, b)
    t2 = oracle.total_energy(np.mod(w.pos + 0.01, w.L), oracle.make_params(w.L, w.rc, eps=eps * 1.1, sigma=sig),
                             species=w.species)
    assert float(U2) == pytest.approx(t2["U_pair"] + t2["U_tail"], rel=1e-11)


@pytest.mark.parametrize("mixed", [False, True])
def test_graph_replay_continues_the_chain(mixed):
    """Batched steps captured in a HIP graph (device-side move counters) and
    replayed several times, with eager work in between, equal the eager chain;
    also with one launch shape per box (three launch groups on forked streams
    inside the graph)."""
    from paper_1408_3764_amd.box import Batch, Box
    from paper_1408_3764_amd._lib import COUNTER_CONTINUE
    wbs = [workloads.cubic_box(n, rho, 1.2, 2.5, 900 + k) for k, (n, rho) in
           enumerate([(300, 0.5), (800, 0.6), (150, 0.4)])]

    def mk():
        bs = [Box.from_workload(w, max_n=w.n + 2001, box_id=k, seed=5) for k, w in enumerate(wbs)]
        if mixed:
            for b, sh in zip(bs, [(8, 0), (4, 4), (2, 0)]):
                b.set_launch(*sh)
        return bs
    eager, graphed = mk(), mk()
    be, bg = Batch(eager), Batch(graphed)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    from paper_1408_3764_amd import _lib
    st = torch.zeros(len(wbs) * _lib.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    bg.step(10, counter0=0)        # first call uploads descriptors outside the capture
    be.step(10, counter0=0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(4):
            _lib.gcmc_batch_step(bg.handle, 25, COUNTER_CONTINUE, st, s)
    torch.cuda.synchronize()
    done = 10
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        be.step(100, counter0=done)
        done += 100
        torch.cuda.synchronize()
        for a, c in zip(eager, graphed):
            assert np.array_equal(a.particles()[0], c.particles()[0]), rep
        _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
    be.close(); bg.close()


def test_checkpoint_inside_graph_replays_resumes_the_chain():
    """Algorithm 1's periodic dumps with the chain on the device: a batch is
    advanced by replays of a captured HIP graph; halfway through, every box is
    exported (particles, running energy and virial, move counter, cumulative
    statistics), imported into fresh boxes, and those continue with the device
    counter.  The result equals the uninterrupted chain: configurations bit for
    bit, checkpoints (counter, sums, acceptances) equal."""
    from paper_1408_3764_amd import _lib
    from paper_1408_3764_amd.box import Batch, Box
    from paper_1408_3764_amd._lib import COUNTER_CONTINUE
    wbs = [workloads.cubic_box(n, rho, 1.2, 2.5, 700 + k) for k, (n, rho) in
           enumerate([(400, 0.5), (1200, 0.7), (200, 0.3)])]
    mk = lambda: [Box.from_workload(w, max_n=w.n + 3001, box_id=k, seed=13) for k, w in enumerate(wbs)]
    whole, first = mk(), mk()
    for b in whole + first:
        b.set_launch(4, 0)
        b.total_energy()
        b.virial()
    bw, bf = Batch(whole), Batch(first)
    st = torch.zeros(len(wbs) * _lib.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    bf.step(0, counter0=COUNTER_CONTINUE)   # descriptors uploaded outside the capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(2):
            _lib.gcmc_batch_step(bf.handle, 100, COUNTER_CONTINUE, st, s)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
    # 600 moves per box: checkpoint, then resume in fresh boxes for 600 more
    saved = [b.export_state() for b in first]
    assert all(ck["counter"] == 600 and ck["moves"] == 600 for _, _, ck in saved)
    resumed = [Box.from_workload(w, max_n=w.n + 3001, box_id=k, seed=13) for k, w in enumerate(wbs)]
    for b, (pos, sp, ck) in zip(resumed, saved):
        b.set_launch(4, 0)
        b.import_state(pos, ck, species=sp)
    br = Batch(resumed)
    br.step(0, counter0=COUNTER_CONTINUE)
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2, stream=s):
        for _ in range(2):
            _lib.gcmc_batch_step(br.handle, 100, COUNTER_CONTINUE, st, s)
    for _ in range(3):
        g2.replay()
        torch.cuda.synchronize()
    bw.step(1200, counter0=0)
    torch.cuda.synchronize()
    for a, c in zip(whole, resumed):
        assert np.array_equal(a.particles()[0], c.particles()[0])
        ca, cc = a.checkpoint(), c.checkpoint()
        for k in ("n", "counter", "moves", "attempts", "accepts", "sum_n", "sum_n2"):
            assert ca[k] == cc[k], k
        for k in ("u_pair", "w_pair", "sum_u", "sum_w"):
            assert cc[k] == pytest.approx(ca[k], rel=1e-12, abs=1e-9), k
    for bt in (bw, bf, br):
        bt.close()


def test_autograd_backward_after_another_forward():
    """Two forwards on one box, then backward on the first: the gradient is the
    first configuration's (the saved inputs are put back into the box)."""
    from paper_1408_3764_amd.autograd import lj_energy
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    w = workloads.random_box(300, 11.0, rc=3.0, seed=19, species_counts=[150, 150], eps=eps, sigma=sig)
    b = _box(w)
    pos1 = torch.tensor(w.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    E = torch.tensor(eps, dtype=torch.float64, device="cuda", requires_grad=True)
    S = torch.tensor(sig, dtype=torch.float64, device="cuda", requires_grad=True)
    U1 = lj_energy(pos1, E, S, b)
    moved = np.mod(w.pos + 0.05, w.L)
    pos2 = torch.tensor(moved, dtype=torch.float64, device="cuda", requires_grad=True)
    U2 = lj_energy(pos2, E * 1.3, S, b)
    U1.backward()
    p = _params(w)
    g, de, ds = oracle.gradients(w.pos, p, species=w.species)
    assert np.allclose(pos1.grad.cpu().numpy(), g, rtol=1e-7, atol=1e-9 * np.abs(g).max())
    assert np.allclose(E.grad.cpu().numpy(), de, rtol=1e-7)
    assert np.allclose(S.grad.cpu().numpy(), ds, rtol=1e-7)
    pos1.grad = None
    U2.backward()
    g2, _, _ = oracle.gradients(moved, oracle.make_params(w.L, w.rc, eps=eps * 1.3, sigma=sig), species=w.species)
    assert np.allclose(pos2.grad.cpu().numpy(), g2, rtol=1e-7, atol=1e-9 * np.abs(g2).max())
