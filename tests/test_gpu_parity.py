"""Parity of the gfx950 library (through its C ABI) with the CPU oracle.

Bit-exact: cell assignment, cell membership, neighbour sets, chain decisions
(move types, indices, trial positions, accept/reject away from ties), final
configurations.  Within tolerance: energy deltas (1e-10 of the magnitude sum),
total energies, gradients (1e-7).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1408_3764_amd import workloads
from tests.helpers import assert_du, chain_parity, compare_chain_logs, DU_REL

pytestmark = pytest.mark.gpu


def _box(wb, **kw):
    from paper_1408_3764_amd.box import Box
    return Box.from_workload(wb, **kw)


def _params(wb, **over):
    kw = dict(eps=wb.eps, sigma=wb.sigma, beta=wb.beta, mu=wb.mu, lambda3=wb.lambda3, max_disp=wb.max_disp,
              p_disp=wb.p_disp)
    kw.update(over)
    return oracle.make_params(wb.L, wb.rc, **kw)


SMALL_CASES = {
    "L10_M4": dict(n=300, L=10.0, seed=1),
    "L7.4_M3_whole_box": dict(n=120, L=7.4, seed=2),
    "aniso": dict(n=250, L=[7.6, 10.0, 12.7], seed=3),
    "L12.7": dict(n=500, L=12.7, seed=4),
}


@pytest.fixture(scope="module")
def c1():
    return workloads.small()


def _random_moves(wb, rng, m, n):
    from paper_1408_3764_amd.box import make_moves
    types = rng.integers(0, 3, m)
    idx = rng.integers(0, n, m)
    pos = rng.random((m, 3)) * wb.L
    disp = wb.pos[idx] + rng.uniform(-0.3, 0.3, (m, 3))
    disp = np.mod(disp, wb.L)
    disp = np.where(disp >= wb.L, 0.0, disp)
    # a third of the displacements are large jumps (cross-cell)
    far = rng.random(m) < 0.3
    disp[far] = pos[far]
    p = np.where((types == 0)[:, None], disp, pos)
    return make_moves(types, idx, p)


def _oracle_deltas(wb, p, moves):
    dp, dt, sa = [], [], []
    n = wb.n
    counts = [n] if wb.species is None else np.bincount(wb.species, minlength=wb.eps.shape[0])
    for mv in moves:
        t, i = int(mv["type"]), int(mv["index"])
        pt = (mv["x"], mv["y"], mv["z"])
        sp = None if wb.species is None else wb.species
        if t == 0:
            s_i = 0 if sp is None else int(sp[i])
            eo = oracle.position_energy(wb.pos, p, wb.pos[i], exclude=i, species=sp, point_species=s_i)
            en = oracle.position_energy(wb.pos, p, pt, exclude=i, species=sp, point_species=s_i)
            dp.append(en[0] - eo[0]); sa.append(en[1] + eo[1]); dt.append(0.0)
        elif t == 1:
            s_i = int(mv["species"])
            en = oracle.position_energy(wb.pos, p, pt, exclude=-1, species=sp, point_species=s_i)
            dp.append(en[0]); sa.append(en[1]); dt.append(oracle.tail_delta(counts, s_i, +1, p))
        else:
            s_i = 0 if sp is None else int(sp[i])
            eo = oracle.position_energy(wb.pos, p, wb.pos[i], exclude=i, species=sp, point_species=s_i)
            dp.append(-eo[0]); sa.append(eo[1]); dt.append(oracle.tail_delta(counts, s_i, -1, p))
    return np.array(dp), np.array(dt), np.array(sa)


# ------------------------------------------------------------------ cells
@pytest.mark.parametrize("case", list(SMALL_CASES))
def test_cell_assignment_bitexact(case):
    c = SMALL_CASES[case]
    wb = workloads.random_box(c["n"], c["L"], seed=c["seed"])
    b = _box(wb)
    cell_of, count, ids = b.cells()
    ref = oracle.cell_of(wb.pos, wb.L, wb.rc)
    assert np.array_equal(cell_of.astype(np.int64), ref)
    assert np.array_equal(count, np.bincount(ref, minlength=len(count)))
    for cidx in np.nonzero(count)[0]:
        assert sorted(ids[cidx, : count[cidx]].tolist()) == sorted(np.nonzero(ref == cidx)[0].tolist())
    g = oracle.grid(wb.L, wb.rc)
    assert b.info()["cell_m"] == list(g["M"]) and b.info()["span"] == list(g["span"])


@pytest.mark.parametrize("cap", [0, 100])
def test_cell_build_both_sort_paths(cap):
    """The cell build orders entries with one wavefront per cell up to 64 slots per
    cell and with one thread per cell above that; both give the oracle's cells,
    id order inside each cell, and species counts (checked through U_tail)."""
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    wb = workloads.random_box(500, 11.0, rc=3.0, seed=12, species_counts=[250, 250], eps=eps, sigma=sig)
    b = _box(wb, cell_cap=cap)
    assert (b.info()["cell_cap"] > 64) == (cap == 100)
    cell_of, count, ids = b.cells()
    ref = oracle.cell_of(wb.pos, wb.L, wb.rc)
    assert np.array_equal(cell_of.astype(np.int64), ref)
    for cidx in np.nonzero(count)[0]:
        assert ids[cidx, : count[cidx]].tolist() == sorted(np.nonzero(ref == cidx)[0].tolist())
    t = oracle.total_energy(wb.pos, _params(wb), species=wb.species)
    assert b.total_energy()["U_tail"] == pytest.approx(t["U_tail"], rel=1e-13)


def test_cell_assignment_c1_exact_grid(c1):
    b = _box(c1)
    assert b.info()["cell_m"] == [8, 8, 8]
    cell_of, count, _ = b.cells()
    assert np.array_equal(cell_of.astype(np.int64), oracle.cell_of(c1.pos, c1.L, c1.rc))


@pytest.mark.parametrize("case", list(SMALL_CASES))
def test_neighbor_sets_bitexact(case):
    c = SMALL_CASES[case]
    wb = workloads.random_box(c["n"], c["L"], seed=c["seed"])
    b = _box(wb)
    rng = np.random.default_rng(c["seed"])
    g = oracle.grid(wb.L, wb.rc)
    pts = [wb.pos[i] for i in range(0, wb.n, 7)]
    excl = list(range(0, wb.n, 7))
    for _ in range(20):   # random points and points within an ulp of cell faces
        q = rng.random(3) * wb.L
        a = rng.integers(0, 3)
        face = rng.integers(0, g["M"][a]) * (wb.L[a] / g["M"][a])
        q[a] = min(max(face + rng.choice([-1e-12, 0.0, 1e-12]), 0.0), np.nextafter(wb.L[a], 0))
        pts.append(q)
        excl.append(-1)
    got, cnt = b.neighbor_ids(np.array(pts), np.array(excl))
    for k, (q, ex) in enumerate(zip(pts, excl)):
        ref = oracle.neighbor_ids(wb.pos, q, wb.L, wb.rc, exclude=ex)
        assert cnt[k] == len(ref)
        assert np.array_equal(got[k], np.sort(ref)), (k, q)


@pytest.mark.parametrize("req", [[8, 8, 8], [12, 12, 12], [13, 17, 21], [3, 9, 14]])
def test_neighbor_sets_small_cells(req):
    """Cells smaller than rc (k = 2 .. 5 per axis; the stencil less the cells
    beyond the cutoff; one case covers x whole) give the oracle's sets, and
    the library keeps the oracle's number of stencil cells."""
    wb = workloads.random_box(400, 11.0, seed=9)
    req = np.array(req, dtype=np.int32)
    b = _box(wb, cell_m=req)
    g = oracle.grid(wb.L, wb.rc, req)
    assert b.info()["span"] == list(g["span"])
    assert b.info()["n_stencil"] == oracle.stencil_count(wb.L, wb.rc, req)
    got, cnt = b.neighbor_ids(wb.pos[:50], np.arange(50))
    for i in range(50):
        ref = oracle.neighbor_ids(wb.pos, wb.pos[i], wb.L, wb.rc, exclude=i, req_m=req)
        assert np.array_equal(got[i], np.sort(ref))


# ----------------------------------------------------------- energy deltas
@pytest.mark.parametrize("case", list(SMALL_CASES))
@pytest.mark.parametrize("all_pairs", [False, True])
def test_delta_energy_parity(case, all_pairs):
    c = SMALL_CASES[case]
    wb = workloads.random_box(c["n"], c["L"], seed=c["seed"])
    p = _params(wb)
    b = _box(wb, max_n=wb.n + 10)
    rng = np.random.default_rng(100 + c["seed"])
    moves = _random_moves(wb, rng, 300, wb.n)
    gp, gt = b.delta_energy(moves, all_pairs=all_pairs)
    rp, rt, sa = _oracle_deltas(wb, p, moves)
    assert_du(gp, rp, sa, "dU_pair %s" % case)
    assert np.allclose(gt, rt, rtol=1e-12, atol=1e-15)


def test_delta_energy_c1_and_small_cells(c1):
    p = _params(c1)
    rng = np.random.default_rng(7)
    moves = _random_moves(c1, rng, 400, c1.n)
    rp, rt, sa = _oracle_deltas(c1, p, moves)
    for cm in (None, [16, 16, 16], [21, 21, 21], [24, 24, 24]):
        b = _box(c1, max_n=c1.n + 10, cell_m=cm)
        gp, gt = b.delta_energy(moves)
        assert_du(gp, rp, sa, "C1 cell_m=%s" % cm)
        assert np.allclose(gt, rt, rtol=1e-12)


@pytest.mark.parametrize("waves,rows", [(1, 8), (2, 8), (4, 2), (4, 8), (8, 4), (2, 0), (4, 0), (8, 0), (16, 0),
                                        (4, -1), (8, -1), (4, -2), (8, -2), (4, -3), (8, -3)])
def test_chain_launch_shapes_agree(c1, waves, rows):
    """Every launch shape gives the oracle's chain (the tuner may pick any)."""
    p = _params(c1)
    _, _, olog = oracle.chain(c1.pos, 300, p, seed=c1.seed, max_n=c1.n + 400,
                              U0=0.0)
    b = _box(c1, max_n=c1.n + 400)
    b.set_launch(waves, rows)
    _, glog = b.step(300, counter0=0, log=True)
    assert compare_chain_logs(glog, olog, c1.beta) == 300


@pytest.mark.parametrize("cm", [[16, 16, 16], [21, 21, 21], [24, 24, 24]])
@pytest.mark.parametrize("waves,rows", [(4, 4), (8, 2), (8, 0), (4, 0), (16, 0), (8, -2)])
def test_chain_microcells_agree(c1, cm, waves, rows):
    """Microcells (k = 2, 3; pruned stencils of up to several hundred cells): the
    chain kernel gives the oracle's chain, and the cell list it leaves behind
    bins every particle where the oracle does."""
    p = _params(c1)
    opos, _, olog = oracle.chain(c1.pos, 300, p, seed=c1.seed, max_n=c1.n + 400, U0=0.0)
    req = np.array(cm, dtype=np.int32)
    b = _box(c1, max_n=c1.n + 400, cell_m=req)
    assert b.info()["n_stencil"] == oracle.stencil_count(c1.L, c1.rc, req)
    b.set_launch(waves, rows)      # rows = 0 on these stencils (125 to 335 cells): the microcell path
    _, glog = b.step(300, counter0=0, log=True)
    assert compare_chain_logs(glog, olog, c1.beta) == 300
    gpos = b.particles()[0]
    assert np.array_equal(gpos, opos)
    cell_of, _, _ = b.cells()
    assert np.array_equal(cell_of.astype(np.int64), oracle.cell_of(gpos, c1.L, c1.rc, req))


@pytest.mark.parametrize("cm", [[16, 16, 16], [24, 24, 24]])
def test_speculative_microcells_long_chain(c1, cm):
    """The speculative kernel's microcell path over 3,000 moves of the small box
    (r_c/2 and r_c/3 cells): every decision, the final configuration, the cell
    list, and the work counters of the per-move kernel on the same chain."""
    p = _params(c1)
    req = np.array(cm, dtype=np.int32)
    b = _box(c1, max_n=c1.n + 3001, cell_m=req)
    b.set_launch(8, 0)
    b.total_energy()
    r = chain_parity(b, oracle, c1.pos, p, c1.seed, 3000, c1.beta, c1.n + 3001, "speculative microcells")
    assert np.array_equal(b.particles()[0], r["opos"])
    cell_of, _, _ = b.cells()
    assert np.array_equal(cell_of.astype(np.int64), oracle.cell_of(r["opos"], c1.L, c1.rc, req))
    if not r["ties"]:
        ref = _box(c1, max_n=c1.n + 3001, cell_m=req)
        ref.set_launch(4, 4)
        rs, _ = ref.step(3000, counter0=0)
        for f in WORK:
            assert int(r["stats"][f]) == int(rs[f]), f


def test_speculative_microcells_dense_many_candidates():
    """A dense box on a small-cell grid with a large capacity, so that a move's
    candidates exceed one LDS window of record indices (2,048) and the window
    loop runs more than once."""
    wb = workloads.random_box(2500, 14.0, rc=4.0, T=1.2, mu=2.0, seed=78)
    req = np.array([5, 5, 5], dtype=np.int32)      # cells of 2.8 < rc: k = 2 covers every axis, 125 cells
    p = _params(wb)
    b = _box(wb, max_n=wb.n + 2001, cell_m=req, cell_cap=96)
    assert b.info()["n_stencil"] > 32
    b.set_launch(8, 0)
    r = chain_parity(b, oracle, wb.pos, p, wb.seed, 2000, wb.beta, wb.n + 2001, "dense microcells")
    assert np.array_equal(b.particles()[0], r["opos"])
    # every stencil is the whole box (N - 1 candidates): above one window
    assert int(r["stats"]["candidates"]) / max(1, int(r["stats"]["stencils"])) > 2048


@pytest.mark.parametrize("cm", [[21, 21, 21], [24, 24, 24]])
def test_total_energy_virial_backward_microcells(c1, cm):
    """Cell-list total energy, virial and forces over a pruned microcell stencil."""
    p = _params(c1)
    req = np.array(cm, dtype=np.int32)
    b = _box(c1, cell_m=req)
    ref = oracle.total_energy(c1.pos, p, per_particle=True)
    got = b.total_energy(per_particle=True)
    assert abs(got["U_pair"] - ref["U_pair"]) <= 1e-10 * ref["sumabs"]
    assert np.allclose(got["e"], ref["e"], rtol=0, atol=1e-10 * max(1.0, np.abs(ref["e"]).max()))
    vref = oracle.virial(c1.pos, p)
    v = b.virial()
    assert abs(v["W"] - vref["W"]) <= 1e-10 * vref["sumabs"]
    g = b.backward()["grad"]
    for i in range(0, c1.n, 97):
        gr = oracle.particle_gradient(c1.pos, i, p)
        assert np.allclose(g[i], gr, rtol=1e-7, atol=1e-9 * max(1.0, np.abs(gr).max()))


def test_delta_energy_mixture():
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    wb = workloads.random_box(500, 13.0, rc=3.0, seed=5, species_counts=[250, 250], eps=eps, sigma=sig)
    p = _params(wb)
    b = _box(wb, max_n=wb.n + 10)
    rng = np.random.default_rng(3)
    moves = _random_moves(wb, rng, 300, wb.n)
    moves["species"] = rng.integers(0, 2, len(moves))
    gp, gt = b.delta_energy(moves)
    rp, rt, sa = _oracle_deltas(wb, p, moves)
    assert_du(gp, rp, sa, "mixture")
    assert np.allclose(gt, rt, rtol=1e-12)


def test_delta_energy_edge_cases():
    """Overlap (r = 0) gives +inf, out-of-range indices give NaN, an empty box gives 0."""
    from paper_1408_3764_amd.box import Box, make_moves
    wb = workloads.random_box(50, 8.0, seed=3)
    b = _box(wb, max_n=60)
    mv = make_moves([1, 0, 2, 2, 1], [0, 3, -1, 50, 0], [wb.pos[5], wb.pos[3], wb.pos[0], wb.pos[0], [0.0, 0.0, 0.0]])
    gp, gt = b.delta_energy(mv)
    assert gp[0] == math.inf
    assert gp[1] == 0.0 or abs(gp[1]) < 1e-12          # displacement onto itself
    assert math.isnan(gp[2]) and math.isnan(gp[3])
    e = Box(np.zeros((0, 3)), [8.0] * 3, 2.5, max_n=10)
    gp, gt = e.delta_energy(make_moves([1], [0], [[1.0, 2.0, 3.0]]))
    assert gp[0] == 0.0 and gt[0] == pytest.approx(oracle.tail_delta([0], 0, +1, oracle.make_params([8.0] * 3, 2.5)))


# ----------------------------------------------------------- total energy
@pytest.mark.parametrize("case", list(SMALL_CASES))
def test_total_energy_parity(case):
    c = SMALL_CASES[case]
    wb = workloads.random_box(c["n"], c["L"], seed=c["seed"])
    p = _params(wb)
    ref = oracle.total_energy(wb.pos, p, per_particle=True)
    b = _box(wb)
    for ap in (False, True):
        got = b.total_energy(all_pairs=ap, per_particle=True)
        assert abs(got["U_pair"] - ref["U_pair"]) <= 1e-10 * ref["sumabs"]
        assert got["U_tail"] == pytest.approx(ref["U_tail"], rel=1e-13)
        assert np.allclose(got["e"], ref["e"], rtol=0, atol=1e-10 * max(1.0, np.abs(ref["e"]).max()))


@pytest.mark.parametrize("case", list(SMALL_CASES) + ["mixture"])
def test_virial_parity(case):
    """Pair virial and pressure against the oracle's all-pairs sums."""
    if case == "mixture":
        eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
        wb = workloads.random_box(400, 11.0, rc=3.0, seed=6, species_counts=[200, 200], eps=eps, sigma=sig)
        ref = oracle.virial(wb.pos, _params(wb), species=wb.species)
    else:
        c = SMALL_CASES[case]
        wb = workloads.random_box(c["n"], c["L"], seed=c["seed"])
        ref = oracle.virial(wb.pos, _params(wb))
    got = _box(wb).virial()
    V = float(np.prod(wb.L))
    assert abs(got["W"] - ref["W"]) <= 1e-10 * ref["sumabs"]
    assert abs(got["P"] - ref["P"]) <= 1e-10 * (abs(ref["P"]) + ref["sumabs"] / (3 * V))


@pytest.mark.parametrize("cm", [None, [16, 16, 16], [24, 24, 24]])
def test_total_energy_each_pair_once(c1, cm):
    """A total alone takes each pair once (the stencil offsets after (0, 0, 0)
    and larger ids in the home cell, also on pruned microcell stencils); with
    per-particle energies the full stencil runs.  Both equal the oracle's U
    within 1e-10 of the magnitude sum, and each other to the last few bits; the
    pair virial likewise."""
    p = _params(c1)
    ref = oracle.total_energy(c1.pos, p)
    kw = {} if cm is None else {"cell_m": np.array(cm, dtype=np.int32)}
    b = _box(c1, **kw)
    half = b.total_energy()
    full = b.total_energy(per_particle=True)
    for got in (half, full):
        assert abs(got["U_pair"] - ref["U_pair"]) <= 1e-10 * ref["sumabs"]
    assert half["U_pair"] == pytest.approx(full["U_pair"], rel=1e-12)
    assert half["U_pair"] == pytest.approx(0.5 * math.fsum(full["e"]), rel=1e-12)
    vref = oracle.virial(c1.pos, p)
    assert abs(b.virial()["W"] - vref["W"]) <= 1e-10 * vref["sumabs"]


def test_total_energy_c1(c1):
    p = _params(c1)
    ref = oracle.total_energy(c1.pos, p)
    b = _box(c1)
    for ap in (False, True):
        got = b.total_energy(all_pairs=ap)
        assert abs(got["U_pair"] - ref["U_pair"]) <= 1e-10 * ref["sumabs"]


# ------------------------------------------------------------------ chain
def _type_counts(olog):
    att = [int((olog["type"] == t).sum()) for t in range(3)]
    acc = [int(((olog["type"] == t) & (olog["accepted"] == 1)).sum()) for t in range(3)]
    return att, acc


def test_chain_parity_c1(c1):
    """1,000 moves of the small configuration: the GPU chain is the oracle's chain."""
    p = _params(c1)
    b = _box(c1, max_n=c1.n + 1001)
    b.total_energy()
    r = chain_parity(b, oracle, c1.pos, p, c1.seed, c1.n_moves, c1.beta, c1.n + 1001, "C1")
    stats, olog = r["stats"], r["olog"]
    assert int(stats["error"]) == 0
    gpos, _ = b.particles()
    assert np.array_equal(gpos, r["opos"])
    if not r["ties"]:
        att, acc = _type_counts(olog)
        assert int(stats["moves_done"]) == c1.n_moves
        assert list(stats["attempts"]) == att and list(stats["accepts"]) == acc
        assert stats["u_pair"] + stats["u_tail"] == pytest.approx(r["oU"], rel=1e-9)
        assert acc[0] > 0 and acc[1] > 0 and acc[2] > 0
    # the running energy is the recomputed one
    U = b.total_energy()
    assert U["U_pair"] == pytest.approx(stats["u_pair"], rel=1e-9)


WORK = ("stencils", "candidates", "pair_evals", "in_cutoff")


@pytest.mark.parametrize("width,rows", [(8, 0), (16, 0), (8, -1)])
def test_speculative_chain_parity_c1(c1, width, rows):
    """Speculative rounds (W moves evaluated at once, committed in order) give the
    sequential chain: 1,000 moves, same decisions and final configuration; their
    attempt and acceptance counts are the oracle's, and their work counters (the
    benchmark's algorithmic bytes come from them) equal the per-move kernel's."""
    p = _params(c1)
    b = _box(c1, max_n=c1.n + 1001)
    b.set_launch(width, rows)
    b.total_energy()
    r = chain_parity(b, oracle, c1.pos, p, c1.seed, c1.n_moves, c1.beta, c1.n + 1001, "speculative C1")
    stats = r["stats"]
    assert np.array_equal(b.particles()[0], r["opos"])
    cell_of, count, ids = b.cells()
    assert np.array_equal(cell_of.astype(np.int64), oracle.cell_of(r["opos"], c1.L, c1.rc))
    if not r["ties"]:
        assert stats["u_pair"] + stats["u_tail"] == pytest.approx(r["oU"], rel=1e-9)
        att, acc = _type_counts(r["olog"])
        assert list(stats["attempts"]) == att and list(stats["accepts"]) == acc
        ref = _box(c1, max_n=c1.n + 1001)
        ref.set_launch(4, 4)
        rs, _ = ref.step(c1.n_moves, counter0=0)
        for f in WORK:
            assert int(stats[f]) == int(rs[f]), f


def test_speculative_dense_conflicts():
    """A small dense box where most rounds end early (spatial conflicts, N changes)."""
    wb = workloads.random_box(300, 8.0, rc=2.5, T=1.2, mu=2.0, seed=77)
    p = _params(wb)
    ref = _box(wb, max_n=wb.n + 3001)
    ref.set_launch(4, 4)
    rs, _ = ref.step(3000, counter0=0)
    for width, rows in ((4, 0), (16, 0), (8, -1)):
        b = _box(wb, max_n=wb.n + 3001)
        b.set_launch(width, rows)
        r = chain_parity(b, oracle, wb.pos, p, wb.seed, 3000, wb.beta, wb.n + 3001, "dense speculative")
        if not r["ties"]:
            att, acc = _type_counts(r["olog"])
            assert list(r["stats"]["attempts"]) == att and list(r["stats"]["accepts"]) == acc
            for f in WORK:
                assert int(r["stats"][f]) == int(rs[f]), (width, rows, f)


def _oracle_running(olog, n0, U0, W0):
    """N, total energy and pair virial after every move of an oracle chain log."""
    a = olog["accepted"] == 1
    dn = np.where(a, np.where(olog["type"] == 1, 1, np.where(olog["type"] == 2, -1, 0)), 0)
    N = n0 + np.cumsum(dn)
    U = U0 + np.cumsum(np.where(a, olog["dU_pair"] + olog["dU_tail"], 0.0))
    W = W0 + np.cumsum(np.where(a, olog["dW_pair"], 0.0))
    return N.astype(np.float64), U, W


@pytest.mark.parametrize("shape", [(4, 4), (8, 0), (8, -1), "all_pairs"])
def test_chain_averages_match_oracle(c1, shape):
    """The averages the chain keeps on the GPU (Sec. 3.3.4: average energy and
    pressure): sums of N, N^2, U and W after every move, against the same sums
    over the oracle's log (W started from the oracle's total virial), and the
    average pressure built from them; the running W after the launch equals the
    virial recomputed from the final configuration.  Two launches: the box's
    cumulative sums (its checkpoint) hold both."""
    p = _params(c1)
    b = _box(c1, max_n=c1.n + 2001)
    if shape != "all_pairs":
        b.set_launch(*shape)
    ap = shape == "all_pairs"
    moves = 300 if ap else 1000
    b.total_energy()
    v0 = b.virial()
    t0 = oracle.total_energy(c1.pos, p)
    W0 = oracle.virial(c1.pos, p)["W"]
    assert v0["W"] == pytest.approx(W0, rel=1e-10)
    U0 = t0["U_pair"] + t0["U_tail"]
    opos, oU, oW, olog = oracle.chain(c1.pos, 2 * moves, p, seed=c1.seed, max_n=c1.n + 2001, U0=U0, W0=W0)
    N, U, W = _oracle_running(olog, c1.n, U0, W0)
    V = float(np.prod(c1.L))
    kp = oracle.tail_pressure([1], p)
    st1, _ = b.step(moves, counter0=0, all_pairs=ap)
    st2, _ = b.step(moves, counter0=moves, all_pairs=ap)
    for st, sl in ((st1, slice(0, moves)), (st2, slice(moves, 2 * moves))):
        assert int(st["moves_done"]) == moves
        assert st["sum_n"] == N[sl].sum()
        assert st["sum_n2"] == pytest.approx((N[sl] ** 2).sum(), rel=1e-13)
        assert st["sum_u"] == pytest.approx(U[sl].sum(), rel=1e-9)
        assert st["sum_w"] == pytest.approx(W[sl].sum(), rel=1e-9)
        assert st["avg_n"] == pytest.approx(N[sl].mean(), rel=1e-13)
        assert st["avg_u"] == pytest.approx(U[sl].mean(), rel=1e-9)
        P = N[sl] / (c1.beta * V) + W[sl] / (3 * V) + kp * N[sl] ** 2
        assert st["avg_p"] == pytest.approx(P.mean(), rel=1e-9)
    assert st2["w_pair"] == pytest.approx(oW, rel=1e-9)
    assert st2["w_pair"] == pytest.approx(oracle.virial(opos, p)["W"], rel=1e-9)
    _, _, ck = b.export_state()
    assert ck["moves"] == 2 * moves and ck["counter"] == 2 * moves
    assert ck["sum_n"] == N.sum() and ck["sum_w"] == pytest.approx(W.sum(), rel=1e-9)
    assert ck["attempts"] == _type_counts(olog)[0] and ck["accepts"] == _type_counts(olog)[1]


# the per-move kernel (the box's default launch), the speculative and pipelined kernels, the
# paper's cell-per-thread mapping and the box held in LDS
KERNELS = [None, (8, 0), (8, -1), (8, -2), (8, -3)]


def _launch(b, shape):
    if shape:
        b.set_launch(*shape)
    return b


@pytest.mark.parametrize("shape", KERNELS)
def test_chain_resume_split_equals_whole(c1, shape):
    """Counter-based draws: two calls of 400 + 600 moves = one call of 1,000."""
    a = _launch(_box(c1, max_n=c1.n + 1001), shape)
    a.step(1000, counter0=0)
    b = _launch(_box(c1, max_n=c1.n + 1001), shape)
    b.step(400, counter0=0)
    b.step(600, counter0=400)
    pa, _ = a.particles()
    pb, _ = b.particles()
    assert np.array_equal(pa, pb)


@pytest.mark.parametrize("shape", KERNELS)
def test_chain_deterministic(c1, shape):
    a = _launch(_box(c1, max_n=c1.n + 1001), shape)
    b = _launch(_box(c1, max_n=c1.n + 1001), shape)
    sa, la = a.step(1000, log=True)
    sb, lb = b.step(1000, log=True)
    assert la.tobytes() == lb.tobytes()
    assert np.array_equal(a.particles()[0], b.particles()[0])


def test_allpairs_chain_parity(c1):
    p = _params(c1)
    _, _, olog = oracle.chain(c1.pos, 300, p, seed=c1.seed, max_n=c1.n + 301)
    b = _box(c1, max_n=c1.n + 301)
    stats, glog = b.step(300, counter0=0, log=True, all_pairs=True)
    assert compare_chain_logs(glog, olog, c1.beta, "all-pairs chain") == 300
    assert int(stats["moves_done"]) == 300
    # the cell list was kept up to date by the all-pairs commits
    cell_of, _, _ = b.cells()
    pos, _ = b.particles()
    assert np.array_equal(cell_of.astype(np.int64), oracle.cell_of(pos, c1.L, c1.rc))


def test_allpairs_chain_many_workgroups_and_its_capacity_error():
    """The all-pairs chain over many workgroups (a box of 24,000 particles: 12
    chunks of 2,048), against the oracle move for move and with its cell list
    kept; then the capacity error: a chain that fills max_n stops there with
    GCMC_ERR_CAPACITY."""
    w = workloads.random_box(24_000, 34.0, rc=2.5, T=1.2, mu=-2.0, seed=12)
    p = _params(w)
    opos, _, olog = oracle.chain(w.pos, 400, p, seed=5, max_n=w.n + 401)
    b = _box(w, max_n=w.n + 401, seed=5)
    stats, glog = b.step(400, counter0=0, log=True, all_pairs=True)
    assert compare_chain_logs(glog, olog, w.beta, "all-pairs chain, 12 workgroups") == 400
    assert int(stats["moves_done"]) == 400 and int(stats["error"]) == 0
    pos, _ = b.particles()
    assert np.array_equal(pos, opos)
    cell_of, _, _ = b.cells()
    assert np.array_equal(cell_of.astype(np.int64), oracle.cell_of(pos, w.L, w.rc))
    from paper_1408_3764_amd.box import Box
    c = Box(np.zeros((0, 3)), [8.0] * 3, 2.5, mu=5.0, max_n=5, seed=1)
    st, _ = c.step(500, all_pairs=True)
    assert int(st["error"]) == 4 and int(st["n"]) == 5


def test_host_driven_commit_matches_chain():
    """gcmc_delta_energy + gcmc_commit, driven from the host with the oracle's decisions."""
    wb = workloads.random_box(200, 9.0, seed=12, T=1.2)
    p = _params(wb, beta=1 / 1.2, mu=-3.0)
    opos, _, olog = oracle.chain(wb.pos, 400, p, seed=44, max_n=700)
    from paper_1408_3764_amd.box import make_moves
    b = _box(wb, max_n=700)
    b.total_energy()
    b.virial()
    for rec in olog:
        if not rec["accepted"]:
            continue
        t = int(rec["type"])
        mv = make_moves([t], [rec["index"]], [[rec["x"], rec["y"], rec["z"]]])
        gp, _, gw = b.delta_energy(mv, virial=True)
        assert abs(gp[0] - rec["dU_pair"]) <= DU_REL * max(abs(rec["dU_pair"]), rec["sumabs"])
        assert abs(gw[0] - rec["dW_pair"]) <= DU_REL * max(abs(rec["dW_pair"]), rec["wsumabs"])
        b.commit(mv[0], gp[0], gw[0])
    gpos, _ = b.particles()
    assert np.array_equal(gpos, opos)
    # running energy and virial of the commits = the recomputed ones
    ck = b.checkpoint()
    assert ck["u_pair"] == pytest.approx(oracle.total_energy(opos, p)["U_pair"], rel=1e-9)
    assert ck["w_pair"] == pytest.approx(oracle.virial(opos, p)["W"], rel=1e-9)
    # a commit without its virial change leaves the running virial undefined (NaN)
    mv = make_moves([0], [0], [opos[0]])
    b.commit(mv[0], 0.0)
    assert math.isnan(b.checkpoint()["w_pair"])
    cell_of, _, _ = b.cells()
    assert np.array_equal(cell_of.astype(np.int64), oracle.cell_of(opos, wb.L, wb.rc))


@pytest.mark.parametrize("shape", KERNELS)
def test_ideal_gas_on_gpu(shape):
    """eps = 0: N is Poisson with mean V exp(beta mu)."""
    from paper_1408_3764_amd.box import Box
    L, beta, mu = 6.0, 1.0 / 1.3, -0.4
    mean = L ** 3 * math.exp(beta * mu)
    # an empty box sizes its cells for nothing: give the cells room for ~160 particles
    b = Box(np.zeros((0, 3)), [L] * 3, 2.5, beta=beta, mu=mu, eps=0.0, max_n=2000, seed=77, cell_cap=64)
    _launch(b, shape)
    st, _ = b.step(50_000, counter0=0)
    assert int(st["error"]) == 0
    ns = []
    for k in range(40):
        st, _ = b.step(10_000, counter0=50_000 + k * 10_000)
        assert int(st["error"]) == 0
        ns.append(st["sum_n"] / 10_000)
    ns = np.array(ns)
    se = ns.std(ddof=1) / math.sqrt(len(ns))
    assert abs(ns.mean() - mean) < 5 * se + 0.01 * mean, (ns.mean(), mean)


def _cell_sets(cells, n_cells):
    """Per cell the sorted particle ids (the cell list's content, slot order aside)."""
    count, ids = cells[1], cells[2]
    return [np.sort(ids[c, :count[c]]) for c in range(n_cells)]


def _oracle_cell_sets(pos, L, rc, n_cells):
    c = oracle.cell_of(pos, L, rc)
    order = np.argsort(c, kind="stable")
    out = [np.zeros(0, dtype=np.int64)] * n_cells
    for cell in np.unique(c):
        out[cell] = np.sort(order[c[order] == cell])
    return out


def _assert_cells_equal(got_sets, ref_sets):
    assert len(got_sets) == len(ref_sets)
    for c, (g, r) in enumerate(zip(got_sets, ref_sets)):
        assert np.array_equal(g.astype(np.int64), np.asarray(r, dtype=np.int64)), c


def test_speculative_matches_oracle_under_churn():
    """Ideal gas: every insertion and deletion changes N, and most are accepted.
    Every kernel's chain is the oracle's, move for move (index, decision), and
    leaves the oracle's particle array (order included) and cell contents after
    20,000 moves; the speculative kernels also leave the per-move kernel's slot
    order within cells."""
    from paper_1408_3764_amd.box import Box
    L = [6.0] * 3
    p = oracle.make_params(L, 2.5, eps=0.0, beta=1 / 1.3, mu=-0.4)
    opos, _, olog = oracle.chain(np.zeros((0, 3)), 20_000, p, seed=5, max_n=2000)
    out = []
    for shape in ((4, 4), (8, 0), (16, 0), (8, -1)):
        b = Box(np.zeros((0, 3)), L, 2.5, beta=1 / 1.3, mu=-0.4, eps=0.0, max_n=2000, seed=5, cell_cap=64)
        b.set_launch(*shape)
        st, log = b.step(20_000, counter0=0, log=True)
        assert int(st["error"]) == 0
        assert compare_chain_logs(log, olog, 1 / 1.3, "churn %s" % (shape,)) == 20_000
        pos = b.particles()[0]
        assert np.array_equal(pos, opos), shape
        cells = b.cells()
        nc = len(cells[1])
        _assert_cells_equal(_cell_sets(cells, nc), _oracle_cell_sets(opos, L, 2.5, nc))
        out.append(cells)
    count0, ids0 = out[0][1], out[0][2]
    valid = np.arange(ids0.shape[1])[None, :] < count0[:, None]
    for cells in out[1:]:
        assert np.array_equal(np.where(valid, cells[2], -1), np.where(valid, ids0, -1))


def test_speculative_deletion_relabel_invalidates():
    """A deletion moves particle N-1 into the freed index and rewrites its id in
    its cell.  That cell counts as modified: a later move of the same round that
    removes a particle from it (with the relabelled particle as the cell's last
    entry) must be evaluated again.  Ideal gas of about 400 particles in 125
    cells (27-cell stencils), many accepted deletions and insertions: the
    speculative kernels must leave the per-move kernel's particle array and
    cells exactly."""
    from paper_1408_3764_amd.box import Box
    L, beta = 12.5, 1.0
    mu = math.log(400.0 / L ** 3)
    rng = np.random.default_rng(9)
    start = rng.random((400, 3)) * L
    p = oracle.make_params([L] * 3, 2.5, eps=0.0, beta=beta, mu=mu)
    opos, _, olog = oracle.chain(start, 150_000, p, seed=21, max_n=4000)
    assert int(((olog["type"] == 2) & (olog["accepted"] == 1)).sum()) > 10_000
    out = []
    for shape in ((4, 4), (8, 0), (16, 0), (8, -1), (4, -1)):
        b = Box(start, [L] * 3, 2.5, beta=beta, mu=mu, eps=0.0, max_n=4000, seed=21, cell_cap=24)
        b.set_launch(*shape)
        st, _ = b.step(150_000, counter0=0)
        assert int(st["error"]) == 0
        pos = b.particles()[0]
        assert np.array_equal(pos, opos), shape
        cells = b.cells()
        nc = len(cells[1])
        _assert_cells_equal(_cell_sets(cells, nc), _oracle_cell_sets(opos, [L] * 3, 2.5, nc))
        out.append(cells)
    count0, ids0 = out[0][1], out[0][2]
    valid = np.arange(ids0.shape[1])[None, :] < count0[:, None]
    for cells in out[1:]:
        assert np.array_equal(np.where(valid, cells[2], -1), np.where(valid, ids0, -1))


# -------------------------------------------------------- error handling
@pytest.mark.parametrize("shape", KERNELS[:-1])
def test_overflow_latches_and_resumes(shape):
    """A cell over capacity stops the chain before the move; rebuilding with a
    larger capacity and resuming at the stop gives the uninterrupted chain."""
    M = 20_000
    # a sparse start (about 2 per cell) under a high chemical potential: cells fill up
    wb = workloads.random_box(1000, 20.0, rc=2.5, T=1.2, mu=10.0, seed=31)
    ref = _launch(_box(wb, max_n=wb.n + M + 1, cell_cap=64), shape)
    ref.step(M, counter0=0)
    assert ref.status() == 0
    maxc0 = int(_box(wb, max_n=wb.n + 1).cells()[1].max())
    assert int(ref.cells()[1].max()) > maxc0
    b2 = _launch(_box(wb, max_n=wb.n + M + 1, cell_cap=maxc0), shape)   # no headroom: the first growth overflows
    st, _ = b2.step(M, counter0=0)
    assert int(st["error"]) == 3
    stop = int(st["error_move"])
    assert 0 <= stop < M and int(st["moves_done"]) == stop
    assert b2.status() == 3
    n_at_stop = b2.n
    b2.cell_build(new_cap=64)
    assert b2.status() == 0 and b2.n == n_at_stop
    st2, _ = b2.step(M - stop, counter0=stop)
    assert int(st2["error"]) == 0
    assert np.array_equal(b2.particles()[0], ref.particles()[0])


def test_resident_overflow_latches_after_the_launch():
    """The box held in LDS keeps no cells during a launch: a cell over capacity
    shows when they are rebuilt at its end.  The chain itself is complete (every
    move done, the counter after the last); the error is latched, and a rebuild
    with a larger capacity restores the cells and lets the chain continue as the
    uninterrupted one."""
    M = 4000
    wb = workloads.random_box(1000, 20.0, rc=2.5, T=1.2, mu=10.0, seed=31)
    ref = _launch(_box(wb, max_n=wb.n + 2 * M + 1, cell_cap=64), (8, -3))
    ref.step(2 * M, counter0=0)
    assert ref.status() == 0
    maxc0 = int(_box(wb, max_n=wb.n + 1).cells()[1].max())
    b2 = _launch(_box(wb, max_n=wb.n + 2 * M + 1, cell_cap=maxc0), (8, -3))
    st, _ = b2.step(M, counter0=0)
    assert int(st["error"]) == 3
    assert int(st["error_move"]) == M and int(st["moves_done"]) == M
    assert b2.status() == 3
    n_after = b2.n
    b2.cell_build(new_cap=64)
    assert b2.status() == 0 and b2.n == n_after
    st2, _ = b2.step(M, counter0=M)
    assert int(st2["error"]) == 0
    assert np.array_equal(b2.particles()[0], ref.particles()[0])


@pytest.mark.parametrize("waves", [4, 8])
def test_resident_chain_cells_and_continuation(waves):
    """Dense small boxes whose stencil covers the whole box, held in LDS: the
    oracle's chain move for move, the cell list rebuilt at the launch's end in
    the layout of a fresh build (each particle in the cell of its position, a
    cell's entries in id order, back-pointers to their slots), and the chain
    continued by the speculative kernel on those cells is still the oracle's."""
    for k, (n, rho, T) in enumerate([(300, 0.7, 1.0), (640, 0.68, 1.03), (1400, 0.75, 1.0)]):
        w = workloads.cubic_box(n, rho, T, 2.5, 900 + k)
        p = _params(w)
        opos, oU, olog = oracle.chain(w.pos, 1500, p, seed=7, max_n=w.n + 1501)
        b = _launch(_box(w, max_n=w.n + 1501, seed=7), (waves, -3))
        st, glog = b.step(1500, counter0=0, log=True)
        assert compare_chain_logs(glog, olog, w.beta) == 1500, (n, rho)
        # work counters: every decided move read all other particles of its round's state (N
        # within the oracle's range over the chain), a displacement's two positions each
        dn = np.where(olog["accepted"] == 1, np.where(olog["type"] == 1, 1, np.where(olog["type"] == 2, -1, 0)), 0)
        traj = n + np.concatenate([[0], np.cumsum(dn)])
        c = int(st["candidates"])
        assert 1500 * (traj.min() - 1) <= c <= 1500 * traj.max(), (c, traj.min(), traj.max())
        n_disp = int((olog["type"] == 0).sum())
        assert int(st["pair_evals"]) <= c + n_disp * traj.max() and int(st["pair_evals"]) >= c
        assert 0 < int(st["in_cutoff"]) < int(st["pair_evals"])
        gpos, _ = b.particles()
        assert np.array_equal(gpos, opos), (n, rho)
        cell_of, count, ids = b.cells()
        want = oracle.cell_of(opos, w.L, 2.5)
        assert np.array_equal(cell_of[:len(opos)], want)
        for c in range(len(count)):
            members = np.sort(np.nonzero(want == c)[0])
            assert list(ids[c, :count[c]]) == list(members), c
        # continue on the rebuilt cells with the speculative kernel
        opos2, _, olog2 = oracle.chain(opos, 500, p, seed=7, counter0=1500, max_n=w.n + 1501, U0=oU)
        b.set_launch(8, 0)
        _, glog2 = b.step(500, counter0=1500, log=True)
        assert compare_chain_logs(glog2, olog2, w.beta) == 500, (n, rho)
        assert np.array_equal(b.particles()[0], opos2)


def test_resident_box_growing_past_lds():
    """A box that grows past the 2,048 particles held in LDS (the rest read and
    written in global memory) still follows the oracle's chain."""
    w = workloads.random_box(2030, 20.0, rc=2.5, T=1.2, mu=8.0, seed=41)
    p = _params(w)
    opos, _, olog = oracle.chain(w.pos, 1200, p, seed=7, max_n=w.n + 1201)
    assert len(opos) > 2100
    b = _launch(_box(w, max_n=w.n + 1201, seed=7), (8, -3))
    _, glog = b.step(1200, counter0=0, log=True)
    assert compare_chain_logs(glog, olog, w.beta) == 1200
    assert np.array_equal(b.particles()[0], opos)


@pytest.mark.parametrize("shape", KERNELS)
def test_capacity_error(shape):
    from paper_1408_3764_amd.box import Box
    b = _launch(Box(np.zeros((0, 3)), [8.0] * 3, 2.5, mu=5.0, max_n=5, seed=1), shape)
    st, _ = b.step(500)
    assert int(st["error"]) == 4 and int(st["n"]) == 5


@pytest.mark.parametrize("shape", [(8, 0), (8, -1)])
def test_wait_error_latches_and_resumes(c1, shape):
    """The speculative and pipelined chains wait on flags set by other wavefronts
    of the workgroup, each wait bounded.  A negative wait limit (set from the
    host) makes the first wait give up at once: the launch stops before the
    waiting move with GCMC_ERR_INTERNAL latched and every wavefront exits.  After
    a rebuild at the default limit, resuming at the stop gives the uninterrupted
    chain."""
    M = 3000
    ref = _launch(_box(c1, max_n=c1.n + M + 1), shape)
    ref.step(M, counter0=0)
    assert ref.status() == 0
    b = _launch(_box(c1, max_n=c1.n + M + 1), shape)
    b.set_wait_limit(-1)
    st, _ = b.step(M, counter0=0)
    assert int(st["error"]) == 8
    stop = int(st["error_move"])
    assert 0 <= stop < M and int(st["moves_done"]) == stop
    assert stop <= 1                      # the first wait comes at the first or second move
    assert b.status() == 8
    b.set_wait_limit(0)
    b.cell_build()
    assert b.status() == 0
    st2, _ = b.step(M - stop, counter0=stop)
    assert int(st2["error"]) == 0
    assert np.array_equal(b.particles()[0], ref.particles()[0])


def test_invalid_arguments():
    from paper_1408_3764_amd import _lib
    from paper_1408_3764_amd.box import Box
    with pytest.raises(_lib.GcmcError) as e:
        Box(np.zeros((0, 3)), [4.0] * 3, 2.5)                 # rc > L/2
    assert e.value.code == 1
    with pytest.raises(_lib.GcmcError):
        Box(np.array([[1.0, 2.0, 9.0]]), [8.0] * 3, 2.5)      # outside [0, L)
    with pytest.raises(_lib.GcmcError):
        Box(np.zeros((3, 3)), [8.0] * 3, 2.5, max_n=2)          # n > max_n
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    m = Box(np.array([[1.0, 1.0, 1.0]]), [8.0] * 3, 2.5, eps=eps, sigma=sig, species=[1], max_n=4)
    with pytest.raises(_lib.GcmcError) as e:
        m.step(10)                                              # the chain is single-species
    assert e.value.code == 7


@pytest.mark.parametrize("shape", KERNELS)
def test_checkpoint_roundtrip(c1, shape):
    """Export after 700 moves, import into a new box, continue both with the
    device counter: the same chain, running energy and virial, and cumulative
    statistics (the paper's periodic status dumps, Algorithm 1)."""
    from paper_1408_3764_amd._lib import COUNTER_CONTINUE
    a = _launch(_box(c1, max_n=c1.n + 2001), shape)
    a.total_energy()
    a.virial()
    a.step(700, counter0=0)
    pos, sp, ck = a.export_state()
    assert ck["counter"] == 700 and ck["moves"] == 700 and ck["n"] == len(pos)
    b = _launch(_box(c1, max_n=c1.n + 2001), shape)
    b.import_state(pos, ck, species=sp)
    assert b.checkpoint() == ck
    a.step(500, counter0=COUNTER_CONTINUE)
    b.step(500, counter0=COUNTER_CONTINUE)
    assert np.array_equal(a.particles()[0], b.particles()[0])
    ca, cb = a.checkpoint(), b.checkpoint()
    assert ca == cb
    b.clear_averages()
    cc = b.checkpoint()
    assert cc["moves"] == 0 and cc["sum_n"] == 0.0 and cc["counter"] == 1200 and cc["u_pair"] == cb["u_pair"]


def test_set_positions_checks_its_length(c1):
    from paper_1408_3764_amd import _lib
    b = _box(c1)
    with pytest.raises(ValueError):
        b.set_positions(c1.pos[:-1])
    x = torch.zeros(c1.n - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.GcmcError) as e:
        _lib.gcmc_set_positions(b.handle, x, x, x, c1.n - 1)
    assert e.value.code == 1
    # a valid call: the running energy and virial become NaN until recomputed
    b.total_energy()
    b.set_positions(c1.pos)
    ck = b.checkpoint()
    assert math.isnan(ck["u_pair"]) and math.isnan(ck["w_pair"])
    b.total_energy()
    assert not math.isnan(b.checkpoint()["u_pair"])


# --------------------------------------------------------------- gradients
@pytest.mark.parametrize("counts", [[200, 200], [150, 150, 100]])
def test_backward_parity_mixture(counts):
    """Forces and parameter derivatives of a binary and a ternary mixture (the
    pass keeps its per-particle parameter sums in LDS sized by the species
    count: two species, or up to four)."""
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2, 0.9][: len(counts)], [1.0, 0.8, 1.1][: len(counts)])
    wb = workloads.random_box(400, 12.0, rc=3.0, seed=8, species_counts=counts, eps=eps, sigma=sig)
    p = _params(wb)
    g_ref, de_ref, ds_ref = oracle.gradients(wb.pos, p, species=wb.species)
    b = _box(wb)
    got = b.backward()
    scale = np.abs(g_ref).max()
    assert np.allclose(got["grad"], g_ref, rtol=1e-7, atol=1e-7 * scale)
    assert np.allclose(got["d_eps"], de_ref, rtol=1e-7)
    assert np.allclose(got["d_sigma"], ds_ref, rtol=1e-7)


def test_backward_single_species(c1):
    p = _params(c1)
    b = _box(c1)
    got = b.backward()
    rng = np.random.default_rng(2)
    for i in rng.choice(c1.n, 40, replace=False):
        ref = oracle.particle_gradient(c1.pos, i, p)
        assert np.allclose(got["grad"][i], ref, rtol=1e-7, atol=1e-9 * max(1.0, np.abs(ref).max()))
    assert np.abs(got["grad"].sum(axis=0)).max() <= 1e-9 * np.abs(got["grad"]).sum()
    # U is linear in eps
    U = b.total_energy()
    assert got["d_eps"][0, 0] == pytest.approx(U["U_pair"] + U["U_tail"], rel=1e-10)


# ------------------------------------------------------------------ batch
MIXED = [(8, 0), (4, 4), (2, 0), (8, -1), (8, 0)]   # one shape per box: four launch groups
MIXED_LDS = [(8, -3), (4, -3), (8, 0), (2, 0), (8, -3)]


@pytest.mark.parametrize("shape", [(2, 8), (8, 0), (4, -1), (8, -3), "mixed", "mixed_lds"])
def test_batch_matches_single_boxes(shape):
    """Boxes of one batch (one launch per launch shape, the groups on forked
    streams) each follow their own oracle chain."""
    from paper_1408_3764_amd.box import Batch, Box
    sizes = [130, 400, 900, 260, 1500]
    wbs = [workloads.cubic_box(n, rho, T, 2.5, 500 + k) for k, (n, rho, T) in
           enumerate(zip(sizes, [0.3, 0.5, 0.8, 0.6, 0.4], [0.9, 1.2, 1.5, 1.0, 1.1]))]
    boxes = [Box.from_workload(w, max_n=w.n + 301, box_id=k, seed=99) for k, w in enumerate(wbs)]
    for k, b in enumerate(boxes):
        b.set_launch(*({"mixed": MIXED, "mixed_lds": MIXED_LDS}[shape][k] if isinstance(shape, str) else shape))
    bt = Batch(boxes)
    stats = bt.step(300, counter0=0)
    for k, w in enumerate(wbs):
        p = _params(w)
        opos, _, olog = oracle.chain(w.pos, 300, p, seed=99, box=k, max_n=w.n + 301)
        assert int(stats[k]["n"]) == len(opos)
        gpos, _ = boxes[k].particles()
        assert np.array_equal(gpos, opos), k
        assert list(stats[k]["accepts"]) == [int(((olog["type"] == t) & (olog["accepted"] == 1)).sum())
                                             for t in range(3)]


def test_batch_takes_new_launch_shapes(c1):
    """Changing the boxes' launch shapes between two steps of one batch, with the
    grouping of the boxes unchanged, launches the new shapes: under a wait bound
    that fails at once, the per-move kernel (which never waits) runs clean, and the
    speculative kernel that replaces it stops at its first wait with
    GCMC_ERR_INTERNAL."""
    from paper_1408_3764_amd.box import Batch
    boxes = [_box(c1, max_n=c1.n + 2001, box_id=k) for k in range(3)]
    for b in boxes:
        b.set_launch(4, 4)
        b.set_wait_limit(-1)
    bt = Batch(boxes)
    st = bt.step(200, counter0=0)
    assert np.all(st["error"] == 0)
    for b in boxes:
        b.set_launch(8, 0)
    st = bt.step(200, counter0=200)
    assert np.any(st["error"] == 8), st["error"]
    bt.close()


# ------------------------------------------------------------------ tuner
def test_autotune_cells_picks_a_timed_configuration_and_keeps_the_chain(c1):
    """The cell-size and launch-shape tuner: it times the paper's cells and
    twice as many per axis, keeps the fastest (box, shape) it timed, offers the
    speculative shapes on both grids (the microcells' 125-cell stencils take its
    microcell path) but the pipelined shapes only where the stencil has at most
    32 cells, and the box it returns is back in its starting state: its next
    moves (device counter) are the oracle's first moves."""
    from paper_1408_3764_amd import tune
    from paper_1408_3764_amd.box import Box
    from paper_1408_3764_amd._lib import COUNTER_CONTINUE
    made = []

    def mk(cm):
        made.append(cm)
        return Box.from_workload(c1, max_n=c1.n + 20_000, cell_m=cm)

    box, cm, shape, t = tune.autotune_cells(mk, factors=(1, 2), n_moves=200)
    assert made == [None, [16, 16, 16]]
    grid = box.info()["cell_m"]
    assert grid == ([8, 8, 8] if cm is None else cm)
    assert shape in tune.SHAPES + tune.SPEC_SHAPES + tune.ASYNC_SHAPES
    assert min(t, key=t.get) == "%s/%dx%d" % ("x".join(map(str, grid)), shape[0], shape[1])
    assert any(k.startswith("8x8x8/") and k.endswith("x0") for k in t)
    assert any(k.startswith("8x8x8/") and k.endswith("x-1") for k in t)
    assert any(k.startswith("16x16x16/") and k.endswith("x0") for k in t)
    assert not any(k.startswith("16x16x16/") and k.endswith("x-1") for k in t)
    p = _params(c1)
    _, _, olog = oracle.chain(c1.pos, 100, p, seed=c1.seed, max_n=c1.n + 20_000, U0=0.0)
    assert box.checkpoint()["counter"] == 0
    _, glog = box.step(100, counter0=COUNTER_CONTINUE, log=True)
    assert compare_chain_logs(glog, olog, c1.beta) == 100
