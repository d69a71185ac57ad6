"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each uses a closed form, an
exact rational computation, a quadrature, an independent brute-force definition,
an invariant, a statistical law, or a number the paper prints.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1408_3764_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# --------------------------------------------------------------------------
# Philox4x32-10 (the seeded generator shared by both sides)
# --------------------------------------------------------------------------
def test_philox_known_answers(orc):
    path = os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(v, 16) for v in r]
        out = orc.philox4x32_10(w[0:4], w[4:6])
        assert [int(v) for v in out] == w[6:10]


def test_u01_bounds(orc):
    # 27 + 26 bits -> multiples of 2^-53 in [0, 1)
    assert orc.u01(0, 0) == 0.0
    assert orc.u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert orc.u01(1 << 5, 0) == 2.0 ** -27
    assert orc.u01(0, 1 << 6) == 2.0 ** -53


def test_move_draw_layout(orc):
    # counter (move lo, move hi, box, j), key (seed lo, seed hi), doubles from words (0,1),(2,3)
    seed, move, box = 0x0123456789ABCDEF, (7 << 32) | 5, 3
    u = orc.move_draws(seed, move, box)
    for j in range(4):
        w = orc.philox4x32_10([5, 7, box, j], [seed & 0xFFFFFFFF, seed >> 32])
        assert u[2 * j] == orc.u01(w[0], w[1])
        assert u[2 * j + 1] == orc.u01(w[2], w[3])


# --------------------------------------------------------------------------
# Eq. (1): the Lennard-Jones pair energy, truncated at rc
# --------------------------------------------------------------------------
def _lj_exact(r, eps=1, sig=1):
    q = Fraction(sig) / Fraction(r)
    return 4 * Fraction(eps) * (q ** 12 - q ** 6)


def test_lj_closed_forms(orc):
    assert orc.lj_r2(1.0, 1.0, 1.0, 2.5) == 0.0                       # u(sigma) = 0
    rmin2 = 2.0 ** (1.0 / 3.0)                                         # r_min^2 = 2^(1/3)
    assert orc.lj_r2(rmin2, 1.0, 1.0, 2.5) == pytest.approx(-1.0, rel=1e-15, abs=1e-15)
    for r in (0.9, 1.5, 2.0, 2.4999):
        assert orc.lj_r2(r * r, 1.0, 1.0, 2.5) == pytest.approx(float(_lj_exact(Fraction(r))), rel=1e-14)
    assert orc.lj_r2(1.5 ** 2, 1.0, 1.0, 2.5) == pytest.approx(-0.320336594278575, rel=1e-14)
    # scaling: u_{eps,sig}(r) = eps * u_{1,1}(r/sig)
    for eps, sig, r in ((0.8, 1.2, 1.7), (2.0, 0.9, 1.1)):
        assert orc.lj_r2(r * r, eps, sig, 10.0) == pytest.approx(
            eps * float(_lj_exact(Fraction(r) / Fraction(sig))), rel=1e-13)


def test_lj_cutoff_strict(orc):
    rc = 2.5
    assert orc.lj_r2(rc * rc, 1.0, 1.0, rc) == 0.0                    # r == rc is outside
    below = np.nextafter(rc * rc, 0.0)
    assert orc.lj_r2(below, 1.0, 1.0, rc) < 0.0                        # just inside counts
    assert orc.lj_r2(9.0, 1.0, 1.0, 2.5) == 0.0
    assert orc.lj_r2(0.0, 1.0, 1.0, 2.5) == math.inf                   # overlap: +inf, rejected later
    assert orc.lj_r2(0.0, 0.0, 1.0, 2.5) == 0.0                        # ideal gas never interacts


# --------------------------------------------------------------------------
# Minimum image: independent definition = min over all 27 periodic images
# --------------------------------------------------------------------------
def _bruteforce_energy(pos, L, rc, eps=1.0, sig=1.0):
    """Pure-Python all-pairs energy, distance = minimum over the 27 image shifts."""
    n = len(pos)
    shifts = np.array([[a, b, c] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)], dtype=float)
    U = Fraction(0)
    for i in range(n):
        for j in range(i + 1, n):
            d = pos[j] - pos[i] + shifts * L
            r2 = float(np.min((d * d).sum(axis=1)))
            if r2 < rc * rc:
                U += _lj_exact(Fraction(math.sqrt(r2)), eps, sig)
    return float(U)


def test_two_particle_across_boundary(orc):
    L = np.array([10.0, 11.0, 12.0])
    p = orc.make_params(L, 2.5)
    for pos in (np.array([[0.25, 5.0, 6.0], [8.75, 5.0, 6.0]]),          # r = 1.5 through x = 0
                np.array([[0.2, 0.3, 0.4], [9.3, 10.5, 11.6]])):        # diagonal through a corner
        d = pos[1] - pos[0]
        d -= L * np.round(d / L)
        r = float(np.sqrt((d * d).sum()))
        U = orc.total_energy(pos, p)["U_pair"]
        assert U == pytest.approx(float(_lj_exact(Fraction(r))), rel=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_allpairs_equals_image_bruteforce(orc, seed):
    b = workloads.random_box(24, [5.6, 6.1, 7.3], seed=seed)
    p = orc.make_params(b.L, 2.5)
    U = orc.total_energy(b.pos, p)["U_pair"]
    assert U == pytest.approx(_bruteforce_energy(b.pos, b.L, 2.5), rel=1e-12, abs=1e-12)


# --------------------------------------------------------------------------
# Tail correction: closed form vs quadrature of the definition
# --------------------------------------------------------------------------
def test_tail_closed_form_vs_quadrature(orc):
    from scipy.integrate import quad
    for rc in (2.5, 3.0):
        L = np.array([13.0, 14.0, 15.0])
        V = float((L[0] * L[1]) * L[2])
        p = orc.make_params(L, rc)
        N = 1234
        integ, _ = quad(lambda r: r * r * 4.0 * (r ** -12 - r ** -6), rc, np.inf, epsabs=0, epsrel=1e-13)
        ref = 2.0 * math.pi * N * N / V * integ
        assert orc.tail_energy([N], p) == pytest.approx(ref, rel=1e-11)
    # per-N^2/V constants for unit LJ
    p = orc.make_params([1.0, 1.0, 1.0], 2.5)
    assert orc.tail_energy([1], p) == pytest.approx(-0.535433102066, rel=1e-11)
    p = orc.make_params([1.0, 1.0, 1.0], 3.0)
    assert orc.tail_energy([1], p) == pytest.approx(-0.310138880850, rel=1e-11)


def test_tail_mixture_vs_quadrature(orc):
    from scipy.integrate import quad
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    L = np.array([20.0, 21.0, 22.0])
    V = float((L[0] * L[1]) * L[2])
    rc = 3.0
    p = orc.make_params(L, rc, eps=eps, sigma=sig)
    counts = [700, 300]
    ref = 0.0
    for a in range(2):
        for b in range(2):
            f = lambda r, e=eps[a, b], s=sig[a, b]: r * r * 4.0 * e * ((s / r) ** 12 - (s / r) ** 6)
            integ, _ = quad(f, rc, np.inf, epsabs=0, epsrel=1e-13)
            ref += 2.0 * math.pi / V * counts[a] * counts[b] * integ
    assert orc.tail_energy(counts, p) == pytest.approx(ref, rel=1e-11)


def test_tail_delta_exact_differences(orc):
    """The algebraic insertion/deletion delta equals U(N +- e_s) - U(N)."""
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    for ns in (1, 2):
        p = orc.make_params([30.0, 31.0, 32.0], 3.0, eps=eps[:ns, :ns], sigma=sig[:ns, :ns])
        base = [262144, 1000][:ns]
        for sp in range(ns):
            for sign in (+1, -1):
                after = list(base)
                after[sp] += sign
                ref = orc.tail_energy(after, p) - orc.tail_energy(base, p)
                got = orc.tail_delta(base, sp, sign, p)
                assert abs(got - ref) <= 1e-12 * abs(orc.tail_energy(base, p))
                if ns == 1:
                    # exact rational: U_tail is k N^2, so the delta is k ((N +- 1)^2 - N^2)
                    k1 = Fraction(orc.tail_energy([1], p))
                    exact = k1 * (Fraction(base[0] + sign) ** 2 - Fraction(base[0]) ** 2)
                    assert got == pytest.approx(float(exact), rel=1e-14)


# --------------------------------------------------------------------------
# Invariants of the total energy
# --------------------------------------------------------------------------
def test_half_sum_identity(orc):
    b = workloads.random_box(300, 9.0, seed=11)
    p = orc.make_params(b.L, 2.5)
    r = orc.total_energy(b.pos, p, per_particle=True)
    assert 0.5 * math.fsum(r["e"]) == pytest.approx(r["U_pair"], rel=1e-13)


def test_translation_invariance(orc):
    b = workloads.random_box(300, [9.0, 10.0, 11.0], seed=12)
    p = orc.make_params(b.L, 2.5)
    U0 = orc.total_energy(b.pos, p)["U_pair"]
    rng = np.random.default_rng(5)
    for _ in range(3):
        shift = rng.uniform(-20, 20, 3)
        q = np.mod(b.pos + shift, b.L)
        q = np.where(q >= b.L, 0.0, q)
        U = orc.total_energy(q, p)["U_pair"]
        assert U == pytest.approx(U0, rel=1e-12)
        # and the energy change of a fixed trial displacement is invariant too
        t = b.pos[7] + np.array([0.2, -0.1, 0.25])
        e0 = orc.position_energy(b.pos, p, np.mod(t, b.L), exclude=7)[0]
        e1 = orc.position_energy(q, p, np.mod(t + shift, b.L), exclude=7)[0]
        assert e1 == pytest.approx(e0, rel=1e-12, abs=1e-13)


# --------------------------------------------------------------------------
# Cell grid: the paper's worked numbers (Sec. 3.2.2, Sec. 3.3, Sec. 3.3.2)
# --------------------------------------------------------------------------
def test_cell_size_worked_example(orc, golden):
    g = golden["cell_size_example"]
    r = orc.grid([g["L"]] * 3, g["rc"])
    assert int(r["M"][0]) == g["T"]
    S = g["L"] / r["M"][0]
    assert round(S, g["S_print_digits"]) == g["S_printed"]
    assert S >= g["rc"]
    sm = golden["small_box_rule"]
    r = orc.grid([sm["L"]] * 3, sm["rc"])
    assert int(r["M"][0]) == sm["T"]
    assert int(r["span"][0]) == 3                                     # the whole axis is in the stencil


def test_cell_count_exact_box_length(orc):
    # L = cbrt(8000) = 20 exactly gives 8 cells of side 2.5; 8000**(1/3) would give 7
    assert int(orc.grid([np.cbrt(8000.0)] * 3, 2.5)["M"][0]) == 8
    assert int(orc.grid([8000.0 ** (1 / 3)] * 3, 2.5)["M"][0]) == 7


def test_stencil_volume_numbers(golden):
    g = golden["stencil_volume"]
    assert round(4.0 / 3.0 * math.pi * g["rc"] ** 3, 2) == g["sphere_volume"]
    assert 27 * g["S_a"] ** 3 > g["cells_volume_a"]
    assert 27 * g["S_b"] ** 3 == g["cells_volume_b"]
    assert (4.0 / 3.0 * math.pi * g["rc"] ** 3) / (27 * g["S_b"] ** 3) < g["max_useful_fraction"]


def test_microcell_offset_example(orc, golden):
    """sigma-sized cells with rc = 2.5: the stencil of cell (7,6,5) is the 7x7x7 cube (4,3,2)..(10,9,8)."""
    g = golden["microcell_offset_example"]
    L = 20.0
    req = np.array([20, 20, 20], dtype=np.int32)                       # unit cells
    r = orc.grid([L] * 3, 2.5, req)
    assert list(r["span"]) == [g["cube"]] * 3
    cells = np.array([[x + 0.5, y + 0.5, z + 0.5] for x in range(20) for y in range(20) for z in range(20)])
    ids = orc.neighbor_ids(cells, np.array(g["center"]) + 0.5, [L] * 3, 2.5, req_m=req)
    got = cells[ids] - 0.5
    lo, hi = np.array(g["first_cell"]), np.array(g["last_cell"])
    # The cube bounds the stencil; its cells with two offsets of 3 (two whole unit
    # cells of gap on each of two axes: 2^2 + 2^2 = 8 > 2.5^2) are dropped: 3 axis
    # pairs x 4 sign pairs x 5 offsets <= 2 on the third axis + 8 corners = 68.
    assert len(ids) == g["cube"] ** 3 - 68
    assert np.all(got.min(axis=0) == lo) and np.all(got.max(axis=0) == hi)
    assert orc.stencil_count([L] * 3, 2.5, req) == g["cube"] ** 3 - 68


@pytest.mark.parametrize("m,kept", [(8, 27), (16, 125), (20, 251), (24, 275)])
def test_pruned_stencil_counts(orc, m, kept):
    """Kept stencil cells counted by hand, cubic box L = 30, rc = 3.5 (rc^2 = 12.25).

    Along an axis the gap to a cell |d| cells away is (|d| - 1) S for |d| >= 2.
    m = 8:  S = 3.75 >= rc, k = 1: no gaps, all 27 kept.
    m = 16: S = 1.875, k = 2: at most three gaps of S, 3 S^2 = 10.55 <= 12.25: 125.
    m = 20: S = 1.5, k = 3: squared gaps 2.25 (|d| = 2), 9 (|d| = 3).  Dropped:
            two or three axes at |d| = 3 (>= 18): 3 axis pairs x 4 signs x 5 values
            of the third offset + 8 corners = 68; one axis at 3 and both others at
            2 (13.5): 3 x 2 x 4 = 24.  343 - 92 = 251.
    m = 24: S = 1.25, k = 3: squared gaps 1.5625, 6.25.  Only two axes at |d| = 3
            (>= 12.5) are dropped (3, 2, 2 gives 9.375): 343 - 68 = 275.
    """
    assert orc.stencil_count([30.0] * 3, 3.5, [m] * 3) == kept


def test_paper_box_volumes(golden):
    g = golden["table1_box_volumes"]
    assert round(g["n_small"] / g["rho"], g["print_decimals"]) == g["V_small"]
    # The printed 436905.6 is N/rho for rho = 0.6 only to 2.5e-6 relative (N/0.6 = 436906.7);
    # the workloads take V = N/rho exactly (a reading of an inconsistency in the paper).
    assert g["n_large"] / g["rho"] == pytest.approx(g["V_large"], rel=3e-6)


# --------------------------------------------------------------------------
# Cell list = all-pairs (brute force on tiny boxes, including points at faces)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,n,seed,req", [(7.4, 120, 1, None), (10.0, 300, 2, None), (12.7, 300, 3, None),
                                          ([7.6, 10.0, 12.7], 250, 4, None),
                                          (10.0, 300, 5, [12, 12, 12]),     # k = 3, pruned stencil
                                          (12.7, 300, 6, [13, 17, 21]),     # k = 2, 3, 5 per axis
                                          ([7.6, 10.0, 12.7], 250, 7, [3, 9, 16])])   # x whole, pruned y, z
def test_cell_list_covers_cutoff(orc, L, n, seed, req):
    b = workloads.random_box(n, L, seed=seed)
    pos = b.pos.copy()
    req = None if req is None else np.array(req, dtype=np.int32)
    g = orc.grid(b.L, 2.5, req)
    # push a few particles to within 1e-12 of cell faces
    rng = np.random.default_rng(seed)
    for i in range(0, n, 17):
        a = rng.integers(0, 3)
        f = rng.integers(0, g["M"][a]) * (b.L[a] / g["M"][a])
        pos[i, a] = min(max(f + rng.choice([-1e-12, 0.0, 1e-12]), 0.0), np.nextafter(b.L[a], 0))
    p = orc.make_params(b.L, 2.5)
    rc2 = 2.5 * 2.5
    for i in range(0, n, 5):
        ids = orc.neighbor_ids(pos, pos[i], b.L, 2.5, exclude=i, req_m=req)
        d = pos - pos[i]
        d -= b.L * np.round(d / b.L)
        r2 = (d * d).sum(axis=1)
        within = set(np.nonzero(r2 < rc2)[0]) - {i}
        missing = within - set(ids.tolist())
        for j in missing:   # only pairs at the cutoff to rounding accuracy may be missed
            assert abs(math.sqrt(r2[j]) - 2.5) <= 1e-12 * 2.5
        e_all = orc.position_energy(pos, p, pos[i], exclude=i)[0]
        e_cell = math.fsum(orc.lj_r2(orc.min_image(pos[j, 0] - pos[i, 0], b.L[0]) ** 2
                                     + orc.min_image(pos[j, 1] - pos[i, 1], b.L[1]) ** 2
                                     + orc.min_image(pos[j, 2] - pos[i, 2], b.L[2]) ** 2, 1.0, 1.0, 2.5)
                           for j in ids)
        assert e_cell == pytest.approx(e_all, rel=1e-13, abs=1e-13)


# --------------------------------------------------------------------------
# GCMC acceptance: ideal-gas limit (Poisson), displacement accepts all
# --------------------------------------------------------------------------
def test_ideal_gas_poisson(orc):
    """eps = 0: N is Poisson with mean V exp(beta mu) / Lambda^3.  Pins the sign of
    the insertion exponent and the prefactors of Eqs. (4)-(5)."""
    L = np.array([4.0, 4.0, 4.0])
    V = 64.0
    beta, mu = 1.0 / 1.3, -0.4
    mean = V * math.exp(beta * mu) / 1.0
    p = orc.make_params(L, 1.5, eps=0.0, beta=beta, mu=mu)
    pos = np.zeros((0, 3))
    n_moves = 400_000
    _, _, log = orc.chain(pos, n_moves, p, seed=99, max_n=400)
    d = np.where(log["accepted"] == 1, np.where(log["type"] == 1, 1, np.where(log["type"] == 2, -1, 0)), 0)
    n_t = np.cumsum(d)[50_000:]
    nb = 50
    means = np.array([c.mean() for c in np.array_split(n_t, nb)])
    se = means.std(ddof=1) / math.sqrt(nb)
    assert abs(n_t.mean() - mean) < 5 * se + 0.01 * mean, (n_t.mean(), mean, se)
    assert n_t.var() == pytest.approx(mean, rel=0.1)
    # the flipped reading exp(-beta(mu - dU)) would give V exp(-beta mu): far away
    assert abs(V * math.exp(-beta * mu) - n_t.mean()) > 20 * se


def test_ideal_gas_displacements_all_accepted(orc):
    b = workloads.random_box(50, 6.0, seed=3)
    p = orc.make_params(b.L, 2.5, eps=0.0, p_disp=1.0)
    _, _, log = orc.chain(b.pos, 2000, p, seed=7)
    assert np.all(log["type"] == 0) and np.all(log["accepted"] == 1)


# --------------------------------------------------------------------------
# Algorithm 2 (a random particle, moved within a cube around it) and
# Algorithm 1's move draws: the displacement proposal and the particle pick,
# pinned by their distributions (uniform cube of half-width max_disp, each
# axis its own draw, wrapped into [0, L); index uniform over 0 .. N-1, from
# the bit fields of the spare draw with floor(u N) as the fallback).
# --------------------------------------------------------------------------
def _displacement_law_ok(d, half, n_sigma=5.0):
    """d: (m, 3) minimum-image displacements.  Uniform on [-half, half)^3 with
    independent axes: bounds, mean 0, variance half^2/3, Kolmogorov-Smirnov,
    no correlation between axes.  Returns the list of failed checks."""
    from scipy import stats
    m = len(d)
    bad = []
    if not (np.all(d >= -half) and np.all(d < half)):
        bad.append("bounds")
    for a in range(3):
        x = d[:, a]
        if abs(x.mean()) > n_sigma * half / math.sqrt(3 * m):
            bad.append("mean%d" % a)
        # variance of a uniform on [-h, h): h^2/3; sd of the sample variance: h^2 sqrt(4/45 / m)
        if abs(x.var() - half * half / 3) > n_sigma * half * half * math.sqrt(4.0 / 45.0 / m):
            bad.append("var%d" % a)
        if stats.kstest(x, stats.uniform(loc=-half, scale=2 * half).cdf).pvalue < 1e-6:
            bad.append("ks%d" % a)
    for a, b in ((0, 1), (0, 2), (1, 2)):
        if abs(np.corrcoef(d[:, a], d[:, b])[0, 1]) > n_sigma / math.sqrt(m):
            bad.append("corr%d%d" % (a, b))
    return bad


def _pick_law_ok(idx, n):
    """idx: picks from N = n particles.  Uniform over 0 .. n-1 by chi-square,
    and the last index drawn about as often as the others."""
    from scipy import stats
    bad = []
    if idx.min() < 0 or idx.max() > n - 1:
        bad.append("range")
    cnt = np.bincount(idx, minlength=n)[:n]
    if stats.chisquare(cnt).pvalue < 1e-6:
        bad.append("chi2")
    e = len(idx) / n
    if abs(cnt[n - 1] - e) > 6 * math.sqrt(e):
        bad.append("last")
    return bad


def _displacement_chain(orc, n=37, L=7.0, moves=30_000, half=0.3, seed=17):
    """Ideal gas (eps = 0), displacements only: every move is accepted, so the
    chain's positions follow from the log alone."""
    b = workloads.random_box(n, L, seed=4)
    p = orc.make_params(b.L, 2.5, eps=0.0, p_disp=1.0, max_disp=half)
    fin, _, log = orc.chain(b.pos, moves, p, seed=seed)
    assert np.all(log["type"] == 0) and np.all(log["accepted"] == 1)
    pos = b.pos.copy()
    d = np.zeros((moves, 3))
    for m in range(moves):
        i = int(log["index"][m])
        new = np.array([log["x"][m], log["y"][m], log["z"][m]])
        dd = new - pos[i]
        d[m] = dd - b.L * np.round(dd / b.L)   # minimum image: |d| <= half << L/2
        pos[i] = new
    assert np.array_equal(pos, fin)
    return b, p, log, d


def test_displacement_proposal_is_a_uniform_cube(orc):
    b, p, log, d = _displacement_chain(orc)
    assert _displacement_law_ok(d, 0.3) == []
    # every trial coordinate lies in [0, L)
    for a, k in enumerate("xyz"):
        assert np.all(log[k] >= 0.0) and np.all(log[k] < b.L[a])


def test_displacement_wraps_across_the_boundary(orc):
    """Particles next to a face: displacements that cross it re-enter at the
    opposite face (trial coordinates stay in [0, L) and the minimum-image step
    is still the uniform cube)."""
    L = np.array([5.0, 5.0, 5.0])
    pos = np.array([[0.05, 4.98, 2.5], [4.99, 0.01, 0.1], [0.1, 0.1, 4.95]])
    p = orc.make_params(L, 2.4, eps=0.0, p_disp=1.0, max_disp=0.3)
    _, _, log = orc.chain(pos, 20_000, p, seed=23)
    cur = pos.copy()
    d = np.zeros((len(log), 3))
    crossed = 0
    for m in range(len(log)):
        i = int(log["index"][m])
        new = np.array([log["x"][m], log["y"][m], log["z"][m]])
        assert np.all(new >= 0.0) and np.all(new < L)
        raw = new - cur[i]
        crossed += int(np.any(np.abs(raw) > 2.5))
        d[m] = raw - L * np.round(raw / L)
        cur[i] = new
    assert crossed > 100
    assert _displacement_law_ok(d, 0.3) == []


def test_particle_pick_is_uniform_including_the_last(orc):
    _, _, log, _ = _displacement_chain(orc)
    assert _pick_law_ok(log["index"].astype(np.int64), 37) == []


def test_pick_uniform_while_n_changes(orc):
    """Displacements and deletions of a grand-canonical ideal gas pick from the
    N of the moment: (index + w) / N with w ~ U[0, 1) is then exactly uniform."""
    from scipy import stats
    p = orc.make_params([6.0] * 3, 2.5, eps=0.0, beta=1.0, mu=-0.5)
    _, _, log = orc.chain(np.zeros((0, 3)), 120_000, p, seed=31, max_n=1000)
    d = np.where(log["accepted"] == 1, np.where(log["type"] == 1, 1, np.where(log["type"] == 2, -1, 0)), 0)
    n_before = np.concatenate([[0], np.cumsum(d)[:-1]])
    sel = (log["type"] != 1) & ((log["flags"] & 1) == 0)
    idx, nb = log["index"][sel].astype(np.float64), n_before[sel].astype(np.float64)
    assert np.all(idx >= 0) and np.all(idx < nb)
    w = np.random.default_rng(5).random(len(idx))
    assert stats.kstest((idx + w) / nb, "uniform").pvalue > 1e-6
    # the last particle is picked 1/N of the time
    assert abs(np.mean(idx == nb - 1) - np.mean(1.0 / nb)) < 6 * math.sqrt(np.mean(1.0 / nb) / len(idx))


def _pick_draws(orc, moves, seed=41):
    """(u_pick, u_spare) of the first `moves` moves of a stream: u[2] and u[7]."""
    u = np.array([orc.move_draws(seed, m) for m in range(moves)])
    return u[:, 2], u[:, 7]


def _pick_binned_ok(idx, n, bins=64):
    """Picks among n > 64 particles: 64 equal index ranges hit uniformly
    (chi-square on counts with the ranges' exact sizes) and (idx + w) / n with
    w ~ U[0, 1) uniform (Kolmogorov-Smirnov)."""
    from scipy import stats
    bad = []
    if idx.min() < 0 or idx.max() > n - 1:
        bad.append("range")
    edges = (np.arange(bins + 1) * n) // bins
    cnt = np.histogram(idx, bins=edges)[0]
    exp = len(idx) * np.diff(edges) / n
    if stats.chisquare(cnt, exp).pvalue < 1e-6:
        bad.append("chi2")
    w = np.random.default_rng(9).random(len(idx))
    if stats.kstest((idx + w) / n, "uniform").pvalue < 1e-6:
        bad.append("ks")
    return bad


def test_pick_uniform_at_every_field_width(orc):
    """The pick is uniform over 0 .. n-1 where the b-bit fields of the spare
    draw almost always hit (n = 2^b), where about half of each field's values
    miss (n = 2^(b-1) + 1), where several fields fit in 53 bits and where only
    one does (b >= 27: the floor(u n) branch then decides half the picks)."""
    u2, u7 = _pick_draws(orc, 60_000)
    pick = np.vectorize(orc.pick, otypes=[np.int64])
    assert np.all(pick(u2[:50], u7[:50], 1) == 0)
    for n in (2, 3, 5, 17, 33, 37, 63, 64, 65):
        assert _pick_law_ok(pick(u2, u7, n), n) == [], n
    for n in (1000, 4097, 1_500_000, (1 << 26) + 1, (1 << 27) + 5, 3 << 25, (1 << 31) - 1):
        assert _pick_binned_ok(pick(u2, u7, n), n) == [], n


def test_pick_rarely_changes_with_n(orc):
    """What the pick is for: one pair of draws names the same particle at
    neighbouring N (a move evaluated before an earlier insertion or deletion
    is decided keeps its particle), unlike floor(u N), which differs about
    half the time.  (Where n and the neighbouring N straddle a power of two
    the field width changes and the picks differ.)"""
    u2, u7 = _pick_draws(orc, 4000)
    pick = np.vectorize(orc.pick, otypes=[np.int64])
    assert np.mean(pick(u2, u7, 1 << 18) == pick(u2, u7, (1 << 18) + 1)) < 0.1
    for n in (300, 4000, 262_000, 1_500_000):
        a, b, c = pick(u2, u7, n), pick(u2, u7, n + 1), pick(u2, u7, n - 3)
        assert np.mean(a == b) > 0.9 and np.mean(a == c) > 0.8, n
        f0, f1 = np.floor(u2 * n), np.floor(u2 * (n + 1))
        assert np.mean(f0 == f1) < 0.6


def test_pick_checks_have_power(orc):
    """The uniformity checks reject misreadings of the pick built from the same
    draws: fields one bit too narrow (2^b < n: the top indices come only from
    the fallback) and a field kept when it equals n."""
    u2, u7 = _pick_draws(orc, 60_000)
    k = (u7 * 2.0 ** 53).astype(np.uint64)

    def variant(n, narrow=False, le=False):
        b = max(0, int(math.ceil(math.log2(n))) - (1 if narrow else 0))
        out = np.full(len(k), -1, dtype=np.int64)
        for t in range(1, (53 // b if b else 1) + 1):
            v = ((k >> np.uint64(53 - b * t)) & np.uint64((1 << b) - 1)).astype(np.int64)
            hit = (out < 0) & ((v <= n) if le else (v < n))
            out[hit] = v[hit]
        fb = np.minimum(np.floor(u2 * n), n - 1).astype(np.int64)
        return np.where(out < 0, fb, out)

    assert _pick_law_ok(variant(37), 37) == []
    assert _pick_law_ok(variant(37, narrow=True), 37) != []
    assert _pick_law_ok(variant(37, le=True), 37) != []
    assert _pick_law_ok(variant(33, le=True), 33) != []
    for n in ((1 << 27) + 5, 3 << 25):
        assert _pick_binned_ok(variant(n), n) == []
    assert _pick_binned_ok(variant(3 << 25, narrow=True), 3 << 25) != []


def test_pick_and_displacement_checks_have_power(orc):
    """The checks above reject the plausible misreadings, built here from the
    same Philox draws: a one-sided step d u, one draw for all three axes, no
    wrap (a coordinate leaves [0, L)), and a pick of floor(u (N - 1))."""
    n, moves, half = 37, 30_000, 0.3
    u = np.array([orc.move_draws(17, m) for m in range(moves)])
    one_sided = half * u[:, 4:7]
    one_draw = np.repeat((half * (2 * u[:, 4] - 1))[:, None], 3, axis=1)
    assert _displacement_law_ok(one_sided, half) != []
    assert _displacement_law_ok(one_draw, half) != []
    assert _pick_law_ok(np.floor(u[:, 2] * (n - 1)).astype(np.int64), n) != []
    assert _pick_law_ok(np.minimum(np.floor(u[:, 2] * n), n - 1).astype(np.int64), n) == []
    x = np.full(moves, 0.1) + half * (2 * u[:, 4] - 1)   # unwrapped step from next to a face
    assert np.any(x < 0.0)


def test_chain_energy_bookkeeping(orc):
    """Running U (sum of accepted dU) equals the recomputed U_pair + U_tail after many moves."""
    b = workloads.random_box(200, 8.0, seed=21, T=1.2)
    p = orc.make_params(b.L, 2.5, beta=1.0 / 1.2, mu=-3.0)
    t0 = orc.total_energy(b.pos, p)
    U0 = t0["U_pair"] + t0["U_tail"]
    pos, U, log = orc.chain(b.pos, 3000, p, seed=5, U0=U0)
    t1 = orc.total_energy(pos, p)
    assert U == pytest.approx(t1["U_pair"] + t1["U_tail"], rel=1e-10, abs=1e-9)
    kinds = {int(t): int(log["accepted"][log["type"] == t].sum()) for t in (0, 1, 2)}
    assert kinds[0] > 0 and kinds[1] > 0 and kinds[2] > 0
    assert len(pos) == 200 + kinds[1] - kinds[2]


def test_chain_empty_box_rejects(orc):
    p = orc.make_params([6.0] * 3, 2.5, mu=-30.0)
    _, _, log = orc.chain(np.zeros((0, 3)), 300, p, seed=3)
    empty = (log["flags"] & 1) == 1
    assert np.all(log["type"][empty] != 1) and np.all(log["accepted"][empty] == 0)
    assert empty.any()


def test_acceptance_rule_forms(orc):
    """Eq. (3)-(5) with Lambda^3 = 1: ratio = min(1, B_F), V B_F'/(N+1), N B_F''/V."""
    p = orc.make_params([5.0, 6.0, 7.0], 2.5, beta=0.5, mu=-1.5, lambda3=2.0)
    V = 210.0
    assert math.exp(orc.accept_arg(0, 0.7, 10, p)) == pytest.approx(math.exp(-0.5 * 0.7), rel=1e-14)
    assert math.exp(orc.accept_arg(1, 0.7, 10, p)) == pytest.approx(
        V / (2.0 * 11) * math.exp(0.5 * (-1.5 - 0.7)), rel=1e-14)
    assert math.exp(orc.accept_arg(2, 0.7, 10, p)) == pytest.approx(
        2.0 * 10 / V * math.exp(-0.5 * (-1.5 + 0.7)), rel=1e-14)
    assert orc.accept(0.1, 0.0, 0.999) == 1
    assert orc.accept(-1.0, 1.0, math.exp(-1.0)) == 0                 # strict A < ratio
    assert orc.accept(-math.inf, math.inf, 0.0) == 0
    assert orc.accept(0.0, float("nan"), 0.0) == 0


# --------------------------------------------------------------------------
# Gradients: closed form, Newton's third law, homogeneity, virial, FD
# --------------------------------------------------------------------------
def test_two_particle_force_closed_form(orc):
    L = np.array([10.0, 10.0, 10.0])
    p = orc.make_params(L, 2.5)
    for r in (1.05, 1.3, 2.2):
        pos = np.array([[1.0, 2.0, 3.0], [1.0 + r, 2.0, 3.0]])
        g, _, _ = orc.gradients(pos, p)
        dudr = float(-24 * (2 * Fraction(r) ** -13 - Fraction(r) ** -7))   # d/dr 4(r^-12 - r^-6)
        assert g[1, 0] == pytest.approx(dudr, rel=1e-13)
        assert g[0, 0] == pytest.approx(-dudr, rel=1e-13)
        assert abs(g[0, 1]) < 1e-15 and abs(g[1, 2]) < 1e-15


def test_gradient_invariants(orc):
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    b = workloads.random_box(160, 9.0, seed=31, species_counts=[80, 80], eps=eps, sigma=sig)
    p = orc.make_params(b.L, 3.0, eps=eps, sigma=sig)
    g, de, ds = orc.gradients(b.pos, p, species=b.species)
    scale = np.abs(g).sum()
    assert np.all(np.abs(g.sum(axis=0)) <= 1e-12 * scale)            # Newton's third law
    tot = orc.total_energy(b.pos, p, species=b.species)
    # Euler: U is linear in eps
    assert (eps * de).sum() == pytest.approx(tot["U_pair"] + tot["U_tail"], rel=1e-12)
    # virial: sum sigma dU_pair/dsigma = sum_pairs r * dU/dr contribution (pure-Python pair loop)
    tail_s = 0.0
    V = b.volume
    counts = np.bincount(b.species, minlength=2)
    for a in range(2):
        for c in range(2):
            q = sig[a, c] / 3.0
            tail_s += 8 * math.pi / (3 * V) * counts[a] * counts[c] * eps[a, c] * (
                4 * sig[a, c] ** 3 * q ** 9 - 6 * sig[a, c] ** 3 * q ** 3)
    vir = 0.0
    for i in range(b.n):
        d = b.pos - b.pos[i]
        d -= b.L * np.round(d / b.L)
        r2 = (d * d).sum(axis=1)
        for j in range(i + 1, b.n):
            if r2[j] < 9.0:
                s2 = sig[b.species[i], b.species[j]] ** 2 / r2[j]
                s6 = s2 ** 3
                vir += 24 * eps[b.species[i], b.species[j]] * (2 * s6 * s6 - s6)   # = -r u'(r)
    assert (sig * ds).sum() - tail_s == pytest.approx(vir, rel=1e-11)


def test_gradient_finite_differences(orc):
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    b = workloads.random_box(120, 8.5, seed=41, species_counts=[60, 60], eps=eps, sigma=sig)
    rc = 3.0
    p = orc.make_params(b.L, rc, eps=eps, sigma=sig)
    g, de, ds = orc.gradients(b.pos, p, species=b.species)
    h = 1e-6

    def U(pos, e=eps, s=sig):
        q = orc.make_params(b.L, rc, eps=e, sigma=s)
        t = orc.total_energy(pos, q, species=b.species)
        return t["U_pair"] + t["U_tail"]

    rng = np.random.default_rng(0)
    checked = 0
    for i in rng.choice(b.n, 20, replace=False):
        d = b.pos - b.pos[i]
        d -= b.L * np.round(d / b.L)
        r = np.sqrt((d * d).sum(axis=1))
        if np.any(np.abs(r - rc) < 10 * h):
            continue
        for a in range(3):
            pp = b.pos.copy(); pp[i, a] += h
            pm = b.pos.copy(); pm[i, a] -= h
            fd = (U(pp) - U(pm)) / (2 * h)
            assert fd == pytest.approx(g[i, a], rel=1e-5, abs=1e-6)
        checked += 1
    assert checked >= 10
    # parameters: a symmetric perturbation of an off-diagonal entry moves both [a][b] and [b][a]
    for (a, c) in ((0, 0), (0, 1), (1, 1)):
        E = np.zeros((2, 2)); E[a, c] = E[c, a] = 1.0
        fd_e = (U(b.pos, e=eps + h * E) - U(b.pos, e=eps - h * E)) / (2 * h)
        fd_s = (U(b.pos, s=sig + h * E) - U(b.pos, s=sig - h * E)) / (2 * h)
        want_e = de[a, c] + (de[c, a] if a != c else 0.0)
        want_s = ds[a, c] + (ds[c, a] if a != c else 0.0)
        assert fd_e == pytest.approx(want_e, rel=1e-6)
        assert fd_s == pytest.approx(want_s, rel=1e-5)


# --------------------------------------------------------------------------
# Virial and pressure: the tail against quadrature of its definition, the
# pair virial against the derivative of U_pair under uniform scaling
# --------------------------------------------------------------------------
def test_tail_pressure_vs_quadrature(orc):
    """P_tail = -(2 pi/3) sum_ab rho_a rho_b int_rc^inf r^3 u_ab'(r) dr, with u'
    taken by central differences of the potential (one and two species)."""
    from scipy.integrate import quad

    def u(r, e, s):
        return 4.0 * e * ((s / r) ** 12 - (s / r) ** 6)

    def du(r, e, s):
        h = 1e-5 * r
        return (u(r + h, e, s) - u(r - h, e, s)) / (2 * h)

    L = np.array([13.0, 14.0, 15.0])
    V = float((L[0] * L[1]) * L[2])
    for rc in (2.5, 3.0):
        p = orc.make_params(L, rc)
        integ, _ = quad(lambda r: r ** 3 * du(r, 1.0, 1.0), rc, np.inf, epsabs=0, epsrel=1e-12)
        N = 1234
        ref = -(2.0 * math.pi / 3.0) * (N / V) ** 2 * integ
        assert orc.tail_pressure([N], p) == pytest.approx(ref, rel=1e-8)
    eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    p = orc.make_params(L, 3.0, eps=eps, sigma=sig)
    counts = [700, 300]
    ref = 0.0
    for a in range(2):
        for b in range(2):
            integ, _ = quad(lambda r: r ** 3 * du(r, eps[a, b], sig[a, b]), 3.0, np.inf, epsabs=0, epsrel=1e-12)
            ref += -(2.0 * math.pi / 3.0) * counts[a] * counts[b] / V ** 2 * integ
    assert orc.tail_pressure(counts, p) == pytest.approx(ref, rel=1e-8)


@pytest.mark.parametrize("mixture", [False, True])
def test_virial_is_scaling_derivative(orc, mixture):
    """W = sum r u'(r) with the sign of -dU_pair/d lambda at lambda = 1 when every
    position and the box are scaled by lambda (no pair near the cutoff)."""
    if mixture:
        eps, sig = workloads.lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
        b = workloads.random_box(160, 8.5, seed=43, species_counts=[80, 80], eps=eps, sigma=sig)
        rc, sp = 3.0, b.species
    else:
        eps, sig = 1.0, 1.0
        b = workloads.random_box(200, 8.0, seed=44)
        rc, sp = 2.5, None
    d = b.pos[:, None, :] - b.pos[None, :, :]
    d -= b.L * np.round(d / b.L)
    r = np.sqrt((d * d).sum(axis=2))
    assert not np.any(np.abs(r[np.triu_indices(b.n, 1)] - rc) < 1e-5 * rc)
    h = 1e-6

    def U(lam):
        q = orc.make_params(np.asarray(b.L) * lam, rc, eps=eps, sigma=sig)
        return orc.total_energy(b.pos * lam, q, species=sp)["U_pair"]

    p = orc.make_params(b.L, rc, eps=eps, sigma=sig)
    v = orc.virial(b.pos, p, species=sp)
    fd = (U(1 + h) - U(1 - h)) / (2 * h)
    assert abs(v["W"] + fd) <= 1e-6 * v["sumabs"]
    assert v["sumabs"] > 0


def test_virial_ideal_gas(orc):
    b = workloads.random_box(100, 7.0, seed=45)
    p = orc.make_params(b.L, 2.5, eps=0.0, beta=1 / 1.7)
    v = orc.virial(b.pos, p)
    V = float(np.prod(b.L))
    assert v["W"] == 0.0 and v["P_tail"] == 0.0
    assert v["P"] == pytest.approx(100 * 1.7 / V, rel=1e-15)


# --------------------------------------------------------------------------
# The running virial of the chain (Sec. 3.1.2: an accepted move updates the
# virial pressure with the energy)
# --------------------------------------------------------------------------
def test_position_virial_two_particle_closed_form(orc):
    """w(r) = -r du/dr = 24 eps [2 (sigma/r)^12 - (sigma/r)^6] inside the cutoff, exact rationals."""
    L = np.array([9.0, 9.0, 9.0])
    p = orc.make_params(L, 2.5, eps=1.5, sigma=1.25)
    for r in (1.0, 1.25, 1.5, 2.0, 2.49):
        pos = np.array([[0.5, 4.0, 4.0], [0.5 + r, 4.0, 4.0]])
        q = Fraction(5, 4) / Fraction(r)
        want = float(24 * Fraction(3, 2) * (2 * q ** 12 - q ** 6))
        got, _ = orc.position_virial(pos, p, pos[0], exclude=0)
        assert got == pytest.approx(want, rel=1e-14, abs=1e-15)
    # across the periodic boundary, and zero beyond the cutoff
    pos = np.array([[0.2, 4.0, 4.0], [8.0, 4.0, 4.0]])
    q = Fraction(5, 4) / Fraction(12, 10)
    assert orc.position_virial(pos, p, pos[0], exclude=0)[0] == pytest.approx(
        float(24 * Fraction(3, 2) * (2 * q ** 12 - q ** 6)), rel=1e-13)
    pos = np.array([[0.5, 4.0, 4.0], [3.0, 4.0, 4.0]])
    assert orc.position_virial(pos, p, pos[0], exclude=0)[0] == 0.0


def test_position_virial_half_sum(orc):
    b = workloads.random_box(150, 8.0, seed=61)
    p = orc.make_params(b.L, 2.5)
    s = sum(orc.position_virial(b.pos, p, b.pos[i], exclude=i)[0] for i in range(b.n))
    assert s == pytest.approx(2 * orc.virial(b.pos, p)["W"], rel=1e-12)


def test_chain_virial_bookkeeping(orc):
    """The running W (starting from the total virial, plus every accepted move's
    dW) equals the total virial of the final configuration; ideal-gas moves change
    nothing."""
    b = workloads.random_box(200, 8.0, seed=21, T=1.2)
    p = orc.make_params(b.L, 2.5, beta=1.0 / 1.2, mu=-3.0)
    W0 = orc.virial(b.pos, p)["W"]
    pos, _, W, log = orc.chain(b.pos, 3000, p, seed=5, W0=W0)
    assert W == pytest.approx(orc.virial(pos, p)["W"], rel=1e-10, abs=1e-9)
    acc = log["accepted"] == 1
    assert np.any(acc & (log["dW_pair"] != 0.0))
    q = orc.make_params(b.L, 2.5, eps=0.0, mu=-1.0)
    _, _, Wq, logq = orc.chain(b.pos, 500, q, seed=6, W0=0.0)
    assert Wq == 0.0 and np.all(logq["dW_pair"] == 0.0)


# --------------------------------------------------------------------------
# The CPU-baseline variants of the oracle chain (several threads; a cell
# list): the same chain as the plain all-pairs loop, decision for decision
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,L,seed,mu", [(400, 10.0, 3, -2.0), (120, 7.4, 4, -1.0), (300, [8.0, 9.5, 12.7], 5, 0.5)])
def test_chain_variants_equal_plain_chain(orc, n, L, seed, mu):
    b = workloads.random_box(n, L, seed=seed, T=1.2)
    p = orc.make_params(b.L, 2.5, beta=1.0 / 1.2, mu=mu)
    t0 = orc.total_energy(b.pos, p)
    U0 = t0["U_pair"] + t0["U_tail"]
    W0 = orc.virial(b.pos, p)["W"]
    ref = orc.chain(b.pos, 2000, p, seed=11, max_n=n + 2001, U0=U0, W0=W0)
    acc = ref[3]["accepted"] == 1
    assert acc.sum() > 100 and np.any(acc & (ref[3]["type"] == 2)) and np.any(acc & (ref[3]["type"] == 1))
    for kw in ({"threads": 4}, {"threads": 7}, {"mode": "cells"}):
        got = orc.chain(b.pos, 2000, p, seed=11, max_n=n + 2001, U0=U0, W0=W0, **kw)
        for f in ("type", "index", "accepted", "flags", "x", "y", "z"):
            assert np.array_equal(got[3][f], ref[3][f]), (kw, f)
        assert np.allclose(got[3]["dU_pair"], ref[3]["dU_pair"], rtol=0,
                           atol=1e-12 * max(1.0, np.abs(ref[3]["sumabs"]).max()))
        assert np.array_equal(got[0], ref[0])
        assert got[1] == pytest.approx(ref[1], rel=1e-12)
        assert got[2] == pytest.approx(ref[2], rel=1e-12)
