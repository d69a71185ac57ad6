"""Seeded synthetic inputs shaped like the paper's Lennard-Jones workloads.

This module only *generates inputs*: random particle placements with overlap
rejection, box sizes and ensemble parameters.  It holds none of the method's
arithmetic (no pair energies, no acceptance rules, no cell list) and is the
only code that both the GPU path and the CPU oracle consume.

Placement recipe (random sequential addition, batched): candidate points are
drawn uniformly in the target region with numpy's PCG64 generator seeded by
``seed``; a candidate is kept if no kept particle lies closer than
``0.8 * sigma_ab`` (periodic distance), and within one batch a candidate that
conflicts with an earlier candidate of the same batch is dropped.  The result is
deterministic for a given seed.

Workloads (the paper's shapes: LJ fluids at reduced density 0.5-0.8, cutoff
2.5-3 sigma, from small boxes to over a million particles; Sec. 4):

* ``small``   N=4,000, rho=0.5, L=cbrt(8000)=20 exactly, T*=1.2, rc=2.5, 1,000 moves
* ``large``   N=262,144, rho=0.7, T*=1.0, rc=3.0, 100,000 moves
* ``slab``    box a x a x 4a, liquid slab z in [a,3a) at rho=0.8 inside vapour at
              rho=0.02, N~1,500,000, T*=0.85, rc=2.5, 200,000 moves
* ``batched`` 512 boxes, N log-uniform in [128, 32768], rho U[0.3,0.8], T* U[0.9,1.5]
* ``mixture`` binary 50/50, N=262,144, sigma=[1.0,1.2], eps=[1.0,0.8],
              Lorentz-Berthelot mixing, rho=0.6, rc=3.0 (2.5 sigma_max)

All use mu*=-3.0, Lambda^3=1, displacement half-width 0.3, and the move mix
1/3 displace, 1/3 insert, 1/3 delete.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BASE_SEED = 1408376400


@dataclasses.dataclass
class Box:
    """One simulation box: positions in [0, L) and the ensemble parameters."""
    pos: np.ndarray                 # (N, 3) float64
    L: np.ndarray                   # (3,) float64
    rc: float
    beta: float
    mu: float = -3.0
    lambda3: float = 1.0
    max_disp: float = 0.3
    p_disp: float = 1.0 / 3.0
    eps: np.ndarray = dataclasses.field(default_factory=lambda: np.ones((1, 1)))
    sigma: np.ndarray = dataclasses.field(default_factory=lambda: np.ones((1, 1)))
    species: Optional[np.ndarray] = None   # (N,) int32 or None (single species)
    seed: int = 0                   # Philox key of the move stream
    n_moves: int = 0
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def volume(self) -> float:
        return float((self.L[0] * self.L[1]) * self.L[2])


def lorentz_berthelot(sig, eps):
    """Pair tables from per-species sigma and epsilon: arithmetic / geometric means."""
    sig = np.asarray(sig, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    s = 0.5 * (sig[:, None] + sig[None, :])
    e = np.sqrt(eps[:, None] * eps[None, :])
    return e, s


def _min_dist_table(sigma_tab):
    return 0.8 * np.asarray(sigma_tab, dtype=np.float64)


def rsa_place(n, L, rng, lo=None, hi=None, existing=None, species_counts=None, existing_species=None,
              sigma_tab=None, max_batch=2_000_000):
    """Place n points uniformly in the region [lo, hi) of a periodic box of size L,
    rejecting any point closer than 0.8*sigma_ab to a kept point.  With
    species_counts, candidates draw their species in proportion to what is still
    missing, and exactly species_counts[s] points of species s are kept.

    Returns (points (n,3), species (n,) int32 or None)."""
    from scipy.spatial import cKDTree

    L = np.asarray(L, dtype=np.float64)
    lo = np.zeros(3) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = L.copy() if hi is None else np.asarray(hi, dtype=np.float64)
    sig = np.ones((1, 1)) if sigma_tab is None else np.asarray(sigma_tab, dtype=np.float64)
    dmin = _min_dist_table(sig)
    dmax = float(dmin.max())
    ns = dmin.shape[0]
    top = np.nextafter(L, 0.0)

    kept = np.zeros((0, 3)) if existing is None else np.asarray(existing, dtype=np.float64)
    kept_sp = (np.zeros(len(kept), dtype=np.int32) if existing_species is None
               else np.asarray(existing_species, dtype=np.int32))
    n_old = len(kept)
    missing = None if species_counts is None else np.asarray(species_counts, dtype=np.int64).copy()
    if missing is not None:
        assert missing.sum() == n
    placed = 0
    acc = 0.5
    while placed < n:
        need = n - placed
        B = int(min(max_batch, max(256, math.ceil(1.2 * need / max(acc, 0.02)))))
        cand = lo + rng.random((B, 3)) * (hi - lo)
        cand = np.minimum(cand, top)
        if missing is None:
            csp = np.zeros(B, dtype=np.int32)
        else:
            cum = np.cumsum(missing) / missing.sum()
            csp = np.searchsorted(cum, rng.random(B), side="right").astype(np.int32)
            csp = np.minimum(csp, len(missing) - 1)
        ok = np.ones(B, dtype=bool)
        if len(kept):
            tree = cKDTree(kept, boxsize=L)
            kq = 12 if ns > 1 else 1
            d, idx = tree.query(cand, k=kq, distance_upper_bound=dmax)
            if kq == 1:
                d = d[:, None]
                idx = idx[:, None]
            hit = np.isfinite(d)
            idx_c = np.where(hit, idx, 0)
            thr = dmin[csp[:, None], kept_sp[idx_c]]
            ok &= ~np.any(hit & (d < thr), axis=1)
        c_ok = np.nonzero(ok)[0]
        if len(c_ok) > 1:
            ctree = cKDTree(cand[c_ok], boxsize=L)
            pairs = ctree.query_pairs(dmax, output_type="ndarray")
            if len(pairs):
                a, b = pairs[:, 0], pairs[:, 1]
                pa, pb = cand[c_ok[a]], cand[c_ok[b]]
                dd = np.abs(pa - pb)
                dd = np.minimum(dd, L - dd)
                dist = np.sqrt((dd * dd).sum(axis=1))
                bad = dist < dmin[csp[c_ok[a]], csp[c_ok[b]]]
                later = np.maximum(a[bad], b[bad])
                ok[c_ok[later]] = False
        good = np.nonzero(ok)[0]
        acc = max(len(good) / B, 1e-3)
        if missing is None:
            good = good[:need]
        else:
            sel = []
            for s in range(len(missing)):
                gs = good[csp[good] == s][: int(missing[s])]
                missing[s] -= len(gs)
                sel.append(gs)
            good = np.sort(np.concatenate(sel))
        kept = np.concatenate([kept, cand[good]], axis=0)
        kept_sp = np.concatenate([kept_sp, csp[good]])
        placed += len(good)
    new = kept[n_old:]
    return new, (None if missing is None else kept_sp[n_old:].astype(np.int32))


def cubic_box(n, rho, T, rc, seed, n_moves=0, name="", mu=-3.0):
    L = float(np.cbrt(n / rho))
    rng = np.random.Generator(np.random.PCG64(seed))
    Lv = np.array([L, L, L])
    pos, _ = rsa_place(n, Lv, rng)
    return Box(pos=pos, L=Lv, rc=rc, beta=1.0 / T, mu=mu, seed=seed, n_moves=n_moves, name=name)


def small(seed=BASE_SEED + 0):
    """N=4,000 at rho=0.5: L = cbrt(8000) = 20 exactly, so 8 cells of side 2.5 per axis."""
    b = cubic_box(4000, 0.5, 1.2, 2.5, seed, n_moves=1000, name="small N=4000 rho=0.5 rc=2.5")
    assert b.L[0] == 20.0
    return b


def large(seed=BASE_SEED + 1, n=262_144):
    return cubic_box(n, 0.7, 1.0, 3.0, seed, n_moves=100_000, name="large N=%d rho=0.7 rc=3.0" % n)


def slab(seed=BASE_SEED + 2, n_total=1_500_000, rho_l=0.8, rho_v=0.02):
    """Box a x a x 4a; the middle half in z is liquid, the rest vapour."""
    a = float(np.cbrt(n_total / (2.0 * rho_l + 2.0 * rho_v)))
    L = np.array([a, a, 4.0 * a])
    n_l = int(round(2.0 * rho_l * a ** 3))
    n_v = n_total - n_l
    rng = np.random.Generator(np.random.PCG64(seed))
    liq, _ = rsa_place(n_l, L, rng, lo=[0, 0, a], hi=[a, a, 3 * a])
    # vapour: lower and upper quarters, equal shares
    n_v0 = n_v // 2
    v0, _ = rsa_place(n_v0, L, rng, lo=[0, 0, 0], hi=[a, a, a], existing=liq)
    v1, _ = rsa_place(n_v - n_v0, L, rng, lo=[0, 0, 3 * a], hi=[a, a, 4 * a],
                      existing=np.concatenate([liq, v0]))
    pos = np.concatenate([liq, v0, v1], axis=0)
    perm = rng.permutation(len(pos))
    pos = pos[perm]
    return Box(pos=pos, L=L, rc=2.5, beta=1.0 / 0.85, seed=seed, n_moves=200_000,
               name="slab 1:1:4 N=%d rho_l=0.8 rho_v=0.02 rc=2.5" % n_total)


def paper_size(n, seed=BASE_SEED + 5):
    """The paper's size study (Sec. 4): N particles at density 0.67, rc = 2.5,
    30 % displacements and 35 % each insertions and deletions.  The paper states
    no temperature or chemical potential for it: T* = 1.2, mu* = -3 are taken."""
    b = cubic_box(n, 0.67, 1.2, 2.5, seed, name="size study N=%d rho=0.67 rc=2.5" % n)
    b.p_disp = 0.3
    return b


def paper_cutoff(rcs, seed=BASE_SEED + 6, n=87_296, volume=131_072.0):
    """The paper's cutoff study (Sec. 4): one configuration of 87,296 particles in
    a cube of 128K sigma^3 (density 0.666), the same move mix and state as the
    size study, one box per cutoff in rcs."""
    L = float(np.cbrt(volume))
    rng = np.random.Generator(np.random.PCG64(seed))
    Lv = np.array([L, L, L])
    pos, _ = rsa_place(n, Lv, rng)
    return [Box(pos=pos, L=Lv.copy(), rc=float(rc), beta=1.0 / 1.2, mu=-3.0, p_disp=0.3, seed=seed,
                name="cutoff study N=%d V=%g rc=%g" % (n, volume, rc)) for rc in rcs]


def batched(seed=BASE_SEED + 3, n_boxes=512, n_min=128, n_max=32768) -> List[Box]:
    rng = np.random.Generator(np.random.PCG64(seed))
    ln = rng.uniform(math.log(n_min), math.log(n_max), n_boxes)
    ns = np.clip(np.rint(np.exp(ln)).astype(np.int64), n_min, n_max)
    rhos = rng.uniform(0.3, 0.8, n_boxes)
    Ts = rng.uniform(0.9, 1.5, n_boxes)
    boxes = []
    for b in range(n_boxes):
        bb = cubic_box(int(ns[b]), float(rhos[b]), float(Ts[b]), 2.5, seed * 1000 + b, n_moves=1000,
                       name="batched box %d" % b)
        bb.seed = seed
        boxes.append(bb)
    return boxes


def mixture(seed=BASE_SEED + 4, n=262_144, rho=0.6):
    eps, sig = lorentz_berthelot([1.0, 1.2], [1.0, 0.8])
    L = float(np.cbrt(n / rho))
    Lv = np.array([L, L, L])
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, sp = rsa_place(n, Lv, rng, species_counts=[n // 2, n - n // 2], sigma_tab=sig)
    return Box(pos=pos, L=Lv, rc=2.5 * 1.2, beta=1.0, eps=eps, sigma=sig, species=sp, seed=seed,
               name="mixture N=%d rho=0.6 rc=3.0" % n)


def random_box(n, L, rc=2.5, T=1.0, seed=0, mu=-3.0, min_frac=0.8, species_counts=None, eps=None, sigma=None):
    """A small box for tests: n points with overlap rejection in a box of sides L."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)).copy()
    sig_tab = np.ones((1, 1)) if sigma is None else np.asarray(sigma, dtype=np.float64)
    eps_tab = np.ones((1, 1)) if eps is None else np.asarray(eps, dtype=np.float64)
    pos, sp = rsa_place(n, Lv, rng, species_counts=species_counts, sigma_tab=sig_tab * (min_frac / 0.8))
    return Box(pos=pos, L=Lv, rc=rc, beta=1.0 / T, mu=mu, eps=eps_tab, sigma=sig_tab, species=sp, seed=seed)
