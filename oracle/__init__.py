"""FP64 CPU oracle for the GCMC energy path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never imports it and
shares no code with it: ``gcmc_oracle.c`` is a plain all-pairs implementation of
the method of Schwiebert et al. (arXiv 1408.3764), written independently.

The C library is compiled by :func:`build` (gcc, ``-O2 -ffp-contract=off``) and
loaded through ctypes.  Every wrapper here only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gcmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAX_SPECIES = 4


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (no FMA contraction)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("L", C.c_double * 3),
        ("rc", C.c_double),
        ("ns", C.c_int32),
        ("pad0", C.c_int32),
        ("eps", C.c_double * (MAX_SPECIES * MAX_SPECIES)),
        ("sigma", C.c_double * (MAX_SPECIES * MAX_SPECIES)),
        ("beta", C.c_double),
        ("mu", C.c_double),
        ("lambda3", C.c_double),
        ("max_disp", C.c_double),
        ("p_disp", C.c_double),
    ]


LOG_DTYPE = np.dtype([
    ("type", np.int32), ("index", np.int32), ("accepted", np.int32), ("flags", np.int32),
    ("dU_pair", np.float64), ("dU_tail", np.float64), ("sumabs", np.float64),
    ("x", np.float64), ("y", np.float64), ("z", np.float64),
    ("arg", np.float64), ("a", np.float64), ("dW_pair", np.float64), ("wsumabs", np.float64),
])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        up = C.POINTER(C.c_uint32)
        pp = C.POINTER(Params)
        L.oracle_philox4x32_10.argtypes = [up, up, up]
        L.oracle_u01.argtypes = [C.c_uint32, C.c_uint32]
        L.oracle_u01.restype = C.c_double
        L.oracle_move_draws.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, dp]
        L.oracle_pick.argtypes = [C.c_double, C.c_double, C.c_int64]
        L.oracle_pick.restype = C.c_int64
        L.oracle_lj_r2.argtypes = [C.c_double] * 4
        L.oracle_lj_r2.restype = C.c_double
        L.oracle_min_image.argtypes = [C.c_double, C.c_double]
        L.oracle_min_image.restype = C.c_double
        L.oracle_position_energy.argtypes = [C.c_int64, dp, dp, dp, ip, C.c_double, C.c_double, C.c_double,
                                             C.c_int32, C.c_int64, pp, dp]
        L.oracle_total_energy.argtypes = [C.c_int64, dp, dp, dp, ip, pp, dp, dp]
        L.oracle_tail_energy.argtypes = [lp, pp]
        L.oracle_tail_energy.restype = C.c_double
        L.oracle_tail_delta.argtypes = [lp, C.c_int32, C.c_int32, pp]
        L.oracle_tail_delta.restype = C.c_double
        L.oracle_accept_arg.argtypes = [C.c_int32, C.c_double, C.c_int64, pp]
        L.oracle_accept_arg.restype = C.c_double
        L.oracle_accept.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_accept.restype = C.c_int32
        L.oracle_chain.argtypes = [C.c_int64, dp, dp, dp, lp, dp, dp, pp, C.c_uint64, C.c_uint32, C.c_uint64,
                                   C.c_int64, C.c_void_p]
        for name in ("oracle_chain_mt", "oracle_chain_cells"):
            f = getattr(L, name)
            f.argtypes = L.oracle_chain.argtypes + ([C.c_int32] if name == "oracle_chain_mt" else [])
            f.restype = C.c_int
        L.oracle_position_virial.argtypes = [C.c_int64, dp, dp, dp, ip, C.c_double, C.c_double, C.c_double,
                                             C.c_int32, C.c_int64, pp, dp]
        L.oracle_chain.restype = C.c_int
        L.oracle_grid.argtypes = [dp, C.c_double, ip, ip, dp, ip, ip]
        L.oracle_cell_of.argtypes = [C.c_double, C.c_double, C.c_double, ip, dp]
        L.oracle_cell_of.restype = C.c_int64
        L.oracle_neighbor_ids.argtypes = [C.c_int64, dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_int64,
                                          dp, C.c_double, ip, lp, C.c_int64]
        L.oracle_neighbor_ids.restype = C.c_int64
        L.oracle_stencil_count.argtypes = [dp, C.c_double, ip]
        L.oracle_stencil_count.restype = C.c_int32
        L.oracle_particle_gradient.argtypes = [C.c_int64, dp, dp, dp, ip, C.c_int64, pp, dp]
        L.oracle_gradients.argtypes = [C.c_int64, dp, dp, dp, ip, pp, dp, dp, dp, dp, dp]
        L.oracle_tail_pressure.argtypes = [lp, pp]
        L.oracle_tail_pressure.restype = C.c_double
        L.oracle_virial.argtypes = [C.c_int64, dp, dp, dp, ip, pp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))


def _l(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(L, rc, eps=1.0, sigma=1.0, beta=1.0, mu=0.0, lambda3=1.0, max_disp=0.3, p_disp=1.0 / 3.0):
    """Build the oracle's parameter block.  eps/sigma: scalar or (ns, ns) pair tables."""
    p = Params()
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    for a in range(3):
        p.L[a] = float(L[a])
    p.rc = float(rc)
    e = np.atleast_2d(np.asarray(eps, dtype=np.float64))
    s = np.atleast_2d(np.asarray(sigma, dtype=np.float64))
    ns = e.shape[0]
    assert e.shape == (ns, ns) and s.shape == (ns, ns) and ns <= MAX_SPECIES
    p.ns = ns
    for a in range(ns):
        for b in range(ns):
            p.eps[a * ns + b] = float(e[a, b])
            p.sigma[a * ns + b] = float(s[a, b])
    p.beta, p.mu, p.lambda3, p.max_disp, p.p_disp = float(beta), float(mu), float(lambda3), float(max_disp), float(p_disp)
    return p


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    up = C.POINTER(C.c_uint32)
    lib().oracle_philox4x32_10(c.ctypes.data_as(up), k.ctypes.data_as(up), out.ctypes.data_as(up))
    return out


def u01(a, b):
    return lib().oracle_u01(int(a), int(b))


def move_draws(seed, move, box=0):
    u = np.zeros(8)
    lib().oracle_move_draws(int(seed), int(move), int(box), _d(u))
    return u


def pick(u_pick, u_spare, n):
    """The particle a displacement or deletion picks among n >= 1 (Algorithm 2's
    random particle): the first b-bit field of u_spare's 53 bits (2^b >= n) below
    n, else min(floor(u_pick n), n - 1)."""
    return int(lib().oracle_pick(float(u_pick), float(u_spare), int(n)))


def lj_r2(r2, eps, sigma, rc):
    return lib().oracle_lj_r2(float(r2), float(eps), float(sigma), float(rc))


def min_image(d, L):
    return lib().oracle_min_image(float(d), float(L))


def position_energy(pos, p, point, exclude=-1, species=None, point_species=0):
    """(sum_j u, sum_j |u|) of a particle at `point` with every particle but `exclude`."""
    x, y, z = (_f64(pos[:, a]) for a in range(3))
    sp = None if species is None else np.ascontiguousarray(species, dtype=np.int32)
    out = np.zeros(2)
    lib().oracle_position_energy(len(x), _d(x), _d(y), _d(z), _i(sp), float(point[0]), float(point[1]),
                                 float(point[2]), int(point_species), int(exclude), C.byref(p), _d(out))
    return float(out[0]), float(out[1])


def position_virial(pos, p, point, exclude=-1, species=None, point_species=0):
    """(sum_j w, sum_j |w|) of a particle at `point` with every particle but `exclude`."""
    x, y, z = (_f64(pos[:, a]) for a in range(3))
    sp = None if species is None else np.ascontiguousarray(species, dtype=np.int32)
    out = np.zeros(2)
    lib().oracle_position_virial(len(x), _d(x), _d(y), _d(z), _i(sp), float(point[0]), float(point[1]),
                                 float(point[2]), int(point_species), int(exclude), C.byref(p), _d(out))
    return float(out[0]), float(out[1])


def total_energy(pos, p, species=None, per_particle=False):
    """Returns dict(U_pair, sumabs, U_tail[, e])."""
    x, y, z = (_f64(pos[:, a]) for a in range(3))
    n = len(x)
    sp = None if species is None else np.ascontiguousarray(species, dtype=np.int32)
    out = np.zeros(3)
    e = np.zeros(n) if per_particle else None
    lib().oracle_total_energy(n, _d(x), _d(y), _d(z), _i(sp), C.byref(p), _d(out),
                              _d(e) if e is not None else None)
    r = {"U_pair": float(out[0]), "sumabs": float(out[1]), "U_tail": float(out[2])}
    if e is not None:
        r["e"] = e
    return r


def tail_energy(counts, p):
    c = np.ascontiguousarray(counts, dtype=np.int64)
    return lib().oracle_tail_energy(_l(c), C.byref(p))


def tail_delta(counts, species, sign, p):
    c = np.ascontiguousarray(counts, dtype=np.int64)
    return lib().oracle_tail_delta(_l(c), int(species), int(sign), C.byref(p))


def accept_arg(move_type, dU, n, p):
    return lib().oracle_accept_arg(int(move_type), float(dU), int(n), C.byref(p))


def accept(arg, dU, A):
    return int(lib().oracle_accept(float(arg), float(dU), float(A)))


class ChainError(RuntimeError):
    pass


def chain(pos, n_moves, p, seed, box=0, counter0=0, max_n=None, U0=0.0, W0=None, mode="allpairs", threads=1):
    """Run the serial GCMC chain.  Returns (pos[n], U, log array), or with W0
    given (the starting pair virial) (pos[n], U, W, log array).  mode
    "allpairs" (threads > 1: each position's sums split over that many
    threads) or "cells" (sums over the stencil cells of a cell list): the
    CPU-baseline variants; the parity tests use the default."""
    n0 = pos.shape[0]
    max_n = max_n if max_n is not None else n0 + n_moves + 1
    x = np.zeros(max_n); y = np.zeros(max_n); z = np.zeros(max_n)
    x[:n0], y[:n0], z[:n0] = pos[:, 0], pos[:, 1], pos[:, 2]
    n = C.c_int64(n0)
    U = C.c_double(U0)
    W = C.c_double(0.0 if W0 is None else W0)
    log = np.zeros(int(n_moves), dtype=LOG_DTYPE)
    args = [int(max_n), _d(x), _d(y), _d(z), C.byref(n), C.byref(U), C.byref(W), C.byref(p), int(seed), int(box),
            int(counter0), int(n_moves), log.ctypes.data_as(C.c_void_p)]
    if mode == "cells":
        rc = lib().oracle_chain_cells(*args)
    elif threads > 1:
        rc = lib().oracle_chain_mt(*args, int(threads))
    else:
        rc = lib().oracle_chain(*args)
    if rc != 0:
        raise ChainError("oracle_chain returned %d" % rc)
    k = n.value
    pos_out = np.stack([x[:k], y[:k], z[:k]], axis=1)
    if W0 is None:
        return pos_out, U.value, log
    return pos_out, U.value, W.value, log


def grid(L, rc, req_m=None):
    Lx = _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    rq = np.zeros(3, dtype=np.int32) if req_m is None else np.ascontiguousarray(req_m, dtype=np.int32)
    M = np.zeros(3, dtype=np.int32); invS = np.zeros(3); k = np.zeros(3, dtype=np.int32)
    span = np.zeros(3, dtype=np.int32)
    lib().oracle_grid(_d(Lx), float(rc), _i(rq), _i(M), _d(invS), _i(k), _i(span))
    return {"M": M, "invS": invS, "k": k, "span": span}


def stencil_count(L, rc, req_m=None):
    """Stencil cells kept after dropping those beyond the cutoff."""
    Lx = _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    rq = np.zeros(3, dtype=np.int32) if req_m is None else np.ascontiguousarray(req_m, dtype=np.int32)
    return int(lib().oracle_stencil_count(_d(Lx), float(rc), _i(rq)))


def cell_of(pos, L, rc, req_m=None):
    g = grid(L, rc, req_m)
    M, invS = g["M"], g["invS"]
    f = lib().oracle_cell_of
    return np.array([f(float(q[0]), float(q[1]), float(q[2]), _i(M), _d(invS)) for q in pos], dtype=np.int64)


def neighbor_ids(pos, point, L, rc, exclude=-1, req_m=None):
    x, y, z = (_f64(pos[:, a]) for a in range(3))
    Lx = _f64(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    rq = np.zeros(3, dtype=np.int32) if req_m is None else np.ascontiguousarray(req_m, dtype=np.int32)
    out = np.zeros(len(x), dtype=np.int64)
    cnt = lib().oracle_neighbor_ids(len(x), _d(x), _d(y), _d(z), float(point[0]), float(point[1]),
                                    float(point[2]), int(exclude), _d(Lx), float(rc), _i(rq), _l(out), len(out))
    return out[:cnt].copy()


def particle_gradient(pos, i, p, species=None):
    x, y, z = (_f64(pos[:, a]) for a in range(3))
    sp = None if species is None else np.ascontiguousarray(species, dtype=np.int32)
    g = np.zeros(3)
    lib().oracle_particle_gradient(len(x), _d(x), _d(y), _d(z), _i(sp), int(i), C.byref(p), _d(g))
    return g


def gradients(pos, p, species=None, positions=True):
    """Returns (dU/dpos [n,3] or None, dU/deps [ns,ns], dU/dsigma [ns,ns])."""
    x, y, z = (_f64(pos[:, a]) for a in range(3))
    n = len(x)
    sp = None if species is None else np.ascontiguousarray(species, dtype=np.int32)
    ns = p.ns
    gx = np.zeros(n); gy = np.zeros(n); gz = np.zeros(n)
    de = np.zeros(ns * ns); ds = np.zeros(ns * ns)
    if positions:
        lib().oracle_gradients(n, _d(x), _d(y), _d(z), _i(sp), C.byref(p), _d(gx), _d(gy), _d(gz), _d(de), _d(ds))
        g = np.stack([gx, gy, gz], axis=1)
    else:
        lib().oracle_gradients(n, _d(x), _d(y), _d(z), _i(sp), C.byref(p), None, None, None, _d(de), _d(ds))
        g = None
    return g, de.reshape(ns, ns), ds.reshape(ns, ns)


def virial(pos, p, species=None):
    """Pair virial and pressure: {"W", "sumabs", "P_tail", "P"} (P = N/(beta V) + W/(3V) + P_tail)."""
    x, y, z = (_f64(pos[:, a]) for a in range(3))
    sp = None if species is None else np.ascontiguousarray(species, dtype=np.int32)
    out = np.zeros(4)
    lib().oracle_virial(len(x), _d(x), _d(y), _d(z), _i(sp), C.byref(p), _d(out))
    return {"W": float(out[0]), "sumabs": float(out[1]), "P_tail": float(out[2]), "P": float(out[3])}


def tail_pressure(counts, p):
    c = np.ascontiguousarray(counts, dtype=np.int64)
    return float(lib().oracle_tail_pressure(_l(c), C.byref(p)))
