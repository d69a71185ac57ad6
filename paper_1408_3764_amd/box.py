"""Python-side handle of one box / one batch of boxes on the GPU.

Marshalling only: numpy/torch arrays in, device tensors handed to the C ABI
(``_lib``), results copied back.  Every computation happens in libgcmc.so.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import LOG_DTYPE, MOVE_DTYPE, STATS_DTYPE


def _dev(a, dtype, device):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


def _struct_to_device(arr: np.ndarray, device) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.uint8).copy()).to(device)


def _struct_from_device(t: torch.Tensor, dtype) -> np.ndarray:
    return t.cpu().numpy().view(dtype).copy()


class Box:
    """One periodic box of Lennard-Jones particles held by the GPU library."""

    def __init__(self, pos, L, rc, beta=1.0, mu=0.0, lambda3=1.0, max_disp=0.3, p_disp=1.0 / 3.0, eps=1.0,
                 sigma=1.0, species=None, max_n=None, cell_m=None, cell_cap=0, seed=0, box_id=0,
                 device="cuda", stream=None):
        self.device = torch.device(device)
        self.stream = stream
        pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        n = pos.shape[0]
        e = np.atleast_2d(np.asarray(eps, dtype=np.float64))
        s = np.atleast_2d(np.asarray(sigma, dtype=np.float64))
        self.ns = e.shape[0]
        self._eps = np.ascontiguousarray(e.reshape(-1))
        self._sig = np.ascontiguousarray(s.reshape(-1))
        d = _lib.BoxDesc()
        Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
        for a in range(3):
            d.L[a] = float(Lv[a])
            d.cell_m[a] = 0 if cell_m is None else int(np.broadcast_to(cell_m, (3,))[a])
        d.rc, d.beta, d.mu, d.lambda3 = float(rc), float(beta), float(mu), float(lambda3)
        d.max_disp, d.p_disp = float(max_disp), float(p_disp)
        d.n_species = self.ns
        d.cell_cap = int(cell_cap)
        d.eps = self._eps.ctypes.data_as(C.POINTER(C.c_double))
        d.sigma = self._sig.ctypes.data_as(C.POINTER(C.c_double))
        d.max_n = int(max_n if max_n is not None else max(n, 1))
        d.box_id = int(box_id)
        d.seed = int(seed)
        self.desc = d
        self.L = Lv.copy()
        self.rc = float(rc)
        x = _dev(pos[:, 0], torch.float64, self.device)
        y = _dev(pos[:, 1], torch.float64, self.device)
        z = _dev(pos[:, 2], torch.float64, self.device)
        sp = None if species is None else _dev(species, torch.int32, self.device)
        self.handle = _lib.gcmc_box_create(d, x, y, z, sp, n, stream)
        self.max_n = d.max_n
        self.launch = (4, 4)   # the library's default shape (per-move kernel, 4 x 4)
        # bumped by every call that changes the configuration or the force field
        self.version = 0

    @classmethod
    def from_workload(cls, wb, max_n=None, **kw):
        kw.setdefault("seed", wb.seed)
        return cls(wb.pos, wb.L, wb.rc, beta=wb.beta, mu=wb.mu, lambda3=wb.lambda3, max_disp=wb.max_disp,
                   p_disp=wb.p_disp, eps=wb.eps, sigma=wb.sigma, species=wb.species,
                   max_n=max_n if max_n is not None else wb.n, **kw)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.gcmc_box_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ info
    def info(self):
        i = _lib.gcmc_box_get_info(self.handle)
        return {"cell_m": list(i.cell_m), "span": list(i.span), "cell_cap": i.cell_cap, "n_species": i.n_species,
                "n_cells": i.n_cells, "max_n": i.max_n, "inv_s": list(i.inv_s), "n_stencil": i.n_stencil}

    def set_launch(self, waves, rows):
        _lib.gcmc_box_set_launch(self.handle, waves, rows)
        self.launch = (int(waves), int(rows))

    def set_wait_limit(self, polls):
        """Bound on the chain kernels' in-kernel waits (0: default; < 0: fail at once)."""
        _lib.gcmc_box_set_wait_limit(self.handle, polls)

    # ----------------------------------------------------------------- moves
    def delta_energy(self, moves: np.ndarray, all_pairs=False, virial=False):
        """(dU_pair, dU_tail[, dW_pair]) of each move against the current configuration."""
        moves = np.asarray(moves, dtype=MOVE_DTYPE)
        m = len(moves)
        dm = _struct_to_device(moves, self.device)
        dp = torch.empty(m, dtype=torch.float64, device=self.device)
        dt = torch.empty(m, dtype=torch.float64, device=self.device)
        dw = torch.empty(m, dtype=torch.float64, device=self.device) if virial else None
        f = _lib.gcmc_delta_energy_allpairs if all_pairs else _lib.gcmc_delta_energy
        f(self.handle, dm, m, dp, dt, dw, self.stream)
        if virial:
            return dp.cpu().numpy(), dt.cpu().numpy(), dw.cpu().numpy()
        return dp.cpu().numpy(), dt.cpu().numpy()

    def commit(self, move, dU_pair, dW_pair=None):
        mv = np.asarray([move], dtype=MOVE_DTYPE) if not isinstance(move, np.ndarray) else move.reshape(1)
        dm = _struct_to_device(mv, self.device)
        du = torch.tensor([float(dU_pair)], dtype=torch.float64, device=self.device)
        dw = None if dW_pair is None else torch.tensor([float(dW_pair)], dtype=torch.float64, device=self.device)
        _lib.gcmc_commit(self.handle, dm, du, dw, self.stream)
        self.version += 1
        self.sync()

    def step(self, n_moves, counter0=0, log=False, all_pairs=False):
        st = torch.zeros(STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        lg = torch.zeros(max(1, n_moves) * LOG_DTYPE.itemsize, dtype=torch.uint8, device=self.device) if log else None
        f = _lib.gcmc_step_allpairs if all_pairs else _lib.gcmc_step
        f(self.handle, n_moves, counter0, st, lg, self.stream)
        self.version += 1
        stats = _struct_from_device(st, STATS_DTYPE)[0]
        lgs = _struct_from_device(lg, LOG_DTYPE)[:n_moves] if log else None
        return stats, lgs

    # --------------------------------------------------------------- energy
    def total_energy(self, all_pairs=False, per_particle=False):
        U = torch.zeros(2, dtype=torch.float64, device=self.device)
        n = self.n
        e = torch.zeros(max(n, 1), dtype=torch.float64, device=self.device) if per_particle else None
        _lib.gcmc_total_energy(self.handle, 1 if all_pairs else 0, U, e, self.stream)
        u = U.cpu().numpy()
        out = {"U_pair": float(u[0]), "U_tail": float(u[1])}
        if per_particle:
            out["e"] = e[:n].cpu().numpy()
        return out

    def backward(self, positions=True, params=True):
        n = self.n
        g = torch.zeros(3 * max(n, 1), dtype=torch.float64, device=self.device) if positions else None
        de = torch.zeros(self.ns * self.ns, dtype=torch.float64, device=self.device) if params else None
        ds = torch.zeros(self.ns * self.ns, dtype=torch.float64, device=self.device) if params else None
        _lib.gcmc_backward(self.handle, g, de, ds, self.stream)
        out = {}
        if positions:
            out["grad"] = g[: 3 * n].view(3, n).t().cpu().numpy()
        if params:
            out["d_eps"] = de.view(self.ns, self.ns).cpu().numpy()
            out["d_sigma"] = ds.view(self.ns, self.ns).cpu().numpy()
        return out

    def virial(self):
        """{"W": pair virial, "P": pressure with the ideal and tail terms}; also sets the
        running virial the chain keeps current."""
        out = torch.zeros(2, dtype=torch.float64, device=self.device)
        _lib.gcmc_virial(self.handle, out, self.stream)
        v = out.cpu().numpy()
        return {"W": float(v[0]), "P": float(v[1])}

    # ----------------------------------------------------------- inspection
    @property
    def n(self):
        return int(_lib.gcmc_export_state(self.handle, stream=self.stream).n)

    def checkpoint(self):
        """The box's checkpoint fields (no particles) as a dict."""
        ck = _lib.gcmc_export_state(self.handle, stream=self.stream)
        return checkpoint_dict(ck)

    def particles(self):
        n = self.n
        x = torch.zeros(max(n, 1), dtype=torch.float64, device=self.device)
        y, z = torch.zeros_like(x), torch.zeros_like(x)
        sp = torch.zeros(max(n, 1), dtype=torch.int32, device=self.device)
        n = _lib.gcmc_get_particles(self.handle, x, y, z, sp, self.stream)
        pos = torch.stack([x[:n], y[:n], z[:n]], dim=1).cpu().numpy()
        return pos, sp[:n].cpu().numpy()

    def cells(self):
        info = self.info()
        n = self.n
        cell_of = torch.zeros(max(n, 1), dtype=torch.int32, device=self.device)
        count = torch.zeros(info["n_cells"], dtype=torch.int32, device=self.device)
        ids = torch.zeros(info["n_cells"] * info["cell_cap"], dtype=torch.int32, device=self.device)
        _lib.gcmc_get_cells(self.handle, cell_of, count, ids, self.stream)
        return (cell_of[:n].cpu().numpy(), count.cpu().numpy(),
                ids.view(info["n_cells"], info["cell_cap"]).cpu().numpy())

    def neighbor_ids(self, points, exclude=None, max_ids=4096):
        points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
        m = len(points)
        pts = _dev(points.T.reshape(-1), torch.float64, self.device)
        ex = _dev(np.full(m, -1) if exclude is None else exclude, torch.int32, self.device)
        ids = torch.zeros(max(1, m * max_ids), dtype=torch.int32, device=self.device)
        cnt = torch.zeros(max(m, 1), dtype=torch.int32, device=self.device)
        _lib.gcmc_neighbor_ids(self.handle, pts, ex, m, max_ids, ids, cnt, self.stream)
        ids = ids.cpu().numpy().reshape(max(m, 1), max_ids)
        cnt = cnt.cpu().numpy()
        return [np.sort(ids[i, : min(cnt[i], max_ids)]) for i in range(m)], cnt[:m]

    def export_state(self):
        """A complete checkpoint: (positions (N, 3), species (N,), checkpoint dict)."""
        cap = max(self.max_n, 1)
        x = torch.zeros(cap, dtype=torch.float64, device=self.device)
        y, z = torch.zeros_like(x), torch.zeros_like(x)
        sp = torch.zeros(cap, dtype=torch.int32, device=self.device)
        ck = _lib.gcmc_export_state(self.handle, x, y, z, sp, cap, self.stream)
        n = int(ck.n)
        pos = torch.stack([x[:n], y[:n], z[:n]], dim=1).cpu().numpy()
        return pos, sp[:n].cpu().numpy(), checkpoint_dict(ck)

    def import_state(self, pos, ck, species=None):
        """Restore a checkpoint taken by export_state (ck: its dict)."""
        pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        if pos.shape[0] != int(ck["n"]):
            raise ValueError("the checkpoint holds %d particles, pos has %d" % (int(ck["n"]), pos.shape[0]))
        x = _dev(pos[:, 0], torch.float64, self.device)
        y = _dev(pos[:, 1], torch.float64, self.device)
        z = _dev(pos[:, 2], torch.float64, self.device)
        sp = None if species is None else _dev(species, torch.int32, self.device)
        _lib.gcmc_import_state(self.handle, x, y, z, sp, checkpoint_struct(ck), self.stream)
        self.version += 1

    def snapshot(self):
        """A checkpoint held in device memory: (x, y, z, species, checkpoint dict)."""
        cap = max(self.max_n, 1)
        x = torch.empty(cap, dtype=torch.float64, device=self.device)
        y, z = torch.empty_like(x), torch.empty_like(x)
        sp = torch.empty(cap, dtype=torch.int32, device=self.device)
        ck = _lib.gcmc_export_state(self.handle, x, y, z, sp, cap, self.stream)
        return x, y, z, sp, checkpoint_dict(ck)

    def restore(self, snap):
        """Put a snapshot back (positions, energies, move counter, sums)."""
        x, y, z, sp, ck = snap
        _lib.gcmc_import_state(self.handle, x, y, z, sp, checkpoint_struct(ck), self.stream)
        self.version += 1

    def clear_averages(self):
        _lib.gcmc_clear_averages(self.handle, self.stream)

    def set_positions(self, pos):
        pos = np.asarray(pos, dtype=np.float64)
        n = self.n
        if pos.shape != (n, 3):
            raise ValueError("positions must have shape (%d, 3), got %s" % (n, pos.shape))
        x = _dev(pos[:, 0], torch.float64, self.device)
        y = _dev(pos[:, 1], torch.float64, self.device)
        z = _dev(pos[:, 2], torch.float64, self.device)
        _lib.gcmc_set_positions(self.handle, x, y, z, n, self.stream)
        self.version += 1

    def rescale(self, L_new):
        """Scale the box to edges L_new (coordinates scaled with it), rebuild the
        cell list and return the cell-list energies {"U_pair", "U_tail"} at the
        new volume and {"U_pair_old", "U_tail_old"} at the old one."""
        out = torch.zeros(4, dtype=torch.float64, device=self.device)
        _lib.gcmc_box_rescale(self.handle, L_new, out, self.stream)
        self.version += 1
        self.L = np.broadcast_to(np.asarray(L_new, dtype=np.float64), (3,)).copy()
        v = out.cpu().numpy()
        return {"U_pair": float(v[0]), "U_tail": float(v[1]), "U_pair_old": float(v[2]), "U_tail_old": float(v[3])}

    def set_params(self, eps, sigma):
        _lib.gcmc_set_params(self.handle, np.asarray(eps, dtype=np.float64), np.asarray(sigma, dtype=np.float64))
        self.version += 1

    def set_positions_device(self, pos: torch.Tensor, n=None):
        """pos: (N, 3) float64 device tensor with the current N (n: that N, if the caller knows it)."""
        n = self.n if n is None else int(n)
        if tuple(pos.shape) != (n, 3):
            raise ValueError("positions must have shape (%d, 3), got %s" % (n, tuple(pos.shape)))
        if pos.dtype != torch.float64 or not pos.is_cuda:
            raise TypeError("positions must be a float64 device tensor")
        x, y, z = (pos[:, a].contiguous() for a in range(3))
        _lib.gcmc_set_positions(self.handle, x, y, z, n, self.stream)
        self.version += 1

    def total_energy_device(self, all_pairs=False):
        """(U_pair, U_tail) as a device tensor, no host synchronisation."""
        U = torch.empty(2, dtype=torch.float64, device=self.device)
        _lib.gcmc_total_energy(self.handle, 1 if all_pairs else 0, U, None, self.stream)
        return U

    def backward_device(self, n):
        """(dU/dpos (n,3), dU/deps (ns,ns), dU/dsigma (ns,ns)) as device tensors."""
        g = torch.empty(3 * max(n, 1), dtype=torch.float64, device=self.device)
        de = torch.empty(self.ns * self.ns, dtype=torch.float64, device=self.device)
        ds = torch.empty_like(de)
        _lib.gcmc_backward(self.handle, g, de, ds, self.stream)
        return g[: 3 * n].view(3, n).t(), de.view(self.ns, self.ns), ds.view(self.ns, self.ns)

    def cell_build(self, new_cap=0):
        _lib.gcmc_cell_build(self.handle, new_cap, self.stream)

    def sync(self):
        rc = _lib.gcmc_sync_status(self.handle)
        if rc:
            raise _lib.GcmcError(rc, _lib.gcmc_last_error())

    def status(self):
        return _lib.gcmc_sync_status(self.handle)


def checkpoint_dict(ck) -> dict:
    return {"n": int(ck.n), "u_pair": float(ck.u_pair), "w_pair": float(ck.w_pair), "counter": int(ck.counter),
            "moves": int(ck.moves), "attempts": [int(v) for v in ck.attempts],
            "accepts": [int(v) for v in ck.accepts], "sum_n": float(ck.sum_n), "sum_n2": float(ck.sum_n2),
            "sum_u": float(ck.sum_u), "sum_w": float(ck.sum_w), "error": int(ck.error),
            "error_move": int(ck.error_move)}


def checkpoint_struct(d: dict):
    ck = _lib.Checkpoint()
    for k in ("n", "counter", "moves", "error", "error_move"):
        setattr(ck, k, int(d[k]))
    for k in ("u_pair", "w_pair", "sum_n", "sum_n2", "sum_u", "sum_w"):
        setattr(ck, k, float(d[k]))
    for t in range(3):
        ck.attempts[t] = int(d["attempts"][t])
        ck.accepts[t] = int(d["accepts"][t])
    return ck


class Batch:
    """Many boxes advanced together by one persistent launch."""

    def __init__(self, boxes: Sequence[Box]):
        self.boxes = list(boxes)
        self.device = self.boxes[0].device
        self.handle = _lib.gcmc_batch_create([b.handle for b in self.boxes])

    def step(self, moves_per_box, counter0=0, stream=None):
        st = torch.zeros(len(self.boxes) * STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        _lib.gcmc_batch_step(self.handle, moves_per_box, counter0, st, stream)
        return _struct_from_device(st, STATS_DTYPE)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib.gcmc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_moves(types, index=None, pos=None, species=None) -> np.ndarray:
    types = np.asarray(types, dtype=np.int32)
    m = len(types)
    mv = np.zeros(m, dtype=MOVE_DTYPE)
    mv["type"] = types
    if index is not None:
        mv["index"] = np.asarray(index, dtype=np.int32)
    if pos is not None:
        pos = np.asarray(pos, dtype=np.float64).reshape(m, 3)
        mv["x"], mv["y"], mv["z"] = pos[:, 0], pos[:, 1], pos[:, 2]
    if species is not None:
        mv["species"] = np.asarray(species, dtype=np.int32)
    return mv
