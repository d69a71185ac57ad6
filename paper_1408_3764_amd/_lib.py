"""ctypes binding of ``libgcmc.so`` (the C ABI declared in ``include/gcmc.h``).

Argument marshalling only: every function here has the name of the C entry
point it calls, takes device buffers as torch CUDA tensors (pointers are passed
through ``data_ptr()``) and the stream as a ``torch.cuda.Stream`` (or the
current stream).  There is no CPU fallback: if the library is not built,
:func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgcmc.so")

GCMC_OK = 0
ERRORS = {
    1: "GCMC_ERR_INVALID_ARG", 2: "GCMC_ERR_OOM", 3: "GCMC_ERR_CELL_OVERFLOW", 4: "GCMC_ERR_CAPACITY",
    5: "GCMC_ERR_HIP", 6: "GCMC_ERR_POISONED", 7: "GCMC_ERR_UNSUPPORTED", 8: "GCMC_ERR_INTERNAL",
}
GCMC_ERR_INVALID_ARG, GCMC_ERR_OOM, GCMC_ERR_CELL_OVERFLOW, GCMC_ERR_CAPACITY = 1, 2, 3, 4
GCMC_ERR_HIP, GCMC_ERR_POISONED, GCMC_ERR_UNSUPPORTED, GCMC_ERR_INTERNAL = 5, 6, 7, 8
DISPLACE, INSERT, DELETE = 0, 1, 2
COUNTER_CONTINUE = 0xFFFFFFFFFFFFFFFF
MAX_SPECIES = 4

# every symbol include/gcmc.h declares
EXPORTS = [
    "gcmc_box_create", "gcmc_box_destroy", "gcmc_box_get_info", "gcmc_cell_build", "gcmc_set_positions",
    "gcmc_set_params", "gcmc_box_rescale",
    "gcmc_delta_energy", "gcmc_delta_energy_allpairs", "gcmc_commit", "gcmc_box_set_launch", "gcmc_box_set_wait_limit", "gcmc_step",
    "gcmc_step_allpairs", "gcmc_total_energy", "gcmc_total_energy_noalloc", "gcmc_backward", "gcmc_virial",
    "gcmc_batch_create",
    "gcmc_batch_destroy",
    "gcmc_batch_step", "gcmc_get_particles", "gcmc_get_cells", "gcmc_neighbor_ids", "gcmc_export_state",
    "gcmc_import_state", "gcmc_clear_averages", "gcmc_sync_status", "gcmc_last_error", "gcmc_version",
]


class GcmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, str(code)), msg))
        self.code = code


class BoxDesc(C.Structure):
    _fields_ = [
        ("L", C.c_double * 3), ("rc", C.c_double), ("beta", C.c_double), ("mu", C.c_double),
        ("lambda3", C.c_double), ("max_disp", C.c_double), ("p_disp", C.c_double),
        ("n_species", C.c_int32), ("cell_cap", C.c_int32),
        ("eps", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)),
        ("max_n", C.c_int64), ("cell_m", C.c_int32 * 3), ("box_id", C.c_uint32), ("seed", C.c_uint64),
    ]


class BoxInfo(C.Structure):
    _fields_ = [
        ("cell_m", C.c_int32 * 3), ("span", C.c_int32 * 3), ("cell_cap", C.c_int32), ("n_species", C.c_int32),
        ("n_cells", C.c_int64), ("max_n", C.c_int64), ("inv_s", C.c_double * 3),
        ("n_stencil", C.c_int32), ("pad", C.c_int32),
    ]


MOVE_DTYPE = np.dtype({"names": ["type", "index", "x", "y", "z", "species", "pad"],
                       "formats": [np.int32, np.int32, np.float64, np.float64, np.float64, np.int32, np.int32],
                       "offsets": [0, 4, 8, 16, 24, 32, 36], "itemsize": 40})
STATS_DTYPE = np.dtype({"names": ["attempts", "accepts", "n", "moves_done", "u_pair", "u_tail", "sum_n", "sum_u",
                                  "error", "pad", "error_move", "stencils", "candidates", "pair_evals", "in_cutoff",
                                  "w_pair", "sum_w", "sum_n2", "avg_n", "avg_u", "avg_p"],
                        "formats": [(np.int64, 3), (np.int64, 3), np.int64, np.int64, np.float64, np.float64,
                                    np.float64, np.float64, np.int32, np.int32, np.int64, np.int64, np.int64,
                                    np.int64, np.int64] + [np.float64] * 6,
                        "offsets": [0, 24, 48, 56, 64, 72, 80, 88, 96, 100, 104, 112, 120, 128, 136,
                                    144, 152, 160, 168, 176, 184],
                        "itemsize": 192})
LOG_DTYPE = np.dtype({"names": ["type", "index", "accepted", "flags", "dU_pair", "dU_tail", "x", "y", "z", "arg",
                                "dW_pair"],
                      "formats": [np.int32] * 4 + [np.float64] * 7,
                      "offsets": [0, 4, 8, 12, 16, 24, 32, 40, 48, 56, 64], "itemsize": 72})


class Checkpoint(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("u_pair", C.c_double), ("w_pair", C.c_double), ("counter", C.c_uint64),
        ("moves", C.c_int64), ("attempts", C.c_int64 * 3), ("accepts", C.c_int64 * 3),
        ("sum_n", C.c_double), ("sum_n2", C.c_double), ("sum_u", C.c_double), ("sum_w", C.c_double),
        ("error", C.c_int32), ("pad", C.c_int32), ("error_move", C.c_int64),
    ]

_lib = None


def lib():
    """Load libgcmc.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgcmc.so is not built (run __graft_entry__.build() or "
                          "python paper_1408_3764_amd/build.py); the GPU path has no fallback")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
    sig = {
        "gcmc_box_create": [C.POINTER(BoxDesc), dp, dp, dp, dp, i64, vp, C.POINTER(vp)],
        "gcmc_box_destroy": [vp],
        "gcmc_box_get_info": [vp, C.POINTER(BoxInfo)],
        "gcmc_cell_build": [vp, i32, vp],
        "gcmc_set_positions": [vp, dp, dp, dp, i64, vp],
        "gcmc_set_params": [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "gcmc_box_rescale": [vp, C.POINTER(C.c_double), vp, vp],
        "gcmc_delta_energy": [vp, dp, i64, dp, dp, dp, vp],
        "gcmc_delta_energy_allpairs": [vp, dp, i64, dp, dp, dp, vp],
        "gcmc_commit": [vp, dp, dp, dp, vp],
        "gcmc_box_set_launch": [vp, i32, i32],
        "gcmc_box_set_wait_limit": [vp, i32],
        "gcmc_step": [vp, i64, u64, dp, dp, vp],
        "gcmc_step_allpairs": [vp, i64, u64, dp, dp, vp],
        "gcmc_total_energy": [vp, i32, dp, dp, vp],
        "gcmc_total_energy_noalloc": [vp, i32, dp, dp, vp],
        "gcmc_backward": [vp, dp, dp, dp, vp],
        "gcmc_virial": [vp, dp, vp],
        "gcmc_batch_create": [C.POINTER(vp), i32, C.POINTER(vp)],
        "gcmc_batch_destroy": [vp],
        "gcmc_batch_step": [vp, i64, u64, dp, vp],
        "gcmc_get_particles": [vp, dp, dp, dp, dp, C.POINTER(i64), vp],
        "gcmc_get_cells": [vp, dp, dp, dp, vp],
        "gcmc_neighbor_ids": [vp, dp, dp, i64, i32, dp, dp, vp],
        "gcmc_export_state": [vp, dp, dp, dp, dp, i64, C.POINTER(Checkpoint), vp],
        "gcmc_import_state": [vp, dp, dp, dp, dp, C.POINTER(Checkpoint), vp],
        "gcmc_clear_averages": [vp, vp],
        "gcmc_sync_status": [vp],
        "gcmc_last_error": [],
        "gcmc_version": [],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_char_p if name in ("gcmc_last_error", "gcmc_version") else C.c_int
    _lib = L
    return L


def check(rc):
    if rc != GCMC_OK:
        raise GcmcError(rc, lib().gcmc_last_error().decode())
    return rc


def ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return C.c_void_p(t.data_ptr())


def stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# Thin wrappers with the C names ------------------------------------------------
def gcmc_box_create(desc, x, y, z, species, n, stream=None):
    out = C.c_void_p()
    check(lib().gcmc_box_create(C.byref(desc), ptr(x), ptr(y), ptr(z), ptr(species), int(n), stream_handle(stream),
                                C.byref(out)))
    return out


def gcmc_box_destroy(box):
    check(lib().gcmc_box_destroy(box))


def gcmc_box_get_info(box):
    info = BoxInfo()
    check(lib().gcmc_box_get_info(box, C.byref(info)))
    return info


def gcmc_cell_build(box, new_cap=0, stream=None):
    check(lib().gcmc_cell_build(box, int(new_cap), stream_handle(stream)))


def gcmc_set_positions(box, x, y, z, n, stream=None):
    check(lib().gcmc_set_positions(box, ptr(x), ptr(y), ptr(z), int(n), stream_handle(stream)))


def gcmc_set_params(box, eps, sigma):
    e = np.ascontiguousarray(eps, dtype=np.float64).reshape(-1)
    s = np.ascontiguousarray(sigma, dtype=np.float64).reshape(-1)
    check(lib().gcmc_set_params(box, e.ctypes.data_as(C.POINTER(C.c_double)),
                                s.ctypes.data_as(C.POINTER(C.c_double))))


def gcmc_box_rescale(box, L_new, out, stream=None):
    Lh = np.ascontiguousarray(np.broadcast_to(np.asarray(L_new, dtype=np.float64), (3,)))
    check(lib().gcmc_box_rescale(box, Lh.ctypes.data_as(C.POINTER(C.c_double)), ptr(out), stream_handle(stream)))


def gcmc_delta_energy(box, moves, n, dU_pair, dU_tail, dW_pair=None, stream=None):
    check(lib().gcmc_delta_energy(box, ptr(moves), int(n), ptr(dU_pair), ptr(dU_tail), ptr(dW_pair),
                                  stream_handle(stream)))


def gcmc_delta_energy_allpairs(box, moves, n, dU_pair, dU_tail, dW_pair=None, stream=None):
    check(lib().gcmc_delta_energy_allpairs(box, ptr(moves), int(n), ptr(dU_pair), ptr(dU_tail), ptr(dW_pair),
                                           stream_handle(stream)))


def gcmc_commit(box, move, dU_pair, dW_pair=None, stream=None):
    check(lib().gcmc_commit(box, ptr(move), ptr(dU_pair), ptr(dW_pair), stream_handle(stream)))


def gcmc_box_set_launch(box, waves, rows):
    check(lib().gcmc_box_set_launch(box, int(waves), int(rows)))


def gcmc_box_set_wait_limit(box, polls):
    check(lib().gcmc_box_set_wait_limit(box, int(polls)))


def gcmc_step(box, n_moves, counter0, stats, log, stream=None):
    check(lib().gcmc_step(box, int(n_moves), int(counter0), ptr(stats), ptr(log), stream_handle(stream)))


def gcmc_step_allpairs(box, n_moves, counter0, stats, log, stream=None):
    check(lib().gcmc_step_allpairs(box, int(n_moves), int(counter0), ptr(stats), ptr(log), stream_handle(stream)))


def gcmc_total_energy(box, all_pairs, U, e, stream=None):
    check(lib().gcmc_total_energy(box, int(all_pairs), ptr(U), ptr(e), stream_handle(stream)))


def gcmc_total_energy_noalloc(box, all_pairs, U, e, stream=None):
    check(lib().gcmc_total_energy_noalloc(box, int(all_pairs), ptr(U), ptr(e), stream_handle(stream)))


def gcmc_backward(box, grad, deps, dsig, stream=None):
    check(lib().gcmc_backward(box, ptr(grad), ptr(deps), ptr(dsig), stream_handle(stream)))


def gcmc_virial(box, out, stream=None):
    check(lib().gcmc_virial(box, ptr(out), stream_handle(stream)))


def gcmc_batch_create(boxes):
    arr = (C.c_void_p * len(boxes))(*[b.value for b in boxes])
    out = C.c_void_p()
    check(lib().gcmc_batch_create(arr, len(boxes), C.byref(out)))
    return out


def gcmc_batch_destroy(batch):
    check(lib().gcmc_batch_destroy(batch))


def gcmc_batch_step(batch, moves_per_box, counter0, stats, stream=None):
    check(lib().gcmc_batch_step(batch, int(moves_per_box), int(counter0), ptr(stats), stream_handle(stream)))


def gcmc_get_particles(box, x, y, z, species, stream=None):
    n = C.c_int64()
    check(lib().gcmc_get_particles(box, ptr(x), ptr(y), ptr(z), ptr(species), C.byref(n), stream_handle(stream)))
    return n.value


def gcmc_get_cells(box, cell_of, count, ids, stream=None):
    check(lib().gcmc_get_cells(box, ptr(cell_of), ptr(count), ptr(ids), stream_handle(stream)))


def gcmc_neighbor_ids(box, points, exclude, n, max_ids, ids, counts, stream=None):
    check(lib().gcmc_neighbor_ids(box, ptr(points), ptr(exclude), int(n), int(max_ids), ptr(ids), ptr(counts),
                                  stream_handle(stream)))


def gcmc_export_state(box, x=None, y=None, z=None, species=None, capacity=0, stream=None):
    """Returns the Checkpoint struct; the particles go into the given device tensors."""
    ck = Checkpoint()
    check(lib().gcmc_export_state(box, ptr(x), ptr(y), ptr(z), ptr(species), int(capacity), C.byref(ck),
                                  stream_handle(stream)))
    return ck


def gcmc_import_state(box, x, y, z, species, ck, stream=None):
    check(lib().gcmc_import_state(box, ptr(x), ptr(y), ptr(z), ptr(species), C.byref(ck), stream_handle(stream)))


def gcmc_clear_averages(box, stream=None):
    check(lib().gcmc_clear_averages(box, stream_handle(stream)))


def gcmc_sync_status(box):
    return lib().gcmc_sync_status(box)


def gcmc_last_error():
    return lib().gcmc_last_error().decode()


def gcmc_version():
    return lib().gcmc_version().decode()
