"""The C-ABI library loads and exports every entry point include/gcmc.h declares
(no compute: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gcmc.h")
LIB = os.path.join(ROOT, "paper_1408_3764_amd", "libgcmc.so")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(gcmc_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("gcmc_box_create", "gcmc_delta_energy", "gcmc_commit", "gcmc_step", "gcmc_total_energy",
              "gcmc_backward", "gcmc_batch_step", "gcmc_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libgcmc.so is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1408_3764_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_symbols()
    for s in _lib.EXPORTS:
        assert hasattr(_lib, s)


def test_struct_layouts_match_header():
    from paper_1408_3764_amd import _lib
    assert ctypes.sizeof(_lib.BoxDesc) == 128
    assert _lib.MOVE_DTYPE.itemsize == 40
    assert _lib.STATS_DTYPE.itemsize == 144
    assert _lib.LOG_DTYPE.itemsize == 64


def test_version_string_without_gpu():
    from paper_1408_3764_amd import _lib
    assert _lib.gcmc_version().startswith("gcmc-gfx950")
