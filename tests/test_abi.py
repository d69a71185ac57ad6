"""The C-ABI library loads and exports every entry point include/gcmc.h declares
(no compute: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

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


def _header_layout(tmp_path, structs):
    """Sizes and field offsets of the header's structs, printed by a C program
    compiled against include/gcmc.h."""
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "gcmc.h"', "int main(void) {"]
    for name, fields in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f in fields:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        a, b, c = line.split()
        out[(a, b)] = int(c)
    return out


def _dtype_fields(dt):
    return [n for n in dt.names if n != "pad"]


def test_struct_layouts_match_header(tmp_path):
    from paper_1408_3764_amd import _lib
    structs = {"gcmc_move": _dtype_fields(_lib.MOVE_DTYPE), "gcmc_stats": _dtype_fields(_lib.STATS_DTYPE),
               "gcmc_log": _dtype_fields(_lib.LOG_DTYPE),
               "gcmc_box_desc": [f[0] for f in _lib.BoxDesc._fields_],
               "gcmc_box_info": [f[0] for f in _lib.BoxInfo._fields_],
               "gcmc_checkpoint": [f[0] for f in _lib.Checkpoint._fields_]}
    lay = _header_layout(tmp_path, structs)
    for name, dt in (("gcmc_move", _lib.MOVE_DTYPE), ("gcmc_stats", _lib.STATS_DTYPE), ("gcmc_log", _lib.LOG_DTYPE)):
        assert lay[(name, "size")] == dt.itemsize, name
        for f in _dtype_fields(dt):
            assert lay[(name, f)] == dt.fields[f][1], (name, f)
    for name, cls in (("gcmc_box_desc", _lib.BoxDesc), ("gcmc_box_info", _lib.BoxInfo),
                      ("gcmc_checkpoint", _lib.Checkpoint)):
        assert lay[(name, "size")] == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert lay[(name, f[0])] == getattr(cls, f[0]).offset, (name, f[0])


def test_slot_index_range_is_refused_without_a_gpu():
    """Cell slots c * cap + k are 32-bit: a grid whose cells x capacity reach
    2^31 is refused before any device work (GCMC_ERR_INVALID_ARG)."""
    from paper_1408_3764_amd import _lib
    L = _lib.lib()
    eps = (ctypes.c_double * 1)(1.0)
    sig = (ctypes.c_double * 1)(1.0)
    d = _lib.BoxDesc()
    for a in range(3):
        d.L[a] = 1000.0
        d.cell_m[a] = 1000
    d.rc, d.beta, d.lambda3, d.max_disp, d.p_disp = 2.5, 1.0, 1.0, 0.3, 1.0 / 3.0
    d.n_species, d.cell_cap, d.eps, d.sigma, d.max_n = 1, 4, eps, sig, 10
    out = ctypes.c_void_p()
    rc = L.gcmc_box_create(ctypes.byref(d), None, None, None, None, 0, None, ctypes.byref(out))
    assert rc == _lib.GCMC_ERR_INVALID_ARG
    assert "2^31" in _lib.gcmc_last_error()
    assert not out.value


def test_version_string_without_gpu():
    from paper_1408_3764_amd import _lib
    assert _lib.gcmc_version().startswith("gcmc-gfx950")
