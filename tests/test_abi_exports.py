"""The C-ABI library loads and exports every function include/dda.h declares (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dda.h")
LIB = os.path.join(ROOT, "paper_0704_0037_amd", "libdda_mi355x.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dda_[a-z0-9_]+)\s*\(", text)))


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_0704_0037_amd import build
        build.build(verbose=False)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("dda_setup", "dda_matvec", "dda_solve", "dda_cross_sections", "dda_mueller", "dda_free"):
        assert must in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_0704_0037_amd import dda
    assert sorted(dda._SIGS) == _declared()


def test_host_only_entry_points_without_a_gpu():
    _ensure_built()
    from paper_0704_0037_amd import dda
    L = dda.lib()
    assert L.dda_strerror(dda.EBREAKDOWN) == b"Krylov breakdown"
    assert L.dda_num_dipoles(None) == -1
    assert L.dda_free(None) == 0
    # invalid arguments are rejected before any device call
    h = ctypes.c_void_p()
    grid = (ctypes.c_int32 * 3)(0, 4, 4)
    m = (ctypes.c_double * 2)(1.5, 0.0)
    assert L.dda_setup(ctypes.byref(h), grid, None, m, 0.4, 0, None, None) == dda.EINVAL
    assert h.value is None


def test_binding_structs_match_the_header_layout(tmp_path):
    # compile a probe against include/dda.h with the host C compiler and compare every struct's
    # size and field offsets with the ctypes mirrors of the binding
    import shutil
    import subprocess
    import pytest
    from paper_0704_0037_amd import dda
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"dda_beam": dda.Beam, "dda_setup_opts": dda.SetupOpts, "dda_solve_opts": dda.SolveOpts,
               "dda_solve_info": dda.SolveInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dda.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_last_error_describes_the_latest_call_only():
    # no GPU work: a NULL context fails argument checking, and dda_free(NULL) succeeds
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    lib.dda_last_error.restype = ctypes.c_char_p
    lib.dda_padded_grid.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.dda_free.argtypes = [ctypes.c_void_p]
    out = (ctypes.c_int32 * 3)()
    assert lib.dda_padded_grid(None, out) == -1
    assert b"dda_padded_grid" in lib.dda_last_error()
    assert lib.dda_free(None) == 0
    assert lib.dda_last_error() == b""


def test_newer_entry_points_check_arguments_without_a_gpu():
    # every check below fails before any device call
    _ensure_built()
    from paper_0704_0037_amd import dda
    L = dda.lib()
    L.dda_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    grid = (ctypes.c_int32 * 3)(2, 2, 2)
    m = (ctypes.c_double * 4)(1.5, 0.0, 1.2, 0.0)
    mask = (ctypes.c_uint8 * 8)(1, 2, 3, 0, 1, 1, 2, 2)  # value 3 names no material
    assert L.dda_setup_materials(ctypes.byref(h), grid, mask, 2, m, 0.4, 0, None, None) == dda.EINVAL
    assert h.value is None and b"n_mat" in L.dda_last_error()
    assert L.dda_setup_materials(ctypes.byref(h), grid, None, 2, m, 0.4, 0, None, None) == dda.EINVAL
    assert L.dda_setup_materials(ctypes.byref(h), grid, mask, 0, m, 0.4, 0, None, None) == dda.EINVAL
    out = (ctypes.c_double * 5)()
    n = ctypes.c_int32()
    assert L.dda_orientation_average_adaptive(None, 1e-3, 2, 4, 2, 1e-5, None, out, ctypes.byref(n)) == dda.EINVAL
    th = (ctypes.c_double * 1)(0.5)
    M = (ctypes.c_double * 16)()
    assert L.dda_orientation_average_mueller(None, 2, 2, 4, 1e-5, None, th, 1, M, None) == dda.EINVAL
    assert L.dda_checkpoint_save(None, None, b"/nonexistent/ckpt") == dda.EINVAL
    assert L.dda_checkpoint_load(None, None, b"/nonexistent/ckpt") == dda.EINVAL
    assert b"dda_checkpoint_load" in L.dda_last_error()
    # the padded-grid tuner and the no-allocation product refuse bad arguments before any device call
    pad = (ctypes.c_int32 * 3)()
    assert L.dda_tune_padding(grid, mask, m, 0.4, 0, 1, 3, 0, pad, None) == dda.EINVAL  # n_cand < 1
    assert L.dda_tune_padding(grid, None, m, 0.4, 0, 1, 3, 2, pad, None) == dda.EINVAL
    assert b"dda_tune_padding" in L.dda_last_error()
    assert L.dda_matvec_noalloc(None, None, None, None) == dda.EINVAL
    assert b"dda_matvec_noalloc" in L.dda_last_error()
