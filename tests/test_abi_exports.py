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
