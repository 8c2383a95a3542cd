"""CPU checks of the C ABI library: it loads and exports every entry point
declared in include/fftg.h (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fftg.h")).read()
    return re.findall(r"^(?:fftg_status|const char\*)\s+(\w+)\(", src, re.M)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fftg_create", "fftg_destroy", "fftg_last_error", "fftg_solve",
              "helmholtz_solve", "staggered_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2103_04770_amd import binding
    if not os.path.exists(binding.lib_path()):
        from paper_2103_04770_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(binding.lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_create_rejects_bad_grids_without_touching_the_gpu():
    """Validation happens before any device call."""
    from paper_2103_04770_amd import binding
    lib = binding.load_library()
    bad = [(3, (10, 8, 8)), (3, (8, 7, 8)), (4, (8, 8, 8)), (3, (9, 8, 8)), (2, (512 * 3, 8, 1))]
    codes = []
    for ndim, n in bad:
        g = binding.Grid(ndim, (ctypes.c_int * 3)(*n), 1.0, 0, 0)
        h = ctypes.c_void_p()
        codes.append(lib.fftg_create(ctypes.byref(g), None, ctypes.byref(h)))
        assert not h.value
        assert lib.fftg_last_error(None)
    assert codes == [-2, -2, -1, -2, -2]
