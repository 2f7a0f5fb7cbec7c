"""The C-ABI library loads and exports every entry point its header declares
(no GPU calls), and the host-side argument checks reject bad input before
any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmm355.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:fmm_status|const char \*|int64_t)\s*(\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("fmm_create", "fmm_build", "fmm_evaluate", "fmm_forces", "hhs_step", "hhs_init",
                 "fmm_export_tree", "fmm_tree_info", "fmm_invariants", "fmm_destroy",
                 "fmm_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_1712_10116_amd import fmm as F
    lib = F.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(F.EXPORTED) == sorted(_declared())


def test_create_rejects_bad_parameters_without_a_gpu():
    from paper_1712_10116_amd import fmm as F
    lib = F.lib()
    h = ctypes.c_void_p()
    for prm in ((0, 16, 0, 0), (9, 16, 0, 0), (4, 0, 0, 0), (4, 16, 7, 0), (4, 16, 0, 5)):
        p = F._Params(*prm)
        assert lib.fmm_create(ctypes.byref(p), 1000, None, ctypes.byref(h)) == F.FMM_EINVAL
    p = F._Params(4, 16, 0, 0)
    assert lib.fmm_create(ctypes.byref(p), 0, None, ctypes.byref(h)) == F.FMM_EINVAL
    assert lib.fmm_create(None, 10, None, ctypes.byref(h)) == F.FMM_EINVAL
    assert lib.fmm_destroy(None) == F.FMM_EINVAL
    assert lib.fmm_build(None, None, 0, None, 0, 0.0, 0.5) == F.FMM_EINVAL
