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


def test_footprints_without_a_gpu():
    """Arena footprint of a served request: state (84 B per particle) plus the
    integrator scratch (per particle: 18 B per rung and 48 B of buffers),
    256-byte aligned pieces; bad arguments give -1."""
    from paper_1712_10116_amd import fmm as F
    lib = F.lib()
    for n, L in ((1, 1), (1000, 10), (262144, 10), (1 << 20, 16)):
        run = lib.hhs_run_bytes(n, L)
        fp = lib.serve_footprint(n, L)
        assert run >= (48 + 18 * (L + 1)) * n and run % 256 == 0
        assert fp - run >= 84 * n and (fp - run) - 84 * n <= 8 * 256
        assert lib.serve_footprint(2 * n, L) >= fp and lib.serve_footprint(2 * n + 4096, L) > fp
    assert lib.hhs_run_bytes(0, 10) == -1 and lib.serve_footprint(10, 0) == -1
    assert lib.serve_footprint(10, 31) == -1
    h = ctypes.c_void_p()
    assert lib.serve_create(None, None, None, ctypes.byref(h)) == F.FMM_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    """Every ctypes mirror of a header struct has the C layout: size and the
    offset of each field, from a small C program compiled against the header."""
    import shutil
    import subprocess
    from paper_1712_10116_amd import fmm as F
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"fmm_params": F._Params, "fmm_request": F.Request, "hhs_state": F.HHSState,
               "hhs_params": F.HHSParams, "fmm_cosmo_params": F.CosmoParams,
               "serve_params": F.ServeParams, "serve_request": F.ServeRequest,
               "serve_result": F.ServeResult}
    lines = ['#include <stddef.h>', '#include <stdio.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
