"""The C-ABI library loads and exports every entry point the header declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sarabande_hip.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["sb_plan_create", "sb_plan_workspace", "sb_plan_bind", "sb_prepare", "sb_forward",
              "sb_backward", "sb_zeta_size", "sb_zeta_index", "sb_bin_counts", "sb_autotune",
              "sb_forward_graph", "sb_plan_destroy", "sb_status_str", "sb_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2210_10206_amd import _lib
    lib = _lib.load()
    for n in declared_functions():
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, n


def _problem(ndim=3, npcf=3, edges=(0.0, 2.0, 4.0), lmax=2, prec=0, dtype=0, flags=0):
    from paper_2210_10206_amd import _lib
    import numpy as np
    e = np.asarray(edges, dtype=np.float64)
    p = _lib.SbProblem(ndim, npcf, len(e) - 1, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), lmax, prec, dtype,
                       flags)
    return p, e


@pytest.mark.parametrize("kw,shape,expect", [
    (dict(ndim=4), (16, 16, 16), -1),
    (dict(npcf=5), (16, 16, 16), -1),
    (dict(edges=(0.0, 3.0, 2.0)), (16, 16, 16), -1),
    (dict(edges=(-1.0, 3.0)), (16, 16, 16), -1),
    (dict(lmax=-1), (16, 16, 16), -1),
    (dict(lmax=11), (16, 16, 16), -1),
    (dict(prec=7), (16, 16, 16), -1),
    (dict(), (16, 16, 0), -1),
    (dict(), (16, 16, 14), -2),          # 14 = 2 * 7: no radix-7 pass
    (dict(npcf=4, edges=tuple(range(12))), (16, 16, 16), -2),
    (dict(flags=8), (16, 16, 16), -1),                # odd parity is a full-4PCF option
    (dict(ndim=2, npcf=4, flags=8), (16, 16, 16), -1),
])
def test_argument_validation_without_gpu(kw, shape, expect):
    """Argument errors are reported before any device call, so they can be checked on a CPU host."""
    from paper_2210_10206_amd import _lib
    import numpy as np
    lib = _lib.load()
    prob, e = _problem(**kw)
    sh = np.array(shape[:prob.ndim] if prob.ndim in (2, 3) else shape, dtype=np.int64)
    out = ctypes.c_void_p()
    rc = lib.sb_plan_create(ctypes.byref(prob), 1, sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(out))
    assert rc == expect
    assert not out.value
    assert len(lib.sb_last_error()) > 0


def test_status_strings():
    from paper_2210_10206_amd import _lib
    lib = _lib.load()
    for s in range(-6, 1):
        assert lib.sb_status_str(s)
    assert lib.sb_version() >= 1
