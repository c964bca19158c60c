"""Host-side checks of the C ABI: the library loads, exports every entry point that
include/fifa_gp.h declares, and rejects bad arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fifa_gp.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:fg_status|void|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)
    return names


@pytest.fixture(scope="module")
def L():
    from paper_2006_06537_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2006_06537_amd import build_lib
        build_lib.build(verbose=False)
    return _lib.lib()


def test_header_declares_the_hot_path():
    names = _declared()
    for must in ["hodlr_build", "hodlr_factor", "hodlr_solve", "hodlr_logdet", "gp_draw_f",
                 "gibbs_step"]:
        assert must in names


def test_every_declared_symbol_is_exported(L):
    from paper_2006_06537_amd import _lib
    names = _declared()
    assert sorted(names) == sorted(_lib.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_argument_errors_without_device(L):
    from paper_2006_06537_amd import _lib
    out = C.c_void_p()
    k = _lib.Kernel(0, 0.1, 1e-6)
    assert L.hodlr_build(None, 10, k, 64, 1e-10, None, C.byref(out)) == _lib.FG_EINVAL
    assert b"NULL" in L.fg_last_error()
    assert L.hodlr_build(C.c_void_p(8), 0, k, 64, 1e-10, None, C.byref(out)) == _lib.FG_EINVAL
    assert L.hodlr_build(C.c_void_p(8), 10, k, 64, 1e-10, None, None) == _lib.FG_EINVAL
    f = C.c_void_p()
    assert L.hodlr_factor(None, 1.0, 0.0, None, None, C.byref(f)) == _lib.FG_EINVAL
    assert L.hodlr_solve(None, None, None, 1, 10, None) == _lib.FG_EINVAL
    assert L.fg_normals(0, 0, 0, 0, -1, None, None) == _lib.FG_EINVAL
    cfg = _lib.ChainCfg(0, 0.1, 1e-6, 64, 1e-10, 1.0, 1.0, 1, 1, 1, 1, 0, 0, 0, 0)
    ch = C.c_void_p()
    assert L.gibbs_chain_create(C.byref(cfg), C.c_void_p(8), C.c_void_p(8), 10, None,
                                C.byref(ch)) == _lib.FG_EINVAL
    assert b"grid" in L.fg_last_error()


def test_footprint_estimate_host_only():
    """fg_footprint_bytes plans on the host only (no device call): positive, growing
    with n, and larger for a mixed-precision chain, which holds the PCG workspace and keeps
    room for the FP64 factor of M~ it falls back to when the FP32 one fails."""
    import numpy as np
    import paper_2006_06537_amd as fg
    from workloads import sinusoid_1d
    sizes = []
    for n in (2000, 8000, 32000):
        x, _ = sinusoid_1d(n, seed=2)
        sizes.append(fg.footprint_bytes(x, 0.05, leaf=128))
    assert 0 < sizes[0] < sizes[1] < sizes[2]
    assert sizes[2] / sizes[1] > 3.0  # at least linear in n
    x, _ = sinusoid_1d(8000, seed=2)
    assert fg.footprint_bytes(x, 0.05, precision=fg.MIXED) > sizes[1]
    with pytest.raises(fg.FgError):
        fg.footprint_bytes(x, 0.05, leaf=1)
