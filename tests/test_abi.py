"""The C ABI library loads on a machine without a GPU and exports every
function include/stn.h declares; host-only calls behave as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2605_29514_amd import stn as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "stn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stn_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libstn.so not built (run __graft_entry__.build())")
    return B.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(B.EXPORTS) <= set(names)


def cfg(n=17, S=100, chi=64, prec=B.STN_FP64, eps=1e-16):
    return B.StnConfig(n, S, chi, prec, eps, None)


def test_workspace_bytes(lib):
    c64 = cfg(prec=B.STN_FP64)
    c32 = cfg(prec=B.STN_FP32)
    b64 = lib.stn_workspace_bytes(ctypes.byref(c64))
    b32 = lib.stn_workspace_bytes(ctypes.byref(c32))
    assert b64 > b32 > 0
    assert b64 % 256 == 0
    big = lib.stn_workspace_bytes(ctypes.byref(cfg(n=49, S=1024, chi=256, prec=B.STN_FP32)))
    # the d=5 chi 256 bench context (238 GiB, its environment store included)
    # leaves room on one 288 GB device next to the runtime's own allocations
    assert 50e9 < big < 265e9
    for bad in (cfg(n=0), cfg(S=0), cfg(chi=0), cfg(prec=7), cfg(eps=-1.0), cfg(chi=4096)):
        assert lib.stn_workspace_bytes(ctypes.byref(bad)) == 0


def test_init_rejects_bad_arguments(lib):
    c = cfg()
    ctx = ctypes.c_void_p()
    assert lib.stn_init(ctypes.byref(ctx), ctypes.byref(c), None, 0) == -1
    assert lib.stn_init(ctypes.byref(ctx), ctypes.byref(c), ctypes.c_void_p(256), 10) == -2
    assert lib.stn_init(ctypes.byref(ctx), ctypes.byref(c), ctypes.c_void_p(257), 1 << 40) == -1


def test_pack_roundtrip():
    rng = np.random.default_rng(0)
    m = rng.random((130, 7)) < 0.3
    w = B.pack_shots(m)
    assert w.shape == (7, 3)
    assert np.array_equal(B.unpack_shots(w, 130).T, m)
