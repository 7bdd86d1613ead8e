"""C-ABI checks that need no GPU: libhqr.so loads and exports every entry point
declared in include/hqr.h, and argument validation returns the documented
codes before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hqr.h")).read()
    return sorted(set(re.findall(r"^\s*int\s+(hqr_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2007_03576_amd._lib import lib
    return lib()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["hqr_schur", "hqr_schur_batched", "hqr_eig_backward_batched", "hqr_set_params"]:
        assert s in syms


def test_library_exports_every_declared_symbol(L):
    for s in declared_symbols():
        assert hasattr(L, s), f"libhqr.so does not export {s}"


def test_argument_validation_without_device_work(L):
    buf = (ctypes.c_double * 4)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.hqr_schur(p, None, -1, 1, p, p, None) == -3
    assert L.hqr_schur(None, None, 2, 2, p, p, None) == -1
    assert L.hqr_schur(p, None, 3, 2, p, p, None) == -4
    assert L.hqr_schur(p, None, 2, 2, None, p, None) == -5
    assert L.hqr_schur(p, None, 2, 2, p, None, None) == -6
    assert L.hqr_schur(p, None, 0, 1, p, p, None) == 0
    assert L.hqr_schur_batched(p, None, p, p, -1, p, p, p, p, None) == -5
    assert L.hqr_eig_backward_batched(p, p, p, p, -2, p, p, p, p, p, 1, None) == -5
    assert L.hqr_eig_backward_batched(p, p, None, p, 1, p, p, p, p, p, 1, None) == -3
    assert L.hqr_eig_backward_batched(p, p, p, None, 1, p, p, p, p, p, 1, None) == -4
    assert L.hqr_eig_backward_batched(p, p, p, p, 1, p, p, p, p, None, 1, None) == -10
    assert L.hqr_eig_backward_batched(p, p, p, p, 0, p, p, p, p, p, 1, None) == 0


def test_params_roundtrip_and_rejection(L):
    from paper_2007_03576_amd._lib import HqrParams
    old = HqrParams()
    assert L.hqr_get_params(ctypes.byref(old)) == 0
    hp = HqrParams()
    hp.ns, hp.nw, hp.nmin = 64, 256, 60
    assert L.hqr_set_params(ctypes.byref(hp)) == 0
    got = HqrParams()
    assert L.hqr_get_params(ctypes.byref(got)) == 0
    assert (got.ns, got.nw, got.nmin) == (64, 256, 60)
    # deflation conditions: 0 LAPACK-style, 1 norm-stable, 2 fixed with a finite threshold >= 0
    for mode, thold, rc in [(1, 0.0, 0), (2, 1e-12, 0), (2, 0.0, 0), (2, -1.0, -1), (2, float("inf"), -1),
                            (2, float("nan"), -1), (3, 0.0, -1), (-1, 0.0, -1)]:
        hp = HqrParams()
        hp.defl_mode, hp.defl_thold = mode, thold
        assert L.hqr_set_params(ctypes.byref(hp)) == rc, (mode, thold)
    # large-window AED mode: 0 adaptive, 1 sequential, 2 parallel; a window limit >= 0
    for mode, lim, rc in [(0, 0, 0), (1, 256, 0), (2, 0, 0), (3, 0, -1), (-1, 0, -1), (1, -5, -1)]:
        hp = HqrParams()
        hp.aed_mode, hp.aed_seq_max = mode, lim
        assert L.hqr_set_params(ctypes.byref(hp)) == rc, (mode, lim)
    assert L.hqr_set_params(ctypes.byref(old)) == 0
    assert L.hqr_set_params(None) == -1



def test_batched_launch_roundtrip_and_rejection(L):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    assert L.hqr_get_batched_launch(ctypes.byref(a), ctypes.byref(b)) == 0
    old = (a.value, b.value)
    assert old == (2, 320)
    assert L.hqr_set_batched_launch(3, 400) == 0
    assert L.hqr_get_batched_launch(ctypes.byref(a), ctypes.byref(b)) == 0
    assert (a.value, b.value) == (3, 400)
    assert L.hqr_set_batched_launch(0, 400) == -1
    assert L.hqr_set_batched_launch(9, 400) == -1
    assert L.hqr_set_batched_launch(2, 95) == -2
    assert L.hqr_set_batched_launch(2, 4096) == -2
    assert L.hqr_get_batched_launch(None, ctypes.byref(b)) == -1
    assert L.hqr_set_batched_launch(*old) == 0
