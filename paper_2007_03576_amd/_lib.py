"""ctypes loader for libhqr.so (argument marshalling only).

torch is imported before the library is opened so that libhqr.so binds to the
HIP runtime torch already loaded (both carry the soname libamdhip64.so.7);
device pointers and stream handles from torch are then valid in libhqr.
"""
import ctypes
import os

import torch  # noqa: F401  (must precede loading libhqr.so)

from .build import LIB

_lib = None


class HqrParams(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("nw", ctypes.c_int), ("nmin", ctypes.c_int),
                ("nibble", ctypes.c_int), ("kexsh", ctypes.c_int), ("itmax", ctypes.c_int64),
                ("window", ctypes.c_int), ("bulges_per_window", ctypes.c_int),
                ("defl_mode", ctypes.c_int), ("defl_thold", ctypes.c_double),
                ("streams", ctypes.c_int), ("small_shifts", ctypes.c_int),
                ("aed_ns", ctypes.c_int), ("aed_nw", ctypes.c_int), ("aed_nmin", ctypes.c_int),
                ("aed_mode", ctypes.c_int), ("aed_seq_max", ctypes.c_int), ("aed_nibble", ctypes.c_int)]


EXPORTS = ["hqr_set_params", "hqr_get_params", "hqr_schur", "hqr_schur_ex", "hqr_schur_batched",
           "hqr_eig_backward_batched", "hqr_last_stats", "hqr_finalize", "hqr_profile_enable",
           "hqr_profile_reset", "hqr_profile_read", "hqr_profile_ticks", "hqr_set_batched_launch",
           "hqr_get_batched_launch", "hqr_schur_batched_noalloc", "hqr_hessenberg",
           "hqr_eigenvectors", "hqr_set_batched_table", "hqr_get_batched_table", "hqr_qz_batched"]


class HqrError(RuntimeError):
    pass


def lib():
    """Open libhqr.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise HqrError(f"{LIB} is missing: build it first (python -m paper_2007_03576_amd.build "
                       "or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.hqr_set_params.argtypes = [ctypes.POINTER(HqrParams)]
    L.hqr_get_params.argtypes = [ctypes.POINTER(HqrParams)]
    L.hqr_schur.argtypes = [vp, vp, i64, i64, vp, vp, vp]
    L.hqr_schur_ex.argtypes = [vp, vp, i64, i64, vp, vp, vp, ctypes.POINTER(HqrParams)]
    L.hqr_hessenberg.argtypes = [vp, vp, i64, i64, vp]
    L.hqr_eigenvectors.argtypes = [vp, vp, i64, i64, vp, vp, vp, i64, vp]
    L.hqr_schur_batched.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp]
    L.hqr_schur_batched_noalloc.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp]
    L.hqr_qz_batched.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
    L.hqr_set_batched_launch.argtypes = [i32, i32]
    ip = ctypes.POINTER(ctypes.c_int32)
    L.hqr_set_batched_table.argtypes = [i32, ip, ip, ip]
    L.hqr_get_batched_table.argtypes = [ip, ip, ip, ip]
    L.hqr_get_batched_launch.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.hqr_eig_backward_batched.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, i32, vp]
    L.hqr_last_stats.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    L.hqr_finalize.argtypes = []
    L.hqr_profile_enable.argtypes = [ctypes.c_int]
    L.hqr_profile_reset.argtypes = []
    dp = ctypes.POINTER(ctypes.c_double)
    L.hqr_profile_read.argtypes = [dp, ctypes.POINTER(ctypes.c_int64), dp, dp, ctypes.c_int]
    L.hqr_profile_ticks.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    for name in EXPORTS:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return _lib


def check(rc: int, what: str) -> int:
    if rc < 0:
        raise HqrError(f"{what} failed with code {rc}")
    return rc
