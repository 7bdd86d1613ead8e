"""CPU oracle for the multishift QR algorithm with AED -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use this package.  It wraps ``liboracle.so`` (plain C, see
``hqr_oracle.c``) with numpy marshalling.  Nothing here shares code with the
GPU library.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build_oracle

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.hqr_oracle_schur_ex.argtypes = [dp, dp, i64, i64, dp, dp, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, i64, ctypes.POINTER(ctypes.c_int64)]
        L.hqr_oracle_schur_defl.argtypes = [dp, dp, i64, i64, dp, dp, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, i64, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.c_int, ctypes.c_double]
        L.hqr_oracle_aed_ex.argtypes = [dp, dp, i64, i64, i64, i64, ctypes.c_int, dp, dp,
                                        ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double]
        L.hqr_oracle_swap_rejections.argtypes = [ctypes.c_int]
        L.hqr_oracle_swap_rejections.restype = ctypes.c_int64
        L.hqr_oracle_sweep.argtypes = [dp, dp, i64, i64, i64, i64, ctypes.c_int, dp, dp, ctypes.c_int]
        L.hqr_oracle_swap.argtypes = [dp, dp, i64, i64, i64, ctypes.c_int, ctypes.c_int]
        L.hqr_oracle_std2x2.argtypes = [dp] * 6
        L.hqr_oracle_aed.argtypes = [dp, dp, i64, i64, i64, i64, ctypes.c_int, dp, dp,
                                     ctypes.POINTER(ctypes.c_int)]
        L.hqr_oracle_eig_backward.argtypes = [dp, dp, i64, i64, dp, dp, dp, dp, dp, ctypes.c_int]
        L.hqr_oracle_qz.argtypes = [dp, dp, dp, dp, i64, i64, dp, dp, dp, i64]
        L.hqr_oracle_set_mutation.argtypes = [ctypes.c_int]
        L.hqr_oracle_set_mutation.restype = None
        L.hqr_oracle_force_swap_failure.argtypes = [ctypes.c_int]
        L.hqr_oracle_force_swap_failure.restype = None
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fortran(a):
    return np.array(a, dtype=np.float64, order="F", copy=True)


def set_mutation(m: int) -> None:
    lib().hqr_oracle_set_mutation(int(m))


def force_swap_failure(on: bool) -> None:
    lib().hqr_oracle_force_swap_failure(1 if on else 0)


def swap_rejections(reset=False) -> int:
    """Swaps rejected by the stability test since the last reset."""
    return int(lib().hqr_oracle_swap_rejections(1 if reset else 0))


def schur(H, want_q=True, Q0=None, ns=0, nw=0, nmin=0, itmax=0, defl_mode=0, defl_thold=0.0):
    """Returns (T, Q, w, info, stats); w is complex in diagonal order.
    defl_mode: 0 LAPACK-style, 1 norm-stable, 2 fixed (threshold defl_thold)."""
    T = _fortran(H)
    n = T.shape[0]
    Q = None
    if want_q:
        Q = _fortran(Q0) if Q0 is not None else np.asfortranarray(np.eye(n))
    wr = np.zeros(max(n, 1))
    wi = np.zeros(max(n, 1))
    st = (ctypes.c_int64 * 6)()
    info = lib().hqr_oracle_schur_defl(_p(T), _p(Q), n, max(n, 1), _p(wr), _p(wi), ns, nw, nmin,
                                       itmax, st, int(defl_mode), float(defl_thold))
    return T, Q, (wr + 1j * wi)[:n], info, list(st)


def qz(H, T, want_qz=True, itmax=0):
    """Generalized real Schur form of the Hessenberg-triangular pair (H, T):
    returns (S, Tt, Q, Z, alpha, beta, info) with Q^T H Z = S, Q^T T Z = Tt,
    alpha complex and beta >= 0 in diagonal order (beta = 0: infinite)."""
    S = _fortran(H)
    Tt = _fortran(T)
    n = S.shape[0]
    Q = Z = None
    if want_qz:
        Q = np.asfortranarray(np.eye(n))
        Z = np.asfortranarray(np.eye(n))
    ar = np.zeros(max(n, 1))
    ai = np.zeros(max(n, 1))
    be = np.zeros(max(n, 1))
    info = lib().hqr_oracle_qz(_p(S), _p(Tt), _p(Q), _p(Z), n, max(n, 1), _p(ar), _p(ai), _p(be), int(itmax))
    return S, Tt, Q, Z, (ar + 1j * ai)[:n], be[:n], info


def sweep(H, Q, ktop, kbot, shifts, vigilant=False):
    T = _fortran(H)
    n = T.shape[0]
    Qo = _fortran(Q) if Q is not None else None
    s = np.asarray(shifts, dtype=np.complex128)
    sr = np.ascontiguousarray(s.real)
    si = np.ascontiguousarray(s.imag)
    rc = lib().hqr_oracle_sweep(_p(T), _p(Qo), n, n, ktop, kbot, len(s), _p(sr), _p(si),
                                1 if vigilant else 0)
    if rc != 0:
        raise ValueError(f"hqr_oracle_sweep returned {rc}")
    return T, Qo


def swap(T, Q, j, p, q):
    Tn = _fortran(T)
    n = Tn.shape[0]
    Qo = _fortran(Q) if Q is not None else None
    rc = lib().hqr_oracle_swap(_p(Tn), _p(Qo), n, n, j, p, q)
    return Tn, Qo, rc


def std2x2(B):
    v = [ctypes.c_double(float(x)) for x in (B[0][0], B[0][1], B[1][0], B[1][1])]
    cs, sn = ctypes.c_double(), ctypes.c_double()
    cplx = lib().hqr_oracle_std2x2(*[ctypes.byref(x) for x in v], ctypes.byref(cs), ctypes.byref(sn))
    Bn = np.array([[v[0].value, v[1].value], [v[2].value, v[3].value]])
    return Bn, cs.value, sn.value, cplx


def aed(H, Q, ktop, kbot, nw, defl_mode=0, defl_thold=0.0):
    T = _fortran(H)
    n = T.shape[0]
    Qo = _fortran(Q) if Q is not None else None
    cr = np.zeros(n + 1)
    ci = np.zeros(n + 1)
    nc = ctypes.c_int(0)
    nd = lib().hqr_oracle_aed_ex(_p(T), _p(Qo), n, n, ktop, kbot, nw, _p(cr), _p(ci), ctypes.byref(nc),
                                 int(defl_mode), float(defl_thold))
    if nd < 0:
        raise ValueError(f"hqr_oracle_aed_ex returned {nd}")
    return T, Qo, nd, (cr + 1j * ci)[: nc.value]


def eig_backward(T, Q, w, g, hess_mask=True):
    Tn = _fortran(T)
    n = Tn.shape[0]
    Qn = _fortran(Q)
    w = np.asarray(w, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    wr, wi = np.ascontiguousarray(w.real), np.ascontiguousarray(w.imag)
    gr, gi = np.ascontiguousarray(g.real), np.ascontiguousarray(g.imag)
    dH = np.zeros((n, n), order="F")
    rc = lib().hqr_oracle_eig_backward(_p(Tn), _p(Qn), n, n, _p(wr), _p(wi), _p(gr), _p(gi), _p(dH),
                                       1 if hess_mask else 0)
    if rc != 0:
        raise ValueError(f"hqr_oracle_eig_backward returned {rc}")
    return dH
