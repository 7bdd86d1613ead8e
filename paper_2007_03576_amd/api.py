"""Public Python API over the C-ABI of libhqr.so (include/hqr.h)."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from ._lib import HqrError, HqrParams, check, lib

__all__ = ["schur", "schur_colmajor", "schur_batched", "eigvals", "set_params", "params",
           "last_stats", "HqrError"]


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _params(p: Optional[dict]) -> Optional[HqrParams]:
    if p is None:
        return None
    hp = HqrParams()
    for k, v in p.items():
        if not hasattr(hp, k):
            raise ValueError(f"unknown parameter {k}")
        setattr(hp, k, v)
    return hp


def set_params(**kw) -> None:
    hp = _params(kw)
    check(lib().hqr_set_params(ctypes.byref(hp)), "hqr_set_params")


def params() -> dict:
    hp = HqrParams()
    check(lib().hqr_get_params(ctypes.byref(hp)), "hqr_get_params")
    return {k: getattr(hp, k) for k, _ in HqrParams._fields_}


def last_stats() -> dict:
    arr = (ctypes.c_int64 * 8)()
    lib().hqr_last_stats(arr, 8)
    keys = ["aed_steps", "sweeps", "shifts", "aed_deflated", "small_solves", "host_syncs",
            "launches", "chase_windows"]
    return dict(zip(keys, list(arr)))


def _fortran(x: torch.Tensor) -> torch.Tensor:
    """Column-major copy (strides (1, n)) of a square matrix."""
    return x.t().contiguous().t()


def _require_device(x: torch.Tensor, name: str) -> None:
    if not x.is_cuda:
        raise HqrError(f"{name} must be a GPU tensor (no CPU path exists)")
    if x.dtype != torch.float64:
        raise HqrError(f"{name} must be float64")


def schur_colmajor(Hf: torch.Tensor, Qf: Optional[torch.Tensor], wr: torch.Tensor, wi: torch.Tensor,
                   params: Optional[dict] = None, stream=None) -> int:
    """In-place call on caller-owned column-major buffers (strides (1, ld)).
    Returns the library's info code (0 or +i); raises on argument/HIP errors."""
    _require_device(Hf, "H")
    n = Hf.shape[0]
    if Hf.dim() != 2 or Hf.shape[1] != n or (n > 1 and Hf.stride(0) != 1):
        raise HqrError("H must be square and column major")
    ld = Hf.stride(1) if n > 1 else 1
    qp = None
    if Qf is not None:
        _require_device(Qf, "Q")
        if Qf.shape != Hf.shape or (n > 1 and Qf.stride() != Hf.stride()):
            raise HqrError("Q must match H's shape and strides")
        qp = ctypes.c_void_p(Qf.data_ptr())
    hp = _params(params)
    rc = lib().hqr_schur_ex(ctypes.c_void_p(Hf.data_ptr()), qp, n, ld, ctypes.c_void_p(wr.data_ptr()),
                            ctypes.c_void_p(wi.data_ptr()), _stream_handle(stream),
                            ctypes.byref(hp) if hp is not None else None)
    return check(rc, "hqr_schur")


def schur(H: torch.Tensor, want_q: bool = True, Q0: Optional[torch.Tensor] = None,
          params: Optional[dict] = None, stream=None):
    """Real Schur form of an upper Hessenberg H (float64, on the GPU).
    Returns (T, Q, w, info) with H = Q T Q^T, w complex eigenvalues in diagonal order."""
    _require_device(H, "H")
    n = H.shape[0]
    Hf = _fortran(H)
    Qf = None
    if want_q:
        Qf = _fortran(Q0) if Q0 is not None else _fortran(torch.eye(n, dtype=H.dtype, device=H.device))
    wr = torch.empty(max(n, 1), dtype=torch.float64, device=H.device)
    wi = torch.empty_like(wr)
    info = schur_colmajor(Hf, Qf, wr, wi, params=params, stream=stream)
    w = torch.complex(wr[:n], wi[:n])
    return Hf, Qf, w, info


def schur_batched(mats: Sequence[torch.Tensor], want_q: bool = True, stream=None):
    """Batched form: list of square Hessenberg matrices (orders <= 96) on one device.
    Returns (list of T, list of Q or None, list of w, info tensor)."""
    dev = mats[0].device
    sizes = [int(m.shape[0]) for m in mats]
    offs = [0]
    for s in sizes[:-1]:
        offs.append(offs[-1] + s * s)
    eoffs = [0]
    for s in sizes[:-1]:
        eoffs.append(eoffs[-1] + s)
    packed = torch.cat([m.t().contiguous().reshape(-1) for m in mats]).to(torch.float64)
    Qp = None
    if want_q:
        Qp = torch.cat([torch.eye(s, dtype=torch.float64, device=dev).reshape(-1) for s in sizes])
    d_off = torch.tensor(offs, dtype=torch.int64, device=dev)
    d_n = torch.tensor(sizes, dtype=torch.int32, device=dev)
    d_eo = torch.tensor(eoffs, dtype=torch.int64, device=dev)
    tot = sum(sizes)
    wr = torch.empty(max(tot, 1), dtype=torch.float64, device=dev)
    wi = torch.empty_like(wr)
    info = torch.empty(len(mats), dtype=torch.int32, device=dev)
    rc = lib().hqr_schur_batched(ctypes.c_void_p(packed.data_ptr()),
                                 ctypes.c_void_p(Qp.data_ptr()) if Qp is not None else None,
                                 ctypes.c_void_p(d_off.data_ptr()), ctypes.c_void_p(d_n.data_ptr()),
                                 len(mats), ctypes.c_void_p(wr.data_ptr()), ctypes.c_void_p(wi.data_ptr()),
                                 ctypes.c_void_p(d_eo.data_ptr()), ctypes.c_void_p(info.data_ptr()),
                                 _stream_handle(stream))
    check(rc, "hqr_schur_batched")
    Ts, Qs, ws = [], [], []
    for s, o, eo in zip(sizes, offs, eoffs):
        Ts.append(packed[o:o + s * s].reshape(s, s).t())
        Qs.append(Qp[o:o + s * s].reshape(s, s).t() if Qp is not None else None)
        ws.append(torch.complex(wr[eo:eo + s], wi[eo:eo + s]))
    return Ts, Qs, ws, info


def eigvals(H: torch.Tensor) -> torch.Tensor:
    """Differentiable eigenvalues (defined in autograd.py)."""
    from .autograd import SchurEig
    return SchurEig.apply(H)
