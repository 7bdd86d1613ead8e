"""Public Python API over the C-ABI of libhqr.so (include/hqr.h)."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from ._lib import HqrError, HqrParams, check, lib

__all__ = ["schur", "schur_colmajor", "schur_batched", "eigvals", "hessenberg", "eigenvectors", "set_params", "params",
           "set_batched_table", "batched_table",
           "last_stats", "HqrError", "BatchedProblem", "BatchedGraph", "set_batched_launch",
           "batched_launch"]


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
    arr = (ctypes.c_int64 * 12)()
    lib().hqr_last_stats(arr, 12)
    keys = ["aed_steps", "sweeps", "shifts", "aed_deflated", "small_solves", "host_syncs",
            "launches", "chase_windows", "deflation_windows", "reordering_windows",
            "sequential_aeds", "parallel_aeds"]
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


def hessenberg(A: torch.Tensor, want_q: bool = True, stream=None):
    """Upper Hessenberg form of a dense square float64 GPU matrix:
    returns (H, Q) with A = Q H Q^T (hqr_hessenberg)."""
    _require_device(A, "A")
    n = A.shape[0]
    Af = _fortran(A)
    Qf = _fortran(torch.eye(n, dtype=A.dtype, device=A.device)) if want_q else None
    rc = lib().hqr_hessenberg(ctypes.c_void_p(Af.data_ptr()), ctypes.c_void_p(Qf.data_ptr()) if want_q else None,
                              n, max(n, 1), _stream_handle(stream))
    check(rc, "hqr_hessenberg")
    return Af, Qf


def eigenvectors(T: torch.Tensor, Q: torch.Tensor, w: torch.Tensor, stream=None) -> torch.Tensor:
    """Right eigenvectors of H = Q T Q^T from the real Schur form that schur()
    returns (T, Q column major, w complex in diagonal order): a complex
    (n x n) tensor whose column j is the unit eigenvector of w[j]
    (hqr_eigenvectors, dgeev layout unpacked)."""
    _require_device(T, "T")
    n = T.shape[0]
    Tf, Qf = _fortran(T), _fortran(Q)
    wr = w.real.contiguous().to(torch.float64)
    wi = w.imag.contiguous().to(torch.float64)
    X = _fortran(torch.empty(n, n, dtype=torch.float64, device=T.device))
    rc = lib().hqr_eigenvectors(ctypes.c_void_p(Tf.data_ptr()), ctypes.c_void_p(Qf.data_ptr()), n, max(n, 1),
                                ctypes.c_void_p(wr.data_ptr()), ctypes.c_void_p(wi.data_ptr()),
                                ctypes.c_void_p(X.data_ptr()), max(n, 1), _stream_handle(stream))
    check(rc, "hqr_eigenvectors")
    V = torch.complex(X, torch.zeros_like(X))
    # columns j, j+1 of a conjugate pair hold Re and Im of the eigenvector of
    # w[j] (dgeev layout); the pair starts are found on the host, the columns
    # are unpacked in two vectorized assignments
    wi_h = wi.cpu().numpy()
    starts = []
    j = 0
    while j < n:
        if wi_h[j] > 0 and j + 1 < n:
            starts.append(j)
            j += 2
        else:
            j += 1
    if starts:
        p = torch.tensor(starts, dtype=torch.int64, device=X.device)
        re, im = X[:, p], X[:, p + 1]
        V[:, p] = torch.complex(re, im)
        V[:, p + 1] = torch.complex(re, -im)
    return V


def set_batched_launch(wg_per_cu: int, wide_n: int) -> None:
    """Launch shape of the batched global-memory grid (hqr_set_batched_launch)."""
    check(lib().hqr_set_batched_launch(int(wg_per_cu), int(wide_n)), "hqr_set_batched_launch")


def set_batched_table(upper: Sequence[int], nw: Sequence[int], ns: Sequence[int]) -> None:
    """Per-size-bucket AED window nw and shifts per step ns of the batched
    form for orders above 96 (hqr_set_batched_table): bucket i takes the
    orders up to upper[i]; nw = 0 selects double-shift Francis.  Empty
    sequences restore double shifts everywhere."""
    k = len(upper)
    arr = lambda v: (ctypes.c_int32 * max(k, 1))(*[int(x) for x in v])
    check(lib().hqr_set_batched_table(k, arr(upper), arr(nw), arr(ns)), "hqr_set_batched_table")


def batched_table() -> dict:
    n = ctypes.c_int32()
    u, w, s = (ctypes.c_int32 * 8)(), (ctypes.c_int32 * 8)(), (ctypes.c_int32 * 8)()
    check(lib().hqr_get_batched_table(ctypes.byref(n), u, w, s), "hqr_get_batched_table")
    k = n.value
    return {"upper": list(u)[:k], "nw": list(w)[:k], "ns": list(s)[:k]}


def batched_launch() -> dict:
    a, b = ctypes.c_int32(), ctypes.c_int32()
    check(lib().hqr_get_batched_launch(ctypes.byref(a), ctypes.byref(b)), "hqr_get_batched_launch")
    return {"wg_per_cu": a.value, "wide_n": b.value}


class BatchedProblem:
    """Device buffers of one packing of the batched form: matrices of the given
    orders stored back to back column major (offsets = running sums of n^2),
    Q (identity on entry) likewise, eigenvalue slots (offsets = running sums
    of n) and per-matrix info."""

    def __init__(self, sizes: Sequence[int], want_q: bool = True, device="cuda"):
        dev = torch.device(device)
        self.sizes = [int(s) for s in sizes]
        offs, eoffs = [0], [0]
        for s in self.sizes[:-1]:
            offs.append(offs[-1] + s * s)
            eoffs.append(eoffs[-1] + s)
        self.offs, self.eoffs = offs, eoffs
        tot2 = sum(s * s for s in self.sizes)
        self.H = torch.zeros(max(tot2, 1), dtype=torch.float64, device=dev)
        self.Q = torch.zeros_like(self.H) if want_q else None
        self.Q0 = None
        if want_q:
            self.Q0 = torch.cat([torch.eye(s, dtype=torch.float64, device=dev).reshape(-1)
                                 for s in self.sizes]) if self.sizes else torch.zeros(1, dtype=torch.float64,
                                                                                       device=dev)
        self.d_off = torch.tensor(offs, dtype=torch.int64, device=dev)
        self.d_n = torch.tensor(self.sizes, dtype=torch.int32, device=dev)
        self.d_eo = torch.tensor(eoffs, dtype=torch.int64, device=dev)
        tot = sum(self.sizes)
        self.wr = torch.empty(max(tot, 1), dtype=torch.float64, device=dev)
        self.wi = torch.empty_like(self.wr)
        self.info = torch.empty(len(self.sizes), dtype=torch.int32, device=dev)

    def load(self, packed: torch.Tensor) -> None:
        """Copy packed inputs in (and Q0 = I) on the current stream."""
        self.H[:packed.numel()].copy_(packed)
        if self.Q is not None:
            self.Q.copy_(self.Q0)

    def solve(self, stream=None) -> None:
        P = lambda t: ctypes.c_void_p(t.data_ptr())
        rc = lib().hqr_schur_batched(P(self.H), P(self.Q) if self.Q is not None else None, P(self.d_off),
                                     P(self.d_n), len(self.sizes), P(self.wr), P(self.wi), P(self.d_eo),
                                     P(self.info), _stream_handle(stream))
        check(rc, "hqr_schur_batched")

    def results(self):
        Ts, Qs, ws = [], [], []
        for s, o, eo in zip(self.sizes, self.offs, self.eoffs):
            Ts.append(self.H[o:o + s * s].reshape(s, s).t())
            Qs.append(self.Q[o:o + s * s].reshape(s, s).t() if self.Q is not None else None)
            ws.append(torch.complex(self.wr[eo:eo + s], self.wi[eo:eo + s]))
        return Ts, Qs, ws, self.info


class BatchedGraph:
    """The batched solve of one packing captured once into a HIP graph
    (through torch.cuda.CUDAGraph) and replayed: run() copies new inputs into
    the captured buffers, replays, and returns the buffers.  The library's
    work queue for the capture stream is allocated by an uncaptured warm-up
    solve before capture."""

    def __init__(self, sizes: Sequence[int], want_q: bool = True, device="cuda"):
        self.prob = BatchedProblem(sizes, want_q, device)
        self.stream = torch.cuda.Stream(device=device)
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            if self.prob.Q is not None:
                self.prob.Q.copy_(self.prob.Q0)
            self.prob.solve()  # warm-up: queue buffer and kernel attributes
        self.stream.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream, capture_error_mode="relaxed"):
            self.prob.solve()

    def run(self, packed: torch.Tensor):
        self.prob.load(packed)
        self.graph.replay()
        return self.prob.results()


def pack(mats: Sequence[torch.Tensor]) -> torch.Tensor:
    """Column-major packing of square matrices back to back."""
    return torch.cat([m.t().contiguous().reshape(-1) for m in mats]).to(torch.float64)


def schur_batched(mats: Sequence[torch.Tensor], want_q: bool = True, stream=None):
    """Batched form: list of square Hessenberg matrices of any orders on one
    device.  Returns (list of T, list of Q or None, list of w, info tensor)."""
    dev = mats[0].device
    prob = BatchedProblem([int(m.shape[0]) for m in mats], want_q, dev)
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):
        prob.load(pack(mats))
    prob.solve(s)
    return prob.results()


def eigvals(H: torch.Tensor) -> torch.Tensor:
    """Differentiable eigenvalues (defined in autograd.py)."""
    from .autograd import SchurEig
    return SchurEig.apply(H)


def qz_batched(Hs: Sequence[torch.Tensor], Ts: Sequence[torch.Tensor], want_qz: bool = True, stream=None):
    """QZ variant for batches of pairs: lists of square float64 GPU matrices
    (H_b upper Hessenberg, T_b upper triangular, one device; orders up to 64
    are reduced in LDS, larger ones in global memory).
    Returns (S list, T list, Q list or None, Z list or None, alpha list
    (complex), beta list, info tensor) with Q^T H Z = S, Q^T T Z = T' per pair
    (hqr_qz_batched)."""
    if len(Hs) != len(Ts):
        raise ValueError("Hs and Ts differ in length")
    for H, T in zip(Hs, Ts):
        _require_device(H, "H")
        _require_device(T, "T")
        if H.shape != T.shape or H.dim() != 2 or H.shape[0] != H.shape[1]:
            raise ValueError("each pair must be two square matrices of the same order")
    if not Hs:
        return [], [], [], [], [], [], torch.zeros(0, dtype=torch.int32)
    dev = Hs[0].device
    sizes = [int(H.shape[0]) for H in Hs]
    offs, eoffs = [0], [0]
    for n in sizes[:-1]:
        offs.append(offs[-1] + n * n)
        eoffs.append(eoffs[-1] + n)
    Hp, Tp = pack(Hs), pack(Ts)
    Qp = Zp = None
    if want_qz:
        Qp = torch.cat([torch.eye(n, dtype=torch.float64, device=dev).reshape(-1) for n in sizes])
        Zp = Qp.clone()
    tot = max(sum(sizes), 1)
    ar = torch.zeros(tot, dtype=torch.float64, device=dev)
    ai = torch.zeros_like(ar)
    be = torch.zeros_like(ar)
    info = torch.zeros(len(sizes), dtype=torch.int32, device=dev)
    d_off = torch.tensor(offs, dtype=torch.int64, device=dev)
    d_n = torch.tensor(sizes, dtype=torch.int32, device=dev)
    d_eo = torch.tensor(eoffs, dtype=torch.int64, device=dev)
    P = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    rc = lib().hqr_qz_batched(P(Hp), P(Tp), P(Qp), P(Zp), P(d_off), P(d_n), len(sizes), P(ar), P(ai), P(be),
                              P(d_eo), P(info), _stream_handle(stream))
    check(rc, "hqr_qz_batched")
    S, Tt, Q, Z, alpha, beta = [], [], [], [], [], []
    for b, n in enumerate(sizes):
        o, e = offs[b], eoffs[b]
        S.append(Hp[o:o + n * n].reshape(n, n).t())
        Tt.append(Tp[o:o + n * n].reshape(n, n).t())
        if want_qz:
            Q.append(Qp[o:o + n * n].reshape(n, n).t())
            Z.append(Zp[o:o + n * n].reshape(n, n).t())
        alpha.append(torch.complex(ar[e:e + n], ai[e:e + n]))
        beta.append(be[e:e + n])
    return S, Tt, (Q if want_qz else None), (Z if want_qz else None), alpha, beta, info
