"""Differentiable eigenvalues: torch.autograd.Function over the GPU Schur solver.

forward: real Schur form H = Q T Q^T (hqr_schur for one matrix,
hqr_schur_batched for a stack of equal-order matrices); returns the complex
eigenvalues in diagonal order.
backward: hqr_eig_backward_batched forms the right and left eigenvectors of T
by quasi-triangular substitution, back-transforms them with Q and assembles
dL/dH = Re(conj(Y) diag(conj(g)/(y^H x)) X^T) with FP64-MFMA products; entries
below the first subdiagonal get zero gradient (the forward never reads them).
"""
import ctypes

import torch

from ._lib import check, lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr())


class SchurEig(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H):
        if H.dtype != torch.float64 or not H.is_cuda:
            raise TypeError("SchurEig expects float64 CUDA tensors")
        single = H.dim() == 2
        Hb = H.unsqueeze(0) if single else H
        B, n, _ = Hb.shape
        # column-major packed copies: block b holds H_b^T row-major = H_b column-major
        T = Hb.transpose(1, 2).contiguous()
        Q = torch.eye(n, dtype=torch.float64, device=H.device).expand(B, n, n).contiguous()
        wr = torch.empty(B * n, dtype=torch.float64, device=H.device)
        wi = torch.empty_like(wr)
        L = lib()
        if single:
            rc = L.hqr_schur(_ptr(T), _ptr(Q), n, n, _ptr(wr), _ptr(wi), _stream())
            check(rc, "hqr_schur")
            if rc > 0:
                raise RuntimeError(f"Schur reduction did not converge (info={rc})")
        else:
            offs = torch.arange(B, dtype=torch.int64, device=H.device) * (n * n)
            eo = torch.arange(B, dtype=torch.int64, device=H.device) * n
            nn = torch.full((B,), n, dtype=torch.int32, device=H.device)
            info = torch.empty(B, dtype=torch.int32, device=H.device)
            check(L.hqr_schur_batched(_ptr(T), _ptr(Q), _ptr(offs), _ptr(nn), B, _ptr(wr), _ptr(wi), _ptr(eo),
                                      _ptr(info), _stream()), "hqr_schur_batched")
            if int(info.abs().max()) != 0:
                raise RuntimeError("batched Schur reduction did not converge")
        ctx.save_for_backward(T, Q, wr, wi)
        ctx.single = single
        w = torch.complex(wr, wi).reshape(B, n)
        return w[0] if single else w

    @staticmethod
    def backward(ctx, gw):
        T, Q, wr, wi = ctx.saved_tensors
        B, n, _ = T.shape
        g = gw.reshape(B * n)
        gr = g.real.contiguous().to(torch.float64)
        gi = g.imag.contiguous().to(torch.float64)
        dH = torch.empty_like(T)
        offs = torch.arange(B, dtype=torch.int64, device=T.device) * (n * n)
        nn = torch.full((B,), n, dtype=torch.int32, device=T.device)
        check(lib().hqr_eig_backward_batched(_ptr(T), _ptr(Q), _ptr(offs), _ptr(nn), B, _ptr(wr), _ptr(wi),
                                             _ptr(gr), _ptr(gi), _ptr(dH), 1, _stream()),
              "hqr_eig_backward_batched")
        out = dH.transpose(1, 2)  # column-major blocks -> logical matrices
        return out[0] if ctx.single else out


class PackedSchurEig(torch.autograd.Function):
    """Eigenvalues of matrices of uneven orders packed back to back column
    major (the batched form's layout); forward hqr_schur_batched, backward
    hqr_eig_backward_batched with the same offsets."""

    @staticmethod
    def forward(ctx, packed, sizes):
        if packed.dtype != torch.float64 or not packed.is_cuda:
            raise TypeError("PackedSchurEig expects a float64 CUDA tensor")
        dev = packed.device
        sz = [int(s) for s in sizes]
        offs_l, eo_l = [0], [0]
        for s in sz[:-1]:
            offs_l.append(offs_l[-1] + s * s)
            eo_l.append(eo_l[-1] + s)
        offs = torch.tensor(offs_l, dtype=torch.int64, device=dev)
        eo = torch.tensor(eo_l, dtype=torch.int64, device=dev)
        nn = torch.tensor(sz, dtype=torch.int32, device=dev)
        T = packed.detach().clone()
        Q = torch.cat([torch.eye(s, dtype=torch.float64, device=dev).reshape(-1) for s in sz])
        tot = sum(sz)
        wr = torch.empty(max(tot, 1), dtype=torch.float64, device=dev)
        wi = torch.empty_like(wr)
        info = torch.empty(len(sz), dtype=torch.int32, device=dev)
        check(lib().hqr_schur_batched(_ptr(T), _ptr(Q), _ptr(offs), _ptr(nn), len(sz), _ptr(wr), _ptr(wi),
                                      _ptr(eo), _ptr(info), _stream()), "hqr_schur_batched")
        if int(info.abs().max()) != 0:
            raise RuntimeError("batched Schur reduction did not converge")
        ctx.save_for_backward(T, Q, wr, wi, offs, nn)
        return torch.complex(wr[:tot], wi[:tot])

    @staticmethod
    def backward(ctx, gw):
        T, Q, wr, wi, offs, nn = ctx.saved_tensors
        gr = torch.zeros_like(wr)
        gi = torch.zeros_like(wi)
        gr[:gw.numel()] = gw.real.to(torch.float64)
        gi[:gw.numel()] = gw.imag.to(torch.float64)
        dH = torch.empty_like(T)
        check(lib().hqr_eig_backward_batched(_ptr(T), _ptr(Q), _ptr(offs), _ptr(nn), nn.numel(), _ptr(wr),
                                             _ptr(wi), _ptr(gr), _ptr(gi), _ptr(dH), 1, _stream()),
              "hqr_eig_backward_batched")
        return dH, None


def eigvals_uneven(mats):
    """Differentiable eigenvalues of a list of square Hessenberg matrices of
    any orders (one batched solve, one batched backward); returns a list of
    complex eigenvalue tensors in diagonal order."""
    sizes = tuple(int(m.shape[0]) for m in mats)
    packed = torch.cat([m.transpose(0, 1).reshape(-1) for m in mats])
    w = PackedSchurEig.apply(packed, sizes)
    return list(torch.split(w, list(sizes)))
