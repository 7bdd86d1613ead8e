"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws and shapes random test matrices; it holds none of the
Schur-reduction arithmetic.  The recipes follow the workloads of the paper's
experiments section (synthetic matrices with known eigenvalues, hessrand
matrices) and the benchmark configurations:

  * ``prescribed_hessenberg`` -- normal matrix W blockdiag(Lambda) W^T with real
    eigenvalues and 2x2 blocks [[a, b], [-b, a]] for conjugate pairs, W Haar
    orthogonal, reduced to Hessenberg form on the host (the Hessenberg
    reduction is the phase before the one this project implements);
  * ``gaussian_hessenberg`` -- i.i.d. N(0,1) upper triangle and subdiagonal;
  * ``hessrand`` -- N(0,1) upper triangle, subdiagonal entries chi(n-i);
  * ``syn_matrix`` -- the paper's syn_n (random upper triangular with
    eigenvalues +-1, +-3, ..., half of them lifted to complex pairs, mixed by
    one random Householder reflector), then reduced to Hessenberg form;
  * ``toeplitz_tridiagonal`` -- tridiag(c, a, b) with closed-form eigenvalues;
  * ``batched_sizes`` / ``pack`` -- uneven batch of small matrices packed
    column major with an offset table.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

SEED = 2020  # the paper's test-driver seed


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def haar_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    z = g.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def _lower_zero(H: np.ndarray) -> np.ndarray:
    return np.asfortranarray(np.triu(H, -1))


def prescribed_spectrum(n_real: int, n_pairs: int, g: np.random.Generator,
                        re_lo=-10.0, re_hi=10.0, im_lo=0.1, im_hi=5.0):
    reals = g.uniform(re_lo, re_hi, n_real)
    a = g.uniform(re_lo, re_hi, n_pairs)
    b = g.uniform(im_lo, im_hi, n_pairs)
    return reals, a, b


def separated_spectrum(n_real: int, n_pairs: int, g: np.random.Generator, gap=0.05,
                       lo=-10.0, hi=10.0, im_lo=0.1, im_hi=5.0):
    """Reals on a jittered grid and pairs drawn by rejection so that every two
    eigenvalues are at least ``gap`` apart."""
    s = (hi - lo) / n_real
    jit = max(0.0, (s - gap) / 2.0 * 0.999)
    reals = lo + (np.arange(n_real) + 0.5) * s + g.uniform(-jit, jit, n_real)
    pts = [complex(x, 0.0) for x in reals]
    a_l, b_l = [], []
    arr = np.array(pts)
    while len(a_l) < n_pairs:
        a = g.uniform(lo, hi)
        b = g.uniform(im_lo, im_hi)
        z = complex(a, b)
        if np.min(np.abs(arr - z)) >= gap and np.min(np.abs(arr - np.conj(z))) >= gap:
            a_l.append(a)
            b_l.append(b)
            arr = np.concatenate([arr, [z, np.conj(z)]])
    return reals, np.array(a_l), np.array(b_l)


def blockdiag_from_spectrum(reals, a, b) -> np.ndarray:
    n = len(reals) + 2 * len(a)
    L = np.zeros((n, n))
    k = 0
    for x in reals:
        L[k, k] = x
        k += 1
    for aa, bb in zip(a, b):
        L[k, k] = aa
        L[k + 1, k + 1] = aa
        L[k, k + 1] = bb
        L[k + 1, k] = -bb
        k += 2
    return L


def eigs_from_spectrum(reals, a, b) -> np.ndarray:
    return np.concatenate([np.asarray(reals, dtype=complex), np.asarray(a) + 1j * np.asarray(b),
                           np.asarray(a) - 1j * np.asarray(b)])


def prescribed_hessenberg(n: int, seed: int = SEED, separated: bool = False, shuffle: bool = True):
    """Normal matrix with half real eigenvalues and half conjugate pairs,
    reduced to Hessenberg form.  Returns (H, eigenvalues)."""
    g = rng(seed)
    n_pairs = n // 4
    n_real = n - 2 * n_pairs
    if separated:
        reals, a, b = separated_spectrum(n_real, n_pairs, g)
    else:
        reals, a, b = prescribed_spectrum(n_real, n_pairs, g)
    L = blockdiag_from_spectrum(reals, a, b)
    if shuffle:
        # interleave the real and complex blocks so the Hessenberg form mixes them
        blocks = [(i, 1) for i in range(n_real)] + [(n_real + 2 * j, 2) for j in range(n_pairs)]
        order = g.permutation(len(blocks))
        idx = []
        for o in order:
            s0, sz = blocks[o]
            idx.extend(range(s0, s0 + sz))
        L = L[np.ix_(idx, idx)]
    W = haar_orthogonal(n, g)
    A = W @ L @ W.T
    H = sla.hessenberg(A)
    return _lower_zero(H), eigs_from_spectrum(reals, a, b)


def gaussian_hessenberg(n: int, seed: int = SEED) -> np.ndarray:
    """Upper triangle and first subdiagonal i.i.d. N(0,1); subdiagonal redrawn
    until no entry is below 1e-300 in magnitude."""
    g = rng(seed)
    H = np.triu(g.standard_normal((n, n)))
    sub = g.standard_normal(max(n - 1, 0))
    while np.any(np.abs(sub) < 1e-300):
        bad = np.abs(sub) < 1e-300
        sub[bad] = g.standard_normal(int(bad.sum()))
    H[np.arange(1, n), np.arange(n - 1)] = sub
    return np.asfortranarray(H)


def hessrand(n: int, seed: int = SEED) -> np.ndarray:
    """The paper's hess_n: N(0,1) upper triangle, h_{i+1,i}^2 ~ chi^2(n-i)."""
    g = rng(seed)
    H = np.triu(g.standard_normal((n, n)))
    dof = n - np.arange(1, n)
    H[np.arange(1, n), np.arange(n - 1)] = np.sqrt(g.chisquare(dof))
    return np.asfortranarray(H)


def syn_matrix(n: int, seed: int = SEED):
    """The paper's syn_n in Hessenberg form.  Returns (H, eigenvalues)."""
    g = rng(seed)
    T = np.triu(g.uniform(-1.0, 1.0, (n, n)), 1)
    vals = np.array([(2 * k + 1) * (1 if k % 2 == 0 else -1) for k in range(n)], dtype=float)
    vals = g.permutation(vals)
    npair = n // 4
    sizes = g.permutation([2] * npair + [1] * (n - 2 * npair))
    eig = np.zeros(n, dtype=complex)
    k = 0
    for sz in sizes:
        re = vals[k]
        if sz == 2:
            T[k, k] = T[k + 1, k + 1] = re
            T[k, k + 1] = abs(re)
            T[k + 1, k] = -abs(re)
            eig[k], eig[k + 1] = re + 1j * abs(re), re - 1j * abs(re)
        else:
            T[k, k] = re
            eig[k] = re
        k += sz
    v = g.standard_normal(n)
    v /= np.linalg.norm(v)
    Qb = np.eye(n) - 2.0 * np.outer(v, v)
    A = Qb @ T @ Qb.T
    H = sla.hessenberg(A)
    return _lower_zero(H), eig


def toeplitz_tridiagonal(n: int, a: float, b: float, c: float):
    """tridiag(c (sub), a (diag), b (super)); eigenvalues a + 2 sqrt(bc) cos(k pi/(n+1))."""
    H = np.diag(np.full(n, float(a)))
    if n > 1:
        H += np.diag(np.full(n - 1, float(b)), 1) + np.diag(np.full(n - 1, float(c)), -1)
    k = np.arange(1, n + 1)
    eig = a + 2.0 * np.sqrt(complex(b * c)) * np.cos(k * np.pi / (n + 1))
    return np.asfortranarray(H), eig


def batched_sizes(count: int, lo: int, hi: int, seed: int = SEED) -> np.ndarray:
    return rng(seed).integers(lo, hi + 1, size=count).astype(np.int32)


def batched_gaussian(sizes, seed: int = SEED):
    """Packed column-major storage of len(sizes) Gaussian Hessenberg matrices.
    Returns (packed, offsets) with offsets[i] = sum_{j<i} n_j^2."""
    sizes = np.asarray(sizes, dtype=np.int64)
    offs = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes) > 1:
        offs[1:] = np.cumsum(sizes[:-1] ** 2)
    total = int((sizes ** 2).sum())
    out = np.zeros(total)
    g = rng(seed)
    for i, n in enumerate(sizes):
        n = int(n)
        if n == 0:
            continue
        H = np.triu(g.standard_normal((n, n)))
        sub = g.standard_normal(n - 1)
        sub[np.abs(sub) < 1e-300] = 1.0
        H[np.arange(1, n), np.arange(n - 1)] = sub
        out[offs[i]:offs[i] + n * n] = H.reshape(-1, order="F")
    return out, offs


def unpack(packed, offs, sizes, i):
    n = int(sizes[i])
    return packed[int(offs[i]):int(offs[i]) + n * n].reshape((n, n), order="F")


def eig_offsets(sizes) -> np.ndarray:
    sizes = np.asarray(sizes, dtype=np.int64)
    e = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes) > 1:
        e[1:] = np.cumsum(sizes[:-1])
    return e


def hessenberg_reduce_torch(A):
    """Householder reduction of a square device matrix to upper Hessenberg form
    (input preparation for the large configurations, where the host reduction
    would take minutes).  Returns the Hessenberg matrix with exact zeros below
    the subdiagonal; the orthogonal factor is not formed."""
    import torch
    A = A.clone()
    n = A.shape[0]
    for k in range(n - 2):
        x = A[k + 1:, k]
        alpha = x[0].item()
        tail = torch.linalg.vector_norm(x[1:]).item()
        if tail == 0.0:
            continue
        nrm = float(np.hypot(alpha, tail))
        beta = -nrm if alpha >= 0 else nrm
        tau = (beta - alpha) / beta
        v = x / (alpha - beta)
        v[0] = 1.0
        # left: rows k+1.., columns k..
        w = torch.mv(A[k + 1:, k:].t(), v)
        A[k + 1:, k:].addr_(v, w, alpha=-tau)
        # right: all rows, columns k+1..
        z = torch.mv(A[:, k + 1:], v)
        A[:, k + 1:].addr_(z, v, alpha=-tau)
        A[k + 2:, k] = 0.0
        A[k + 1, k] = beta
    return torch.triu(A, -1)


def hessenberg_reduce_blocked(A, nb: int = 64, progress=None):
    """Blocked Householder reduction of a square device matrix to upper
    Hessenberg form (input preparation at the paper's scale).  Per panel of nb
    columns, with A0 the matrix at the start of the panel, Q = I - V T V^T the
    product of the panel's reflectors and Y = A0 V T:
      column j of the panel is Q_j^T A0 Q_j e_(k+j), formed from A0, Y and V
      (Q_j the first j reflectors); its reflector extends T and Y (one product
      A0 v_j per column); after the panel A <- Q^T (A0 - Y V^T) with three
      matrix products.  Returns the Hessenberg matrix with exact zeros below
      the subdiagonal; Q is not kept."""
    import torch
    A = A.clone()
    n = A.shape[0]
    dt, dev = A.dtype, A.device
    for k0 in range(0, n - 2, nb):
        b = min(nb, n - 2 - k0)
        A0 = A
        V = torch.zeros((n, b), dtype=dt, device=dev)
        T = torch.zeros((b, b), dtype=dt, device=dev)
        Y = torch.zeros((n, b), dtype=dt, device=dev)
        betas = []
        for j in range(b):
            c = k0 + j
            col = A0[:, c].clone()
            if j > 0:
                Vj, Tj, Yj = V[:, :j], T[:j, :j], Y[:, :j]
                col -= Yj @ Vj[c, :]
                col -= Vj @ (Tj.t() @ (Vj.t() @ col))
            x = col[c + 1:]
            alpha = float(x[0])
            tail = float(torch.linalg.vector_norm(x[1:])) if x.numel() > 1 else 0.0
            v = torch.zeros(n, dtype=dt, device=dev)
            v[c + 1] = 1.0
            if tail == 0.0:
                tau, beta = 0.0, alpha
            else:
                nrm = float(np.hypot(alpha, tail))
                beta = -nrm if alpha >= 0 else nrm
                tau = (beta - alpha) / beta
                v[c + 2:] = x[1:] / (alpha - beta)
            betas.append(beta)
            V[:, j] = v
            if j > 0:
                T[:j, j] = -tau * (T[:j, :j] @ (V[:, :j].t() @ v))
            T[j, j] = tau
            yv = A0[:, c + 1:] @ v[c + 1:]
            if j > 0:
                yv = yv - Y[:, :j] @ (V[:, :j].t() @ v)
            Y[:, j] = tau * yv
        M = A0 - Y @ V.t()
        M -= V @ (T.t() @ (V.t() @ M))
        for j in range(b):
            c = k0 + j
            M[c + 2:, c] = 0.0
            M[c + 1, c] = betas[j]
        A = M
        if progress is not None:
            progress(k0 + b, n)
    return torch.triu(A, -1)


def hessenberg_reduce_torch_batched(A):
    """Unblocked Householder reduction of a stack of square matrices (B, n, n)
    to upper Hessenberg form, vectorized over the stack (input preparation of
    the differentiation benchmark).  Returns the Hessenberg matrices with
    exact zeros below the subdiagonal; the orthogonal factors are not formed."""
    import torch
    A = A.clone()
    B, n, _ = A.shape
    for k in range(n - 2):
        x = A[:, k + 1:, k]                                   # (B, n-k-1)
        alpha = x[:, 0]
        tail = torch.linalg.vector_norm(x[:, 1:], dim=1)
        nrm = torch.hypot(alpha, tail)
        beta = torch.where(alpha >= 0, -nrm, nrm)
        live = tail > 0
        denom = torch.where(live, alpha - beta, torch.ones_like(alpha))
        tau = torch.where(live, (beta - alpha) / torch.where(live, beta, torch.ones_like(beta)),
                          torch.zeros_like(beta))
        v = x / denom[:, None]
        v[:, 0] = 1.0
        # left: rows k+1.., columns k..
        sub = A[:, k + 1:, k:]
        w = torch.einsum("bi,bij->bj", v, sub)
        sub -= tau[:, None, None] * v[:, :, None] * w[:, None, :]
        # right: all rows, columns k+1..
        right = A[:, :, k + 1:]
        z = torch.einsum("bij,bj->bi", right, v)
        right -= tau[:, None, None] * z[:, :, None] * v[:, None, :]
        A[:, k + 2:, k] = 0.0
        A[:, k + 1, k] = torch.where(live, beta, alpha)
    return torch.triu(A, -1)


def prescribed_batch_device(count: int, n: int, seed: int = SEED, device="cuda"):
    """Stack of `count` Hessenberg matrices of order n with well-separated
    prescribed spectra (n/2 reals on a jittered grid, n/4 pairs drawn by
    rejection; every two eigenvalues at least 0.05 apart), each a Haar
    orthogonal similarity of its block diagonal, reduced on the GPU.
    Returns (H (count, n, n) row-major device tensor, eigenvalues list)."""
    import torch
    g = rng(seed)
    n_pairs = n // 4
    n_real = n - 2 * n_pairs
    Ls, eigs = [], []
    for _ in range(count):
        reals, a, b = separated_spectrum(n_real, n_pairs, g)
        Ls.append(blockdiag_from_spectrum(reals, a, b))
        eigs.append(eigs_from_spectrum(reals, a, b))
    L = torch.from_numpy(np.stack(Ls)).to(device)
    Z = torch.from_numpy(g.standard_normal((count, n, n))).to(device)
    W, R = torch.linalg.qr(Z)
    d = torch.diagonal(R, dim1=1, dim2=2)
    W = W * torch.where(d < 0, -torch.ones_like(d), torch.ones_like(d))[:, None, :]
    A = torch.bmm(torch.bmm(W, L), W.transpose(1, 2).contiguous())
    return hessenberg_reduce_torch_batched(A), eigs


def prescribed_hessenberg_device(n: int, seed: int = SEED, device="cuda", progress=None):
    """prescribed_hessenberg built on the GPU with torch (Haar W by QR, A = W L W^T,
    blocked Householder Hessenberg reduction; `progress(done, n)` is called after
    each panel).  Returns (H row-major device tensor, eigenvalues)."""
    import torch
    g = rng(seed)
    n_pairs = n // 4
    n_real = n - 2 * n_pairs
    reals, a, b = prescribed_spectrum(n_real, n_pairs, g)
    sizes = np.array([1] * n_real + [2] * n_pairs)
    order = g.permutation(len(sizes))
    Z = torch.from_numpy(g.standard_normal((n, n))).to(device)
    W, R = torch.linalg.qr(Z)
    del Z
    W = W * torch.sign(torch.diagonal(R)).where(torch.diagonal(R) != 0, torch.ones((), device=device, dtype=W.dtype))
    del R
    WL = torch.empty_like(W)
    col = 0
    for o in order:
        if o < n_real:
            WL[:, col] = W[:, col] * reals[o]
            col += 1
        else:
            j = o - n_real
            w1, w2 = W[:, col], W[:, col + 1]
            WL[:, col] = a[j] * w1 - b[j] * w2
            WL[:, col + 1] = b[j] * w1 + a[j] * w2
            col += 2
    A = WL @ W.t()
    del WL, W
    H = hessenberg_reduce_blocked(A, nb=64, progress=progress)
    return H, eigs_from_spectrum(reals, a, b)
