"""GPU tests of the blocked Householder Hessenberg reduction (hqr_hessenberg,
the phase before the Schur reduction; the same kernels restore the
Hessenberg form of large AED windows inside hqr_schur).

The reduction Q^T A Q = H with Q e_1 = e_1 is unique up to the signs of Q's
columns (implicit-Q theorem); with the reflector convention beta =
-sign(alpha) ||x|| it is the one LAPACK's dgehrd computes, so H and Q are
compared entry by entry with scipy.linalg.hessenberg (an independent
implementation) within a few n u ||A||, besides exact structure, backward
error and orthogonality."""
import ctypes
import sys

import numpy as np
import pytest
import scipy.linalg as sla

pytestmark = pytest.mark.gpu
U = 2.0 ** -52


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def hess_gpu(A, want_q=True):
    import torch
    from paper_2007_03576_amd._lib import lib
    n = A.shape[0]
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()  # row-major A^T = column-major A
    Qd = torch.eye(n, dtype=torch.float64, device="cuda") if want_q else None
    rc = lib().hqr_hessenberg(ctypes.c_void_p(Ad.data_ptr()), ctypes.c_void_p(Qd.data_ptr()) if want_q else None,
                              n, max(n, 1), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, Ad.t().cpu().numpy(), (Qd.t().cpu().numpy() if want_q else None)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 33, 34, 67, 130, 257, 700])
def test_hessenberg_matches_lapack(gpu, n):
    _say(f"case hessenberg n={n}")
    A = np.random.default_rng(n).standard_normal((n, n))
    rc, H, Q = hess_gpu(A)
    assert rc == 0
    assert np.all(np.tril(H, -2) == 0.0)
    an = max(np.linalg.norm(A), 1e-300)
    be = np.linalg.norm(Q.T @ A @ Q - H) / an
    ob = np.linalg.norm(Q.T @ Q - np.eye(n))
    _say(f"  backward {be / U:.1f} u  orth {ob / U:.1f} u")
    assert be <= 100 * max(n, 1) * U and ob <= 100 * max(n, 1) * U
    Hs, Qs = sla.hessenberg(A, calc_q=True)
    tol = 100 * max(n, 1) * U * an
    assert np.abs(H - np.triu(Hs, -1)).max() <= tol, np.abs(H - Hs).max()
    assert np.abs(Q - Qs).max() <= 100 * max(n, 1) * U


def test_hessenberg_structured_inputs(gpu):
    # a zero column (reflector of a zero vector: identity) and an already
    # Hessenberg matrix (every reflector the identity: H = A, Q = I exactly)
    n = 90
    A = np.random.default_rng(1).standard_normal((n, n))
    A[:, 10] = 0.0
    rc, H, Q = hess_gpu(A)
    assert rc == 0 and np.all(np.tril(H, -2) == 0.0)
    assert np.linalg.norm(Q.T @ A @ Q - H) <= 100 * n * U * np.linalg.norm(A)
    B = np.triu(np.random.default_rng(2).standard_normal((n, n)), -1)
    rc, H, Q = hess_gpu(B)
    assert rc == 0
    assert np.array_equal(H, B) and np.array_equal(Q, np.eye(n))


def test_hessenberg_rejects_non_finite(gpu):
    n = 40
    A = np.random.default_rng(3).standard_normal((n, n))
    A[30, 2] = np.nan
    rc, _, _ = hess_gpu(A)
    assert rc == -1


def test_hessenberg_then_schur(gpu):
    # phase (i) then phase (ii): eigenvalues of a dense matrix with a known
    # spectrum through both GPU phases
    import torch
    import hqr_inputs as hi
    import paper_2007_03576_amd as hq
    n = 300
    g = np.random.default_rng(5)
    reals, a, b = hi.prescribed_spectrum(n // 2, n // 4, g)
    L = hi.blockdiag_from_spectrum(reals, a, b)
    W = hi.haar_orthogonal(n, g)
    A = W @ L @ W.T
    rc, H, Q = hess_gpu(A)
    assert rc == 0
    T, Z, w, info = hq.schur(torch.from_numpy(H).cuda(), Q0=torch.from_numpy(Q).cuda())
    assert info == 0
    T, Z = T.cpu().numpy(), Z.cpu().numpy()
    assert np.linalg.norm(Z.T @ A @ Z - T) <= 100 * n * U * np.linalg.norm(A)
    from tests import checks
    r, c, d = checks.match(w.cpu().numpy(), hi.eigs_from_spectrum(reals, a, b))
    assert d.max() <= 1e-10 * np.linalg.norm(A)
