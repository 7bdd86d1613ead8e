"""Independent checks of a computed real Schur decomposition (numpy/scipy only).

These definitions follow the paper's accuracy metrics (R_A, R_orth, E_lambda)
and the structure required of a real Schur form; none of them reuse code
from the oracle or the GPU library.
"""
import numpy as np
import scipy.linalg as sla
from scipy.optimize import linear_sum_assignment

U = 2.0 ** -52


def residuals(H, T, Q):
    n = H.shape[0]
    RA = np.linalg.norm(Q @ T @ Q.T - H) / (U * max(np.linalg.norm(H), 1e-300))
    Ro = np.linalg.norm(Q @ Q.T - np.eye(n)) / (U * np.sqrt(max(n, 1)))
    return RA, Ro


def rel_backward(H, T, Q):
    return np.linalg.norm(Q.T @ H @ Q - T) / max(np.linalg.norm(H), 1e-300)


def orth(Q):
    return np.linalg.norm(Q.T @ Q - np.eye(Q.shape[0]))


def structure_ok(T, w=None):
    """Quasi-triangular, no two consecutive nonzero subdiagonals, 2x2 blocks
    standardized (equal diagonal, b*c < 0); returns (ok, message)."""
    n = T.shape[0]
    if n > 2 and np.any(np.tril(T, -2) != 0.0):
        return False, "nonzero below the subdiagonal"
    sub = np.array([T[k + 1, k] for k in range(n - 1)])
    for k in range(n - 2):
        if sub[k] != 0.0 and sub[k + 1] != 0.0:
            return False, f"consecutive nonzero subdiagonals at {k}"
    for k in range(n - 1):
        if sub[k] != 0.0:
            a, b, c, d = T[k, k], T[k, k + 1], T[k + 1, k], T[k + 1, k + 1]
            if a != d:
                return False, f"2x2 block at {k} has unequal diagonal"
            if not (b * c < 0.0):
                return False, f"2x2 block at {k} has real eigenvalues"
    if w is not None:
        w = np.asarray(w)
        k = 0
        while k < n:
            if k + 1 < n and sub[k] != 0.0:
                if not (w[k].imag > 0 and w[k + 1].imag < 0 and w[k].real == w[k + 1].real):
                    return False, f"eigenvalue order/sign at block {k}"
                k += 2
            else:
                if w[k].imag != 0.0 or w[k].real != T[k, k]:
                    return False, f"real eigenvalue mismatch at {k}"
                k += 1
    return True, ""


def match(a, b):
    """Optimal one-to-one matching of two eigenvalue multisets; returns
    (index into a, index into b, |a-b|)."""
    a = np.asarray(a, dtype=complex)
    b = np.asarray(b, dtype=complex)
    C = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(C)
    return r, c, C[r, c]


def eig_condition(H):
    """Eigenvalues and condition numbers kappa_i = ||x|| ||y|| / |y^H x| (scipy/LAPACK)."""
    w, vl, vr = sla.eig(H, left=True, right=True)
    num = np.linalg.norm(vl, axis=0) * np.linalg.norm(vr, axis=0)
    den = np.abs(np.sum(np.conj(vl) * vr, axis=0))
    return w, num / np.maximum(den, 1e-300)
