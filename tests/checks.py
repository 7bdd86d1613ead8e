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


def _quasi_blocks(T):
    """Diagonal blocks of a quasi-triangular T: list of (start, size)."""
    n = T.shape[0]
    out, k = [], 0
    while k < n:
        if k + 1 < n and T[k + 1, k] != 0.0:
            out.append((k, 2))
            k += 2
        else:
            out.append((k, 1))
            k += 1
    return out


def _block_eigs(B):
    if B.shape[0] == 1:
        return [complex(B[0, 0])]
    p, q, r, s = B[0, 0], B[0, 1], B[1, 0], B[1, 1]
    tr, det = p + s, p * s - q * r
    disc = complex(tr * tr / 4.0 - det)
    sq = np.sqrt(disc)
    return [tr / 2.0 + sq, tr / 2.0 - sq]


def _quasi_right_vectors(T, nb=64):
    """Right eigenvectors of the upper quasi-triangular T, one column per
    eigenvalue (block order), by back substitution in row blocks of nb: the
    part below a row block enters through one matrix product, the rows inside
    it are solved one (or one 2x2 block) at a time, vectorized over all
    eigenvalues.  Columns are rescaled when they grow, so they stay finite
    unless the eigenvalue is hopelessly ill conditioned."""
    n = T.shape[0]
    blocks = _quasi_blocks(T)
    lam = np.zeros(n, complex)
    start = np.zeros(n, int)
    X = np.zeros((n, n), complex)
    for s0, m in blocks:
        B = T[s0:s0 + m, s0:s0 + m]
        ev = _block_eigs(B)
        for t in range(m):
            i = s0 + t
            lam[i], start[i] = ev[t], s0
            if m == 1:
                X[s0, i] = 1.0
            else:
                p, q, r, s = B[0, 0], B[0, 1], B[1, 0], B[1, 1]
                if q != 0.0:
                    X[s0, i], X[s0 + 1, i] = q, ev[t] - p
                else:
                    X[s0, i], X[s0 + 1, i] = ev[t] - s, r
    # entries below 1e-280 (denormal territory, far below u ||T||) are dropped:
    # they change no eigenvector meaningfully and make the arithmetic slow
    T = np.ascontiguousarray(np.where(np.abs(T) < 1e-280, 0.0, T))
    Tc = np.empty(T.shape, dtype=complex)
    Tc.real = T
    Tc.imag = 0.0
    smin = U * max(np.abs(T).max(), 1e-300)
    r1 = n
    bidx = len(blocks) - 1
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        while r1 > 0:
            r0 = max(0, r1 - nb)
            if r0 > 0 and T[r0, r0 - 1] != 0.0:
                r0 -= 1  # keep 2x2 blocks whole
            R = Tc[r0:r1, r1:] @ X[r1:, :] if r1 < n else np.zeros((r1 - r0, n), complex)
            while bidx >= 0 and blocks[bidx][0] >= r0:
                j0, m = blocks[bidx]
                act = start > j0  # eigenvalues whose own block lies below this block
                rhs = R[j0 - r0:j0 - r0 + m, :] + Tc[j0:j0 + m, j0 + m:r1] @ X[j0 + m:r1, :]
                if m == 1:
                    d = T[j0, j0] - lam
                    d = np.where(np.abs(d) < smin, smin, d)
                    X[j0] = np.where(act, -rhs[0] / d, X[j0])
                else:
                    a = T[j0, j0] - lam
                    b, c = T[j0, j0 + 1], T[j0 + 1, j0]
                    dd = T[j0 + 1, j0 + 1] - lam
                    det = a * dd - b * c
                    det = np.where(np.abs(det) < smin, smin, det)
                    r0v, r1v = -rhs[0], -rhs[1]
                    X[j0] = np.where(act, (dd * r0v - b * r1v) / det, X[j0])
                    X[j0 + 1] = np.where(act, (a * r1v - c * r0v) / det, X[j0 + 1])
                bidx -= 1
            mx = np.abs(X).max(axis=0)
            big = mx > 1e100
            if np.any(big):
                X[:, big] /= mx[big]
            X[np.abs(X) < 1e-250] = 0.0  # no denormals
            r1 = r0
    return lam, start, X


def schur_eig_condition(T, progress=None):
    """Eigenvalues of the quasi-triangular T (block order) and their condition
    numbers kappa_i = ||x_i|| ||y_i|| / |y_i^H x_i| (the same for any
    orthogonally similar matrix): right vectors x by back substitution, left
    vectors y from the right vectors of the flipped transpose J T^T J (upper
    quasi-triangular) for conj(lambda_i).  Infinite where the substitution
    overflows (kappa beyond about 1e100)."""
    n = T.shape[0]
    lam, start, X = _quasi_right_vectors(T)
    if progress:
        progress("right eigenvectors of the Schur form done")
    F = np.ascontiguousarray(T.T[::-1, ::-1])
    lamF, startF, Z = _quasi_right_vectors(F)
    if progress:
        progress("left eigenvectors of the Schur form done")
    # the block of T at rows s..s+m-1 is the block of F at rows n-s-m..n-1-s;
    # its eigenvector for conj(lambda_i) gives the left vector of lambda_i
    kap = np.full(n, np.inf)
    posF = {}
    for k in range(n):
        posF.setdefault(startF[k], []).append(k)
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        for i in range(n):
            s0 = start[i]
            m = 2 if (s0 + 1 < n and T[s0 + 1, s0] != 0.0) else 1
            cand = posF[n - s0 - m]
            k = min(cand, key=lambda c: abs(lamF[c] - np.conj(lam[i])))
            y = Z[::-1, k]
            x = X[:, i]
            den = abs(np.vdot(y, x))
            v = np.linalg.norm(x) * np.linalg.norm(y) / den if den > 0 else np.inf
            kap[i] = v if np.isfinite(v) else np.inf
    return lam, kap
