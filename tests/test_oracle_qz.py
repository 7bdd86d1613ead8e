"""Pins of the oracle's QZ variant (test infrastructure, CPU only).

The oracle reduces a Hessenberg-triangular pair (H, T) to generalized real
Schur form (Sec. 2, remarks on the generalized case: S quasi upper triangular
with 2x2 blocks only for complex conjugate pairs, T upper triangular,
(S, T) = Q^T (H, T) Z) and reports the generalized eigenvalues alpha / beta,
beta = 0 for an infinite one (|t_kk| <= u ||T||_F, the convention the paper
adopts; Sec. 3.2 'push infinities' chases them up the diagonal).

Pinned against what the mathematics fixes, independently of the oracle:
  * LAPACK's generalized eigensolver (scipy.linalg.eigvals(H, T), dggev):
    finite eigenvalues and the number of infinite ones;
  * T = I: the pencil's eigenvalues are those of H (numpy.linalg.eigvals and
    the standard-case oracle);
  * 2x2 pairs: the roots of det(H - lambda T), a quadratic written out here;
  * structure, backward error and orthogonality of (S, T, Q, Z);
  * planted mistakes in the oracle (a reflector not accumulated into Z, a
    rotation that misses T, a sign error in the shift polynomial) fail here.
"""
import numpy as np
import pytest
import scipy.linalg as sl
from scipy.optimize import linear_sum_assignment

import oracle

U = 2.0 ** -52


def pencil(n, seed, zeros=()):
    g = np.random.default_rng(seed)
    H = np.triu(g.standard_normal((n, n)), -1)
    T = np.triu(g.standard_normal((n, n)))
    for k in zeros:
        T[k, k] = 0.0
    return H, T


def match(a, b):
    if len(a) == 0:
        return 0.0
    C = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(C)
    return C[r, c].max()


def reference(H, T):
    a, b = sl.eigvals(H, T, homogeneous_eigvals=True)
    inf = np.abs(b) <= 1e-12 * np.abs(a)
    return a[~inf] / b[~inf], int(inf.sum())


def structure(S, Tt, alpha, beta):
    n = S.shape[0]
    assert np.all(np.tril(Tt, -1) == 0.0)
    assert np.all(np.tril(S, -2) == 0.0)
    k = 0
    while k < n:
        if k + 1 < n and S[k + 1, k] != 0.0:
            # a 2x2 block: a complex conjugate pair with beta > 0
            assert alpha[k].imag > 0 and alpha[k + 1].imag < 0, k
            assert beta[k] > 0 and beta[k + 1] > 0
            k += 2
        else:
            assert alpha[k].imag == 0.0
            assert beta[k] >= 0.0
            assert alpha[k].real == (S[k, k] if Tt[k, k] >= 0 else -S[k, k])
            k += 1


def solve(H, T):
    S, Tt, Q, Z, alpha, beta, info = oracle.qz(H, T)
    assert info == 0
    n = H.shape[0]
    assert np.linalg.norm(Q.T @ H @ Z - S) <= 100 * n * U * max(np.linalg.norm(H), 1e-300)
    assert np.linalg.norm(Q.T @ T @ Z - Tt) <= 100 * n * U * max(np.linalg.norm(T), 1e-300)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 100 * n * U
    assert np.linalg.norm(Z.T @ Z - np.eye(n)) <= 100 * n * U
    structure(S, Tt, alpha, beta)
    return S, Tt, alpha, beta


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 12, 25, 40])
def test_qz_matches_lapack(n):
    for seed in range(3):
        H, T = pencil(n, 100 * n + seed)
        S, Tt, alpha, beta = solve(H, T)
        lam = alpha[beta > 0] / beta[beta > 0]
        ref, ninf = reference(H, T)
        assert int((beta == 0).sum()) == ninf == 0
        assert len(lam) == len(ref)
        assert match(lam, ref) <= 1e-9 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n,zeros", [(6, (0,)), (6, (5,)), (9, (3,)), (12, (0, 5, 11)), (20, (2, 3, 10)),
                                     (15, (7, 8, 9))])
def test_qz_infinite_eigenvalues(n, zeros):
    H, T = pencil(n, 7 * n + len(zeros), zeros)
    S, Tt, alpha, beta = solve(H, T)
    ref, ninf = reference(H, T)
    assert ninf >= 1
    assert int((beta == 0).sum()) == ninf
    lam = alpha[beta > 0] / beta[beta > 0]
    assert len(lam) == len(ref)
    assert match(lam, ref) <= 1e-8 * max(1.0, np.abs(ref).max())
    # every infinite eigenvalue sits on an exact zero of T's diagonal
    assert np.all(np.diag(Tt)[beta == 0] == 0.0)


@pytest.mark.parametrize("n", [5, 16, 33])
def test_qz_identity_T_is_the_standard_problem(n):
    H, _ = pencil(n, 3 * n)
    S, Tt, alpha, beta = solve(H, np.eye(n))
    lam = alpha / beta
    assert match(lam, np.linalg.eigvals(H)) <= 1e-10 * max(1.0, np.abs(lam).max())
    _, _, w, info, _ = oracle.schur(H, want_q=False)
    assert info == 0
    assert match(lam, w) <= 1e-10 * max(1.0, np.abs(lam).max())


def test_qz_2x2_closed_form():
    g = np.random.default_rng(5)
    for _ in range(50):
        H = g.standard_normal((2, 2))
        T = np.triu(g.standard_normal((2, 2)))
        # det(H - l T) = t11 t22 l^2 - (h11 t22 + h22 t11 - h21 t12) l + (h11 h22 - h12 h21)
        c2 = T[0, 0] * T[1, 1]
        c1 = -(H[0, 0] * T[1, 1] + H[1, 1] * T[0, 0] - H[1, 0] * T[0, 1])
        c0 = H[0, 0] * H[1, 1] - H[0, 1] * H[1, 0]
        roots = np.roots([c2, c1, c0])
        S, Tt, alpha, beta = solve(H, T)
        assert match(alpha / beta, roots) <= 1e-12 * max(1.0, np.abs(roots).max())


@pytest.mark.parametrize("m", [21, 22, 23])
def test_qz_planted_mistakes_are_caught(m):
    H, T = pencil(24, 4242, (5,))
    oracle.set_mutation(m)
    try:
        caught = False
        try:
            S, Tt, Q, Z, alpha, beta, info = oracle.qz(H, T, itmax=8 * 24)
            n = H.shape[0]
            ok = (info == 0
                  and np.linalg.norm(Q.T @ H @ Z - S) <= 100 * n * U * np.linalg.norm(H)
                  and np.linalg.norm(Q.T @ T @ Z - Tt) <= 100 * n * U * np.linalg.norm(T)
                  and np.all(np.tril(Tt, -1) == 0.0))
            if ok:
                ref, ninf = reference(H, T)
                lam = alpha[beta > 0] / beta[beta > 0]
                ok = (int((beta == 0).sum()) == ninf and len(lam) == len(ref)
                      and match(lam, ref) <= 1e-8 * max(1.0, np.abs(ref).max()))
            caught = not ok
        except AssertionError:
            caught = True
        assert caught, f"mutation {m} not caught"
    finally:
        oracle.set_mutation(0)
