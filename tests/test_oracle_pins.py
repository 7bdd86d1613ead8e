"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

The oracle (oracle/hqr_oracle.c) is trusted only through these tests:
closed forms (2x2 eigenvalues, tridiagonal Toeplitz spectra), brute force
(exact characteristic polynomials for n <= 6, roots at 50 digits), prescribed
spectra, invariants (trace, Frobenius norm), special cases (triangular and
zero-subdiagonal inputs), independent libraries (LAPACK through scipy:
eigenvalues, dtrexc block swaps), and the implicit-Q theorem for one sweep.
The mutation tests at the end plant mistakes in the oracle and check that
each is caught by one of these pins.
"""
import cmath
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla
import sympy

import hqr_inputs as hi
import oracle
from tests import checks

U = 2.0 ** -52


def schur_ok(H, T, Q, w, n_u=100):
    n = H.shape[0]
    ok, msg = checks.structure_ok(T, w)
    assert ok, msg
    assert checks.rel_backward(H, T, Q) <= n_u * max(n, 1) * U
    assert checks.orth(Q) <= n_u * max(n, 1) * U


# --------------------------------------------------------------------- 2x2

def closed_form_2x2(a, b, c, d):
    m = (a + d) / 2
    r = cmath.sqrt(((a - d) / 2) ** 2 + b * c)
    return np.array([m + r, m - r])


CASES_2x2 = [
    (1.0, 2.0, 3.0, 4.0),       # real distinct
    (1.0, -5.0, 2.0, 1.0),      # complex, equal diagonal
    (0.3, -2.0, 1.5, -0.7),     # complex
    (2.0, 0.0, 1.0, 5.0),       # b = 0
    (2.0, 7.0, 0.0, 5.0),       # c = 0 (already triangular)
    (1.0, 1e-8, -1e-8, 1.0),    # tiny complex pair
    (4.0, 1.0, 1e-12, 4.0),     # nearly double real
    (-3.0, 2.0, -2.0, 1.0),     # complex with unequal diagonal
]


@pytest.mark.parametrize("blk", CASES_2x2)
def test_std2x2_closed_form(blk):
    a, b, c, d = blk
    B = np.array([[a, b], [c, d]])
    Bn, cs, sn, cplx = oracle.std2x2(B)
    G = np.array([[cs, -sn], [sn, cs]])
    assert abs(cs * cs + sn * sn - 1) < 4 * U
    assert np.linalg.norm(G.T @ B @ G - Bn) <= 8 * U * np.linalg.norm(B)
    ref = closed_form_2x2(a, b, c, d)
    if cplx:
        assert Bn[0, 0] == Bn[1, 1] and Bn[0, 1] * Bn[1, 0] < 0
        w = Bn[0, 0] + 1j * np.sqrt(abs(Bn[0, 1])) * np.sqrt(abs(Bn[1, 0]))
        got = np.array([w, np.conj(w)])
    else:
        assert Bn[1, 0] == 0.0
        got = np.array([Bn[0, 0], Bn[1, 1]], dtype=complex)
    _, _, dist = checks.match(got, ref)
    assert dist.max() <= 1e-14 * max(1.0, np.abs(B).max()) + 1e-7 * np.sqrt(abs(b * c)) * (abs(b * c) < 1e-20)


@pytest.mark.parametrize("blk", CASES_2x2)
def test_schur_n2_closed_form(blk):
    H = np.array([[blk[0], blk[1]], [blk[2], blk[3]]], order="F")
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0
    schur_ok(H, T, Q, w)
    _, _, dist = checks.match(w, closed_form_2x2(*blk))
    assert dist.max() <= 1e-13 * max(1.0, np.abs(H).max())


# --------------------------------------------------------- brute force n<=6

def exact_roots(Hq):
    """Roots of det(xI - H) from the exact rational characteristic polynomial."""
    M = sympy.Matrix(Hq)
    x = sympy.Symbol("x")
    coeffs = [sympy.Rational(c) for c in M.charpoly(x).all_coeffs()]
    mpmath.mp.dps = 50
    rts = mpmath.polyroots([mpmath.mpf(c.p) / c.q for c in coeffs], maxsteps=400, extraprec=400)
    return np.array([complex(r) for r in rts])


@pytest.mark.parametrize("n", [3, 4, 5, 6])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bruteforce_charpoly(n, seed):
    g = np.random.default_rng(1000 * n + seed)
    Hq = [[Fraction(int(g.integers(-8, 9)), 4) if i <= j + 1 else Fraction(0) for j in range(n)]
          for i in range(n)]
    for k in range(n - 1):
        if Hq[k + 1][k] == 0:
            Hq[k + 1][k] = Fraction(1, 2)
    H = np.array([[float(v) for v in row] for row in Hq], order="F")
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0
    schur_ok(H, T, Q, w)
    ref = exact_roots(Hq)
    lam, kap = checks.eig_condition(H)
    _, _, dist = checks.match(w, ref)
    kmax = min(np.max(kap), 1e8)
    assert dist.max() <= 1e-13 * kmax * max(1.0, np.linalg.norm(H)), (dist.max(), kmax)


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n,a,b,c", [(60, 2.0, 1.0, 1.0), (61, -1.0, 1.0, -1.0), (200, 0.5, 1.0, 1.0),
                                     (257, 3.0, 1.0, -1.0), (400, 1.0, 1.0, -1.0)])
def test_toeplitz_tridiagonal(n, a, b, c):
    H, ev = hi.toeplitz_tridiagonal(n, a, b, c)
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0
    schur_ok(H, T, Q, w)
    _, _, dist = checks.match(w, ev)
    assert dist.max() <= 50 * n * U * np.linalg.norm(H)


@pytest.mark.parametrize("n", [100, 256])
def test_prescribed_normal_spectrum(n):
    H, ev = hi.prescribed_hessenberg(n, seed=2020 + n)
    T, Q, w, info, st = oracle.schur(H)
    assert info == 0
    schur_ok(H, T, Q, w)
    _, _, dist = checks.match(w, ev)
    assert dist.max() <= 10 * n * U * np.linalg.norm(H)
    # invariants of an orthogonal similarity
    assert abs(np.sum(w).real - np.trace(H)) <= 10 * n * U * np.abs(np.diag(H)).sum() + 1e-12
    assert abs(np.linalg.norm(T) - np.linalg.norm(H)) <= 10 * n * U * np.linalg.norm(H)
    # normal matrix: sum |lambda|^2 = ||H||_F^2
    assert abs(np.sum(np.abs(w) ** 2) - np.linalg.norm(H) ** 2) <= 100 * n * U * np.linalg.norm(H) ** 2


def test_syn_matrix_known_spectrum():
    H, ev = hi.syn_matrix(200, seed=3)
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0
    schur_ok(H, T, Q, w)
    lam, kap = checks.eig_condition(H)
    r, c, dist = checks.match(w, ev)
    r2, c2, _ = checks.match(ev, lam)
    kap_e = np.empty(len(ev))
    kap_e[r2] = kap[c2]
    assert np.all(dist <= 1e-12 * kap_e[c] * np.linalg.norm(H))


@pytest.mark.parametrize("n,gen", [(150, "gauss"), (300, "hessrand"), (500, "hessrand")])
def test_against_lapack_eigenvalues(n, gen):
    H = hi.gaussian_hessenberg(n, seed=n) if gen == "gauss" else hi.hessrand(n, seed=n)
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0
    schur_ok(H, T, Q, w)
    lam, kap = checks.eig_condition(H)
    r, c, dist = checks.match(w, lam)
    assert np.all(dist <= 1e-11 * np.maximum(kap[c], 1.0) * np.linalg.norm(H))


def test_trace_and_square_trace_invariants():
    H = hi.hessrand(220, seed=9)
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0
    s = np.sum(w)
    assert abs(s.imag) <= 1e-9 and abs(s.real - np.trace(H)) <= 1e-10 * np.abs(H).sum()
    s2 = np.sum(w ** 2)
    assert abs(s2.real - np.trace(H @ H)) <= 1e-10 * np.linalg.norm(H) ** 2


# ----------------------------------------------------------- special cases

def test_triangular_input_unchanged():
    g = np.random.default_rng(4)
    H = np.asfortranarray(np.triu(g.standard_normal((40, 40))))
    T, Q, w, info, st = oracle.schur(H)
    assert info == 0
    assert np.array_equal(T, H) and np.array_equal(Q, np.eye(40))
    assert np.array_equal(w.real, np.diag(H)) and np.all(w.imag == 0)


def test_standardized_quasi_triangular_unchanged():
    g = np.random.default_rng(5)
    n = 30
    T0 = np.triu(g.standard_normal((n, n)))
    for k in range(0, n - 1, 5):
        T0[k + 1, k + 1] = T0[k, k]
        T0[k, k + 1] = abs(T0[k, k + 1]) + 0.5
        T0[k + 1, k] = -0.75
    H = np.asfortranarray(T0)
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0
    assert np.array_equal(T, H) and np.array_equal(Q, np.eye(n))


@pytest.mark.parametrize("n", [1, 2])
def test_tiny_orders(n):
    H = np.asfortranarray(np.array([[3.0, 1.0], [-2.0, 0.5]])[:n, :n])
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0
    schur_ok(H, T, Q, w)
    _, _, d = checks.match(w, np.linalg.eigvals(H))
    assert d.max() < 1e-14 * 4


def test_zero_matrix():
    H = np.zeros((9, 9), order="F")
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0 and np.all(T == 0) and np.all(w == 0)


def test_zero_subdiagonal_splits_spectrum():
    H = hi.hessrand(180, seed=21)
    H[90, 89] = 0.0
    T, Q, w, info, _ = oracle.schur(H)
    assert info == 0
    schur_ok(H, T, Q, w)
    ref = np.concatenate([np.linalg.eigvals(H[:90, :90]), np.linalg.eigvals(H[90:, 90:])])
    lam, kap = checks.eig_condition(H)
    _, c, d = checks.match(w, ref)
    assert d.max() <= 1e-9


def test_nonfinite_rejected():
    H = hi.hessrand(10, seed=1)
    H[3, 5] = np.nan
    _, _, _, info, _ = oracle.schur(H)
    assert info == -1


def test_iteration_limit_reports_failure():
    H = hi.hessrand(120, seed=2)
    T, Q, w, info, _ = oracle.schur(H, itmax=1)
    assert info > 0


# ------------------------------------------------------- sweep: implicit Q

def shifted_first_column(H, shifts):
    n = H.shape[0]
    v = np.zeros(n)
    v[0] = 1.0
    s = list(shifts)
    for j in range(0, len(s), 2):
        s1, s2 = s[j], s[j + 1]
        # (H - s1)(H - s2) v, real for a conjugate pair or two reals
        v = H @ (H @ v) - (s1 + s2).real * (H @ v) + (s1 * s2).real * v
        v /= np.linalg.norm(v)
    return v


@pytest.mark.parametrize("nsh", [2, 4, 8])
def test_sweep_first_column_implicit_q(nsh):
    n = 24
    H = hi.hessrand(n, seed=31 + nsh)
    g = np.random.default_rng(nsh)
    shifts = []
    for j in range(nsh // 2):
        if j % 2 == 0:
            z = complex(g.uniform(-2, 2), g.uniform(0.5, 2))
            shifts += [z, np.conj(z)]
        else:
            shifts += [complex(g.uniform(-2, 2)), complex(g.uniform(-2, 2))]
    # bulge j uses shifts (2j, 2j+1)
    Hn, Qn = oracle.sweep(H, np.eye(n), 0, n - 1, shifts)
    assert np.all(np.tril(Hn, -2) == 0.0)
    assert np.linalg.norm(Qn.T @ H @ Qn - Hn) <= 100 * n * U * np.linalg.norm(H)
    p = shifted_first_column(H, shifts)
    assert abs(abs(Qn[:, 0] @ p) - 1.0) <= 1e-12
    # implicit Q: Q is the Arnoldi basis of K(H, p) up to column signs
    V = np.zeros((n, n))
    V[:, 0] = p
    for k in range(1, n):
        w = H @ V[:, k - 1]
        for _ in range(2):
            w -= V[:, :k] @ (V[:, :k].T @ w)
        V[:, k] = w / np.linalg.norm(w)
    kk = 12  # leading columns, before the Krylov sequence loses accuracy
    assert np.max(np.abs(np.abs(np.sum(V[:, :kk] * Qn[:, :kk], axis=0)) - 1.0)) <= 1e-9


# --------------------------------------------------- swaps against dtrexc

def block_upper(sizes, seed):
    g = np.random.default_rng(seed)
    n = sum(sizes)
    T = np.triu(g.standard_normal((n, n)))
    k = 0
    for s in sizes:
        if s == 2:
            a = g.uniform(-2, 2)
            T[k, k] = T[k + 1, k + 1] = a
            T[k, k + 1] = g.uniform(0.5, 2)
            T[k + 1, k] = -g.uniform(0.5, 2)
        k += s
    return np.asfortranarray(T)


@pytest.mark.parametrize("p,q", [(1, 1), (1, 2), (2, 1), (2, 2)])
def test_swap_matches_lapack_dtrexc(p, q):
    sizes = [1, p, q, 1]
    T = block_upper(sizes, seed=10 * p + q)
    n = T.shape[0]
    Tn, Qn, rc = oracle.swap(T, np.eye(n), 1, p, q)
    assert rc == 0
    assert np.linalg.norm(Qn.T @ T @ Qn - Tn) <= 50 * U * np.linalg.norm(T)
    assert checks.orth(Qn) <= 50 * U
    ok, msg = checks.structure_ok(Tn)
    assert ok, msg
    # LAPACK moves the block at 1-based position 2+p to position 2
    Tl, Ql, info = sla.lapack.dtrexc(T.copy(order="F"), np.eye(n, order="F"), 2 + p, 2)[:3]
    assert info == 0
    ev_o = np.linalg.eigvals(Tn[1:1 + q, 1:1 + q])
    ev_l = np.linalg.eigvals(Tl[1:1 + q, 1:1 + q])
    _, _, d = checks.match(ev_o, ev_l)
    assert d.max() <= 1e-12
    ev_orig = np.linalg.eigvals(T[1 + p:1 + p + q, 1 + p:1 + p + q])
    _, _, d2 = checks.match(ev_o, ev_orig)
    assert d2.max() <= 1e-12


def test_forced_swap_rejection_keeps_a_valid_schur_form():
    # failure forcing: every swap is refused, so each AED halts at its first
    # undeflatable candidate; the result must still be a valid Schur form
    H, ev = hi.prescribed_hessenberg(200, seed=77)
    oracle.force_swap_failure(True)
    try:
        T, Q, w, info, st = oracle.schur(H)
    finally:
        oracle.force_swap_failure(False)
    assert info == 0
    schur_ok(H, T, Q, w)
    _, _, d = checks.match(w, ev)
    assert d.max() <= 1e-10 * np.linalg.norm(H)
    Tn, Qn, rc = oracle.swap(block_upper([1, 2, 1], 3), np.eye(4), 0, 1, 2)
    assert rc == 0


# ------------------------------------------------------------------- AED

def test_aed_window_with_zero_coupling_deflates_all():
    H = hi.hessrand(120, seed=41)
    H[80, 79] = 0.0
    Hn, Qn, nd, cands = oracle.aed(H, np.eye(120), 0, 119, 40)
    assert nd == 40 and len(cands) == 0
    assert np.linalg.norm(Qn.T @ H @ Qn - Hn) <= 200 * U * np.linalg.norm(H)
    ok, _ = checks.structure_ok(Hn[80:, 80:])
    assert ok


def test_aed_preserves_spectrum_and_hessenberg_form():
    H, ev = hi.prescribed_hessenberg(160, seed=43)
    Hn, Qn, nd, cands = oracle.aed(H, np.eye(160), 0, 159, 48)
    assert np.all(np.tril(Hn, -2) == 0.0)
    assert np.linalg.norm(Qn.T @ H @ Qn - Hn) <= 500 * U * np.linalg.norm(H)
    assert len(cands) == 48 - nd
    # the candidates are eigenvalues of the window's undeflated Schur part and
    # the deflated ones are eigenvalues of H (normal matrix: kappa = 1)
    k = 160 - nd
    if nd > 0:
        dev = np.linalg.eigvals(Hn[k:, k:])
        _, _, d = checks.match(dev, ev[checks.match(dev, ev)[1]])
        assert d.max() <= 1e-10 * np.linalg.norm(H)


# ---------------------------------------------------------------- gradient

def loss_and_cotangent(w):
    """L = sum softplus(Re l) + 0.1 |l|^2 and g = dL/dRe + i dL/dIm."""
    re = w.real
    L = np.sum(np.logaddexp(0.0, re)) + 0.1 * np.sum(np.abs(w) ** 2)
    g = 1.0 / (1.0 + np.exp(-re)) + 0.2 * w
    return L, g


def loss_of(H):
    T, Q, w, info, _ = oracle.schur(H, want_q=False)
    assert info == 0
    return loss_and_cotangent(w)[0]


def hess_direction(n, g):
    D = np.triu(g.standard_normal((n, n)), -1)
    return D / np.linalg.norm(D)


def test_gradient_of_trace_is_identity():
    H = hi.hessrand(30, seed=50)
    T, Q, w, info, _ = oracle.schur(H)
    dH = oracle.eig_backward(T, Q, w, np.ones(30))
    assert np.abs(dH - np.eye(30)).max() <= 1e-10


def test_gradient_of_trace_square():
    H = hi.hessrand(25, seed=51)
    T, Q, w, info, _ = oracle.schur(H)
    dH = oracle.eig_backward(T, Q, w, 2.0 * np.conj(w))
    ref = np.triu(2.0 * H.T, -1)
    assert np.abs(dH - ref).max() <= 1e-8 * np.abs(ref).max()


def test_gradient_normal_sum_abs_square():
    H, ev = hi.prescribed_hessenberg(40, seed=52, separated=True)
    T, Q, w, info, _ = oracle.schur(H)
    dH = oracle.eig_backward(T, Q, w, 2.0 * w, hess_mask=False)
    assert np.abs(dH - 2.0 * H).max() <= 1e-9 * np.abs(H).max()


@pytest.mark.parametrize("kind", ["normal", "nonnormal"])
def test_gradient_central_differences(kind):
    n = 24
    if kind == "normal":
        H, _ = hi.prescribed_hessenberg(n, seed=53, separated=True)
    else:
        H, _ = hi.syn_matrix(n, seed=54)
    T, Q, w, info, _ = oracle.schur(H)
    _, g = loss_and_cotangent(w)
    dH = oracle.eig_backward(T, Q, w, g)
    gen = np.random.default_rng(55)
    h = 1e-6
    for _ in range(6):
        D = hess_direction(n, gen)
        fd = (loss_of(H + h * D) - loss_of(H - h * D)) / (2 * h)
        an = np.sum(dH * D)
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)


# -------------------------------------------------------------- mutations

def _catch(fn):
    try:
        fn()
    except AssertionError:
        return True
    return False


MUTATION_PINS = {
    1: lambda: test_sweep_first_column_implicit_q(4),
    2: lambda: test_prescribed_normal_spectrum(100),
    3: lambda: test_prescribed_normal_spectrum(256),
    4: lambda: test_swap_matches_lapack_dtrexc(1, 1),
    5: lambda: test_schur_n2_closed_form(CASES_2x2[1]),
    6: lambda: test_prescribed_normal_spectrum(256),
    7: lambda: test_gradient_central_differences("nonnormal"),
    8: lambda: test_against_lapack_eigenvalues(300, "hessrand"),
}


@pytest.mark.parametrize("m", sorted(MUTATION_PINS))
def test_planted_mistake_is_caught(m):
    oracle.set_mutation(m)
    try:
        caught = _catch(MUTATION_PINS[m])
    finally:
        oracle.set_mutation(0)
    assert caught, f"mutation {m} was not caught by its pin"
