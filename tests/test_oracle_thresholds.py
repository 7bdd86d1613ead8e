"""Pins of the oracle's deflation and swap-acceptance thresholds.

Each threshold is pinned from both sides: inputs are built so that the tested
quantity sits 1 % below and 1 % above the threshold the paper states
(Sec. 5.6 "Comment regarding the deflation conditions and the accuracy",
items 1-3; the swap stability test of Bai and Demmel cited in Sec. 2.5), and
the outcome must flip exactly there.  Swap rejections are pinned to LAPACK's
dtrexc (an independent implementation of the same test), and a planted
mistake in each threshold must be caught.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import hqr_inputs as hi
import oracle
from tests import checks

U = 2.0 ** -52
DBL_MIN = 2.0 ** -1022
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def smlnum(n):
    return DBL_MIN * (n / U)


# ------------------------------------------------- AED spike test, item 1

def aed_1x1(t, s, mode=0, thold=0.0, a=2.0, b=1.5):
    """n = 2, AED window of order 1 holding [t]; the spike is exactly s."""
    H = np.array([[a, b], [s, t]])
    Hn, _, nd, _ = oracle.aed(H, np.eye(2), 0, 1, 1, defl_mode=mode, defl_thold=thold)
    return nd, Hn


def aed_2x2(a, b, c, s, mode=0, thold=0.0):
    """n = 3, AED window of order 2 holding the standardized block
    [[a, b], [c, a]] (b c < 0, left as is by the window's Schur solve); the
    spike is exactly (s, 0)."""
    H = np.array([[1.25, -0.5, 0.75], [s, a, b], [0.0, c, a]])
    Hn, _, nd, _ = oracle.aed(H, np.eye(3), 0, 2, 2, defl_mode=mode, defl_thold=thold)
    return nd, Hn


@pytest.mark.parametrize("t", [3.7, -1e5, 2.0 ** -30])
def test_aed_1x1_threshold_is_u_times_diagonal(t):
    thr = U * abs(t)
    nd, Hn = aed_1x1(t, 0.99 * thr)
    assert nd == 1 and Hn[1, 0] == 0.0
    nd, Hn = aed_1x1(t, 1.01 * thr)
    assert nd == 0 and Hn[1, 0] == 1.01 * thr


def test_aed_1x1_floor_is_smlnum():
    # t = 0: the relative part vanishes and smlnum = nu n / u decides
    nd, _ = aed_1x1(0.0, 0.99 * smlnum(2))
    assert nd == 1
    nd, _ = aed_1x1(0.0, 1.01 * smlnum(2))
    assert nd == 0


@pytest.mark.parametrize("a,b,c", [(3.0, 4.0, -1.0), (-0.5, 0.01, -900.0), (7.0, -2.0, 8.0)])
def test_aed_2x2_threshold_is_u_times_hhat(a, b, c):
    # h^ = sqrt|t_kk t_k-1,k-1| + sqrt|t_k-1,k t_k,k-1| as printed in item 1
    hhat = np.sqrt(abs(a * a)) + np.sqrt(abs(b * c))
    nd, Hn = aed_2x2(a, b, c, 0.99 * U * hhat)
    assert nd == 2 and Hn[1, 0] == 0.0
    nd, Hn = aed_2x2(a, b, c, 1.01 * U * hhat)
    assert nd == 0


# ------------------------------------- norm-stable and fixed, items 2 and 3

@pytest.mark.parametrize("t", [12.0, -0.25])
def test_norm_stable_aed_1x1_threshold(t):
    # ||H||_F of the Hessenberg part, not max |h_ij| (a=3, b=4, t=12: 13 vs 12)
    H = np.array([[3.0, 4.0], [0.0, t]])
    thr = U * np.linalg.norm(H)
    nd, _ = aed_1x1(t, 0.99 * thr, mode=1, a=3.0, b=4.0)
    assert nd == 1
    nd, _ = aed_1x1(t, 1.01 * thr, mode=1, a=3.0, b=4.0)
    assert nd == 0


def test_norm_stable_aed_2x2_needs_both_spike_entries():
    a, b, c = 3.0, 4.0, -1.0
    H = np.array([[1.25, -0.5, 0.75], [0.0, a, b], [0.0, c, a]])
    thr = U * np.linalg.norm(H)
    nd, _ = aed_2x2(a, b, c, 0.99 * thr, mode=1)
    assert nd == 2
    # the spike is (s, 0): only its upper entry is above the threshold
    nd, _ = aed_2x2(a, b, c, 1.01 * thr, mode=1)
    assert nd == 0


@pytest.mark.parametrize("thold", [1e-6, 0.5])
def test_fixed_aed_thresholds(thold):
    nd, _ = aed_1x1(3.7, 0.99 * thold, mode=2, thold=thold)
    assert nd == 1
    nd, _ = aed_1x1(3.7, 1.01 * thold, mode=2, thold=thold)
    assert nd == 0
    nd, _ = aed_2x2(3.0, 4.0, -1.0, 0.99 * thold, mode=2, thold=thold)
    assert nd == 2
    nd, _ = aed_2x2(3.0, 4.0, -1.0, 1.01 * thold, mode=2, thold=thold)
    assert nd == 0


def split_at_start(mode, thold, f, n=30, k=15, seed=21):
    """Sets h_{k,k-1} to f times the threshold and reports whether the solver
    decoupled the matrix there before any transformation crossed row k: then
    Q stays block diagonal exactly."""
    H = hi.hessrand(n, seed=seed)
    if mode == 1:
        H[k, k - 1] = 0.0
        thr = U * np.linalg.norm(H)  # the entry itself changes ||H||_F by O(u^2)
    else:
        thr = thold
    H[k, k - 1] = f * thr
    T, Q, w, info, _ = oracle.schur(H, defl_mode=mode, defl_thold=thold)
    assert info == 0
    checks_ok, msg = checks.structure_ok(T, w)
    assert checks_ok, msg
    return bool(np.all(Q[k:, :k] == 0.0) and np.all(Q[:k, k:] == 0.0))


@pytest.mark.parametrize("mode,thold", [(1, 0.0), (2, 1e-7), (2, 1e-3)])
def test_vigilant_threshold_of_norm_stable_and_fixed(mode, thold):
    assert split_at_start(mode, thold, 0.99)
    assert not split_at_start(mode, thold, 1.01)


@pytest.mark.parametrize("mode,thold", [(1, 0.0), (2, 1e-12)])
@pytest.mark.parametrize("gen", ["hessrand", "syn"])
def test_full_solve_under_other_conditions(mode, thold, gen):
    # the looser conditions still give a Schur form of a nearby matrix
    n = 180
    if gen == "hessrand":
        H = hi.hessrand(n, seed=61)
    else:
        H, _ = hi.syn_matrix(n, seed=62)
    T, Q, w, info, st = oracle.schur(H, defl_mode=mode, defl_thold=thold)
    assert info == 0
    ok, msg = checks.structure_ok(T, w)
    assert ok, msg
    assert checks.rel_backward(H, T, Q) <= 100 * n * U
    assert checks.orth(Q) <= 100 * n * U
    lam, kap = checks.eig_condition(H)
    _, c, d = checks.match(w, lam)
    assert np.all(d <= 1e-10 * np.maximum(kap[c], 1.0) * np.linalg.norm(H))


def test_bad_deflation_mode_rejected():
    H = hi.hessrand(8, seed=1)
    assert oracle.schur(H, defl_mode=3)[3] == -12
    assert oracle.schur(H, defl_mode=2, defl_thold=-1.0)[3] == -12


# ----------------------------------------------- swap acceptance threshold

def std_block(a, w, r):
    return np.array([[a, w * r], [-w / r, a]])


def lapack_rejected_swaps(count, seed=0):
    """Seeded 2x2/2x2 exchanges with nearly equal eigenvalues and large
    coupling that LAPACK's dtrexc refuses (info = 1)."""
    g = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        T = np.zeros((4, 4))
        a = g.uniform(-1, 1)
        T[:2, :2] = std_block(a, 10 ** g.uniform(-10, 0), 10 ** g.uniform(-4, 4))
        T[2:, 2:] = std_block(a + 10 ** g.uniform(-12, -2) * g.standard_normal(), 10 ** g.uniform(-10, 0),
                              10 ** g.uniform(-4, 4))
        T[:2, 2:] = g.standard_normal((2, 2)) * 10 ** g.uniform(0, 10)
        if sla.lapack.dtrexc(np.asfortranarray(T), np.eye(4, order="F"), 3, 1)[-1] == 1:
            out.append(T)
    return out


def test_natural_swap_rejection_matches_lapack():
    oracle.swap_rejections(reset=True)
    cases = lapack_rejected_swaps(4)
    for T in cases:
        Tn, Qn, rc = oracle.swap(T, np.eye(4), 0, 2, 2)
        assert rc == 1
        assert np.array_equal(Tn, T) and np.array_equal(Qn, np.eye(4))  # untouched
    assert oracle.swap_rejections(reset=True) == len(cases)


def test_well_conditioned_swaps_with_large_norm_accepted():
    # ||D|| up to 1e6: the threshold 10 u ||D||_max, not 10 u, must apply
    g = np.random.default_rng(1)
    for _ in range(40):
        T = np.zeros((4, 4))
        T[:2, :2] = std_block(g.uniform(-1, 1), g.uniform(0.5, 2), g.uniform(0.5, 2))
        T[2:, 2:] = std_block(g.uniform(2, 3), g.uniform(0.5, 2), g.uniform(0.5, 2))
        T[:2, 2:] = g.standard_normal((2, 2)) * 10 ** g.uniform(2, 6)
        assert sla.lapack.dtrexc(np.asfortranarray(T), np.eye(4, order="F"), 3, 1)[-1] == 0
        Tn, Qn, rc = oracle.swap(T, np.eye(4), 0, 2, 2)
        assert rc == 0
        assert np.linalg.norm(Qn.T @ T @ Qn - Tn) <= 50 * U * np.linalg.norm(T)


def rejection_case():
    W = np.loadtxt(os.path.join(GOLDEN, "aed_rejection_window.txt"))
    g = np.random.default_rng(7)
    n = 20
    H = np.triu(g.standard_normal((n, n)), -1)
    H[12:, :12] = 0.0
    H[12, 11] = 1.0
    H[12:, 12:] = np.triu(W, -1)
    return H


def test_natural_rejection_halts_aed_with_a_valid_schur_form():
    # no force hook: the window's reordering meets a swap the stability test
    # refuses; the AED halts there (Sec. 3.5, failed swaps) and the solve
    # still ends in a valid Schur form of a nearby matrix
    H = rejection_case()
    n = H.shape[0]
    oracle.swap_rejections(reset=True)
    T, Q, w, info, st = oracle.schur(H, nw=8, ns=4, nmin=12)
    assert oracle.swap_rejections(reset=True) >= 1
    assert info == 0
    ok, msg = checks.structure_ok(T, w)
    assert ok, msg
    assert checks.rel_backward(H, T, Q) <= 100 * n * U
    assert checks.orth(Q) <= 100 * n * U
    lam, kap = checks.eig_condition(H)
    _, c, d = checks.match(w, lam)
    assert np.all(d <= 1e-10 * np.maximum(kap[c], 1.0) * np.linalg.norm(H))


# -------------------------------------------------------------- mutations

def _caught(fn):
    try:
        fn()
    except AssertionError:
        return True
    return False


MUTATION_PINS = {
    9: lambda: test_aed_2x2_threshold_is_u_times_hhat(3.0, 4.0, -1.0),
    10: lambda: test_aed_2x2_threshold_is_u_times_hhat(3.0, 4.0, -1.0),
    11: test_well_conditioned_swaps_with_large_norm_accepted,
    12: test_norm_stable_aed_2x2_needs_both_spike_entries,
    13: lambda: test_norm_stable_aed_1x1_threshold(12.0),
}


@pytest.mark.parametrize("m", sorted(MUTATION_PINS))
def test_planted_threshold_mistake_is_caught(m):
    oracle.set_mutation(m)
    try:
        caught = _caught(MUTATION_PINS[m])
    finally:
        oracle.set_mutation(0)
    assert caught, f"mutation {m} was not caught by its pin"
