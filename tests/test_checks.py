"""The test helpers that decide parity are pinned too: condition numbers from
a quasi-triangular Schur form (used where scipy's eig would be too slow)
against scipy.linalg.eig's left/right eigenvectors, on normal and non-normal
matrices with real and complex eigenvalues."""
import numpy as np
import pytest

import hqr_inputs as hi
import oracle
from tests import checks


@pytest.mark.parametrize("kind,n", [("syn", 6), ("syn", 40), ("syn", 150), ("gauss", 120), ("normal", 64)])
def test_schur_eig_condition_matches_scipy(kind, n):
    if kind == "syn":
        H, _ = hi.syn_matrix(n, seed=n)
    elif kind == "gauss":
        H = hi.gaussian_hessenberg(n, seed=n)
    else:
        H, _ = hi.prescribed_hessenberg(n, seed=n)
    T, _, _, info, _ = oracle.schur(H, want_q=False)
    assert info == 0
    lam, kap = checks.schur_eig_condition(T)
    lam2, kap2 = checks.eig_condition(H)
    r, c, d = checks.match(lam, lam2)
    assert d.max() <= 1e-6 * max(1.0, np.abs(lam2).max())
    ok = kap2[c] < 1e8  # both computations are exact enough there
    assert np.all(np.abs(kap[r][ok] - kap2[c][ok]) <= 1e-6 * kap2[c][ok])
    if kind == "normal":
        assert np.all(np.abs(kap - 1.0) <= 1e-8)
