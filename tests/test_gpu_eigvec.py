"""GPU tests of the eigenvector phase (hqr_eigenvectors): right eigenvectors
of H from its GPU Schur form, checked by their residuals ||H x - lambda x||
(within 100 n u ||H|| kappa-free bound on each unit vector's residual), their
normalization (unit 2-norm, largest component real and positive) and, for
well-conditioned eigenvalues, their direction against scipy.linalg.eig."""
import sys

import numpy as np
import pytest
import scipy.linalg as sla

import hqr_inputs as hi
from tests import checks

pytestmark = pytest.mark.gpu
U = 2.0 ** -52


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kind,n", [("prescribed", 1), ("prescribed", 2), ("prescribed", 40), ("syn", 60),
                                    ("hessrand", 200), ("prescribed", 500)])
def test_eigenvectors(gpu, kind, n):
    import torch
    import paper_2007_03576_amd as hq
    _say(f"case eigenvectors {kind} n={n}")
    if kind == "prescribed":
        H = hi.gaussian_hessenberg(n, seed=3) if n < 4 else hi.prescribed_hessenberg(n, seed=n)[0]
    elif kind == "syn":
        H = hi.syn_matrix(n, seed=n)[0]
    else:
        H = hi.hessrand(n, seed=n)
    T, Q, w, info = hq.schur(torch.from_numpy(np.ascontiguousarray(H)).cuda())
    assert info == 0
    V = hq.eigenvectors(T, Q, w)
    torch.cuda.synchronize()
    V, w = V.cpu().numpy(), w.cpu().numpy()
    hn = np.linalg.norm(H)
    res = np.linalg.norm(H @ V - V * w[None, :], axis=0)
    _say(f"  worst residual {res.max() / (U * hn):.1f} u ||H||")
    assert np.all(res <= 100 * n * U * hn)
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0, atol=1e-12)
    k = np.argmax(np.abs(V), axis=0)
    lead = V[k, np.arange(n)]
    assert np.all(np.abs(lead.imag) <= 1e-14) and np.all(lead.real > 0)
    lam, kap = checks.eig_condition(H)
    ws, Vs = sla.eig(H)
    r, c, d = checks.match(w, ws)
    for i, j in zip(r, c):
        if kap[np.argmin(np.abs(lam - w[i]))] < 1e3 and np.sum(np.abs(ws - ws[j]) < 1e-6) == 1:
            # same direction up to a unit complex factor
            assert abs(abs(np.vdot(Vs[:, j] / np.linalg.norm(Vs[:, j]), V[:, i])) - 1.0) <= 1e-8
