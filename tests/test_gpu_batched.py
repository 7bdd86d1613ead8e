"""GPU parity tests of hqr_schur_batched (uneven sizes, LDS and global-memory
tiers) against the oracle, per matrix: eigenvalues (kappa-scaled), backward
error, orthogonality, standardized quasi-triangular structure."""
import sys

import numpy as np
import pytest

import hqr_inputs as hi
import oracle
from tests import checks

pytestmark = pytest.mark.gpu
U = 2.0 ** -52


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def check_one(H, T, Q, w, info, tag):
    n = H.shape[0]
    assert info == 0, f"{tag}: info {info}"
    ok, msg = checks.structure_ok(T, w)
    assert ok, f"{tag}: {msg}"
    assert checks.rel_backward(H, T, Q) <= 100 * max(n, 1) * U, tag
    assert checks.orth(Q) <= 100 * max(n, 1) * U, tag
    _, _, wo, oi, _ = oracle.schur(H, want_q=False)
    assert oi == 0
    lam, kap = checks.eig_condition(H)
    r, c, d = checks.match(w, wo)
    r2, c2, _ = checks.match(wo, lam)
    kap_o = np.empty(n)
    kap_o[r2] = kap[c2]
    tol = 1e-10 * np.maximum(kap_o[c], 1.0) * max(np.linalg.norm(H), 1.0)
    assert np.all(d <= tol), f"{tag}: eigenvalue mismatch"


@pytest.mark.parametrize("lo,hi_,count,seed", [(1, 12, 30, 1), (16, 96, 40, 2), (90, 200, 16, 3)])
def test_batched_uneven_sizes(gpu, lo, hi_, count, seed):
    import torch
    import paper_2007_03576_amd as hq
    _say(f"case batched sizes {lo}..{hi_} count {count}")
    sizes = hi.batched_sizes(count, lo, hi_, seed=seed)
    mats = [hi.gaussian_hessenberg(int(n), seed=seed * 1000 + i) for i, n in enumerate(sizes)]
    dev = [torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats]
    Ts, Qs, ws, info = hq.schur_batched(dev)
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    for i, H in enumerate(mats):
        check_one(H, Ts[i].cpu().numpy(), Qs[i].cpu().numpy(), ws[i].cpu().numpy(), int(info[i]), f"m{i} n={H.shape[0]}")


def test_batched_prescribed_spectra(gpu):
    import torch
    import paper_2007_03576_amd as hq
    _say("case batched prescribed spectra n=64,128,160")
    mats, evs = [], []
    for i, n in enumerate([64, 128, 160]):
        H, ev = hi.prescribed_hessenberg(n, seed=300 + i)
        mats.append(H)
        evs.append(ev)
    Ts, Qs, ws, info = hq.schur_batched([torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats])
    for i, H in enumerate(mats):
        w = ws[i].cpu().numpy()
        _, _, d = checks.match(w, evs[i])
        assert d.max() <= 1e-10 * np.linalg.norm(H)
        check_one(H, Ts[i].cpu().numpy(), Qs[i].cpu().numpy(), w, int(info[i]), f"p{i}")
