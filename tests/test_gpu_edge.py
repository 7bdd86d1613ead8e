"""Edge cases of the HIP path through the C-ABI, against the oracle or against
what the mathematics fixes for them:

* an exact zero subdiagonal mid-matrix: the spectrum is the union of the two
  diagonal blocks' spectra (Sec. 2.1: the problem decouples);
* upper triangular input and H = 0: already in Schur form, so T = H and
  Q = I exactly;
* a non-finite entry in the Hessenberg part: argument error -1 (raised);
* an iteration limit too small to converge: info > 0, and the returned (T, Q)
  is still an orthogonal similarity of H (backward error and orthogonality
  within 100 n u), with the rows below info converged;
* exceptional shifts forced every step or every other step (kexsh 1, 2):
  still a valid Schur form with the oracle's eigenvalues;
* the norm-stable and fixed deflation conditions (Sec. 5.6, items 2 and 3)
  against the oracle run under the same conditions;
* the batched form with empty, 1x1 and 2x2 matrices among larger ones.
"""
import sys

import numpy as np
import pytest

import hqr_inputs as hi
import oracle
from tests import checks

pytestmark = pytest.mark.gpu
U = 2.0 ** -52


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(H, params=None, want_q=True):
    import torch
    import paper_2007_03576_amd as hq
    Ht = torch.from_numpy(np.ascontiguousarray(H)).cuda()
    T, Q, w, info = hq.schur(Ht, want_q=want_q, params=params)
    torch.cuda.synchronize()
    return T.cpu().numpy(), None if Q is None else Q.cpu().numpy(), w.cpu().numpy(), info


def eig_match_oracle(H, w, wo, tag):
    n = H.shape[0]
    lam, kap = checks.eig_condition(H)
    r, c, d = checks.match(w, wo)
    r2, c2, _ = checks.match(wo, lam)
    kap_o = np.empty(n)
    kap_o[r2] = kap[c2]
    tol = 1e-10 * np.maximum(kap_o[c], 1.0) * max(np.linalg.norm(H), 1.0)
    assert np.all(d <= tol), f"{tag}: eigenvalue mismatch vs oracle, worst {np.max(d / tol)} x tol"


def test_zero_subdiagonal_mid_matrix(gpu):
    n, k = 240, 131
    _say(f"case exact zero subdiagonal n={n} at row {k}")
    H = hi.gaussian_hessenberg(n, seed=41)
    H[k, k - 1] = 0.0
    T, Q, w, info = run_gpu(H, {"ns": 16, "nw": 48})
    assert info == 0
    ok, msg = checks.structure_ok(T, w)
    assert ok, msg
    assert checks.rel_backward(H, T, Q) <= 100 * n * U
    assert checks.orth(Q) <= 100 * n * U
    # the spectrum is the union of the spectra of the two diagonal blocks
    _, _, w1, i1, _ = oracle.schur(H[:k, :k].copy(), want_q=False)
    _, _, w2, i2, _ = oracle.schur(H[k:, k:].copy(), want_q=False)
    assert i1 == 0 and i2 == 0
    eig_match_oracle(H, w, np.concatenate([w1, w2]), "zero-sub")


@pytest.mark.parametrize("kind", ["triangular", "zero"])
def test_already_schur(gpu, kind):
    n = 130
    _say(f"case {kind} input n={n}")
    if kind == "zero":
        H = np.zeros((n, n))
    else:
        H = np.triu(np.random.default_rng(3).standard_normal((n, n)))
    T, Q, w, info = run_gpu(H)
    assert info == 0
    assert np.array_equal(T, H)
    assert np.array_equal(Q, np.eye(n))
    assert np.array_equal(w.real, np.diag(H)) and np.all(w.imag == 0.0)


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_non_finite_input_rejected(gpu, bad):
    from paper_2007_03576_amd import HqrError
    n = 90
    _say(f"case non-finite input {bad}")
    H = hi.gaussian_hessenberg(n, seed=5)
    H[40, 60] = bad
    with pytest.raises(HqrError, match="code -1"):
        run_gpu(H)
    # entries below the subdiagonal are not read
    H = hi.gaussian_hessenberg(n, seed=5)
    H[70, 3] = bad
    T, Q, w, info = run_gpu(H)
    assert info == 0
    Hh = np.triu(H, -1)
    assert checks.rel_backward(Hh, T, Q) <= 100 * n * U


@pytest.mark.parametrize("n,params", [(60, {"itmax": 3}), (300, {"ns": 16, "nw": 48, "itmax": 2})])
def test_iteration_limit(gpu, n, params):
    _say(f"case iteration limit n={n} params={params}")
    H = hi.hessrand(n, seed=9)
    T, Q, w, info = run_gpu(H, params)
    _say(f"info {info}")
    assert 0 < info <= n
    # an orthogonal similarity of H even though it did not converge
    assert checks.rel_backward(H, T, Q) <= 100 * n * U
    assert checks.orth(Q) <= 100 * n * U
    assert np.all(np.tril(T, -2) == 0.0)
    if info < n:
        # rows info..n-1 (0-based) converged: decoupled and quasi-triangular
        assert T[info, info - 1] == 0.0
        Tb = T[info:, info:]
        ok, msg = checks.structure_ok(Tb, w[info:])
        assert ok, msg
        # and their eigenvalues are eigenvalues of H
        _, _, wo, oi, _ = oracle.schur(H, want_q=False)
        assert oi == 0
        d = np.abs(w[info:, None] - wo[None, :]).min(axis=1)
        lam, kap = checks.eig_condition(H)
        assert d.max() <= 1e-10 * max(kap.max(), 1.0) * np.linalg.norm(H)


@pytest.mark.parametrize("kexsh", [1, 2])
@pytest.mark.parametrize("n,params", [(200, {"ns": 16, "nw": 48, "nmin": 12}), (500, {"ns": 32, "nw": 96})])
def test_exceptional_shifts(gpu, kexsh, n, params):
    p = dict(params)
    p["kexsh"] = kexsh
    _say(f"case exceptional shifts n={n} params={p}")
    H = hi.hessrand(n, seed=31 + n)
    T, Q, w, info = run_gpu(H, p)
    assert info == 0
    ok, msg = checks.structure_ok(T, w)
    assert ok, msg
    be, ob = checks.rel_backward(H, T, Q), checks.orth(Q)
    _say(f"backward {be / U:.1f} u orth {ob / U:.1f} u")
    assert be <= 100 * n * U and ob <= 100 * n * U
    _, _, wo, oi, _ = oracle.schur(H, want_q=False)
    assert oi == 0
    eig_match_oracle(H, w, wo, f"kexsh{kexsh}")


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("n,params", [(96, {}), (400, {"ns": 32, "nw": 96}), (600, {"ns": 32, "nw": 160})])
def test_deflation_conditions(gpu, mode, n, params):
    _say(f"case deflation mode {mode} n={n} params={params}")
    H = hi.hessrand(n, seed=17 + n)
    p = dict(params)
    p["defl_mode"] = mode
    thold = 0.0
    if mode == 2:
        thold = 1e-13 * np.linalg.norm(np.triu(H, -1))
        p["defl_thold"] = thold
    T, Q, w, info = run_gpu(H, p)
    assert info == 0
    ok, msg = checks.structure_ok(T, w)
    assert ok, msg
    be, ob = checks.rel_backward(H, T, Q), checks.orth(Q)
    _say(f"backward {be / U:.1f} u orth {ob / U:.1f} u")
    assert be <= 100 * n * U and ob <= 100 * n * U
    _, _, wo, oi, _ = oracle.schur(H, want_q=False, defl_mode=mode, defl_thold=thold)
    assert oi == 0
    eig_match_oracle(H, w, wo, f"defl{mode}")


def test_batched_degenerate_orders(gpu):
    import torch
    import paper_2007_03576_amd as hq
    sizes = [0, 1, 2, 0, 3, 150, 1, 97, 0, 2, 40, 96, 0]
    _say(f"case batched degenerate orders {sizes}")
    mats = [hi.gaussian_hessenberg(s, seed=200 + i) if s > 0 else np.zeros((0, 0)) for i, s in enumerate(sizes)]
    prob = hq.BatchedProblem(sizes)
    packed = np.concatenate([m.T.reshape(-1) for m in mats]) if sum(s * s for s in sizes) else np.zeros(0)
    prob.load(torch.from_numpy(packed).cuda())
    prob.solve()
    torch.cuda.synchronize()
    Ts, Qs, ws, info = prob.results()
    assert int(info.abs().max()) == 0
    for i, (s, H) in enumerate(zip(sizes, mats)):
        if s == 0:
            continue
        T, Q, w = Ts[i].cpu().numpy(), Qs[i].cpu().numpy(), ws[i].cpu().numpy()
        ok, msg = checks.structure_ok(T, w)
        assert ok, (i, msg)
        assert checks.rel_backward(H, T, Q) <= 100 * s * U
        assert checks.orth(Q) <= 100 * s * U
        _, _, wo, oi, _ = oracle.schur(H, want_q=False)
        assert oi == 0
        eig_match_oracle(H, w, wo, f"batched{i}")
