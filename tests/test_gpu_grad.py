"""GPU tests of the differentiable eigenvalues (SchurEig autograd.Function):
gradient against the oracle's gradient, against closed forms and against
central finite differences (h = 1e-6) along directions on the Hessenberg pattern."""
import sys

import numpy as np
import pytest

import hqr_inputs as hi
import oracle

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def loss_t(w):
    import torch
    return (torch.nn.functional.softplus(w.real) + 0.1 * w.abs() ** 2).sum()


def loss_np(w):
    return float(np.sum(np.logaddexp(0.0, w.real)) + 0.1 * np.sum(np.abs(w) ** 2))


def grad_gpu(H):
    import torch
    import paper_2007_03576_amd as hq
    Ht = torch.from_numpy(np.ascontiguousarray(H)).cuda().requires_grad_(True)
    w = hq.eigvals(Ht)
    L = loss_t(w)
    L.backward()
    return Ht.grad.cpu().numpy(), w.detach().cpu().numpy()


def grad_oracle(H):
    T, Q, w, info, _ = oracle.schur(H)
    g = 1.0 / (1.0 + np.exp(-w.real)) + 0.2 * w
    return oracle.eig_backward(T, Q, w, g)


@pytest.mark.parametrize("kind,n", [("normal", 32), ("nonnormal", 24), ("normal", 150)])
def test_gradient_matches_oracle(gpu, kind, n):
    _say(f"case grad {kind} n={n}")
    if kind == "normal":
        H, _ = hi.prescribed_hessenberg(n, seed=500 + n, separated=True)
    else:
        H, _ = hi.syn_matrix(n, seed=501)
    dg, w = grad_gpu(H)
    do = grad_oracle(H)
    err = np.abs(dg - do).max() / max(np.abs(do).max(), 1e-300)
    _say(f"  rel err vs oracle {err:.2e}")
    assert err <= 1e-8
    assert np.all(np.tril(dg, -2) == 0.0)


def test_gradient_trace_closed_form(gpu):
    import torch
    import paper_2007_03576_amd as hq
    H = hi.hessrand(40, seed=9)
    Ht = torch.from_numpy(np.ascontiguousarray(H)).cuda().requires_grad_(True)
    w = hq.eigvals(Ht)
    w.real.sum().backward()
    assert np.abs(Ht.grad.cpu().numpy() - np.eye(40)).max() <= 1e-9


def test_gradient_central_differences(gpu):
    _say("case grad FD n=40 nonnormal")
    H, _ = hi.syn_matrix(40, seed=777)
    dg, _ = grad_gpu(H)
    g = np.random.default_rng(3)
    h = 1e-6
    for _ in range(5):
        D = np.triu(g.standard_normal(H.shape), -1)
        D /= np.linalg.norm(D)
        lp = loss_np(oracle.schur(H + h * D, want_q=False)[2])
        lm = loss_np(oracle.schur(H - h * D, want_q=False)[2])
        fd = (lp - lm) / (2 * h)
        an = float(np.sum(dg * D))
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (fd, an)


def test_batched_gradient(gpu):
    import torch
    import paper_2007_03576_amd as hq
    _say("case batched grad B=5 n=48")
    mats = [hi.prescribed_hessenberg(48, seed=600 + i, separated=True)[0] for i in range(5)]
    Hb = torch.from_numpy(np.stack(mats)).cuda().requires_grad_(True)
    w = hq.eigvals(Hb)
    loss_t(w).backward()
    G = Hb.grad.cpu().numpy()
    for i, H in enumerate(mats):
        do = grad_oracle(H)
        assert np.abs(G[i] - do).max() <= 1e-8 * np.abs(do).max()


def test_uneven_batch_gradient(gpu):
    """Orders differ across the batch (packed layout with offsets): the
    backward through hqr_eig_backward_batched with per-matrix orders against
    the oracle gradient of each matrix, including empty and 1x1 matrices."""
    import torch
    from paper_2007_03576_amd.autograd import eigvals_uneven
    sizes = [48, 0, 17, 1, 130, 64, 2, 97]
    _say(f"case uneven batched grad sizes={sizes}")
    mats = []
    for i, s in enumerate(sizes):
        if s >= 8:
            mats.append(hi.prescribed_hessenberg(s, seed=700 + i, separated=True)[0])
        else:
            mats.append(hi.gaussian_hessenberg(s, seed=700 + i))
    Ts = [torch.from_numpy(np.ascontiguousarray(m)).cuda().requires_grad_(True) for m in mats]
    ws = eigvals_uneven(Ts)
    loss = sum(loss_t(w) for w in ws)
    loss.backward()
    for i, (H, X) in enumerate(zip(mats, Ts)):
        if sizes[i] == 0:
            continue
        G = X.grad.cpu().numpy()
        do = grad_oracle(H)
        scale = max(np.abs(do).max(), 1e-300)
        assert np.abs(G - do).max() <= 1e-8 * scale, (i, sizes[i], np.abs(G - do).max() / scale)
        assert np.all(np.tril(G, -2) == 0.0)
