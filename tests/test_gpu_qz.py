"""QZ variant on the GPU (hqr_qz_batched) against the oracle's QZ: pairs of
orders 1..64 (held in LDS) and 65..200 (reduced in global memory) in one
batch, some with exact zeros on T's diagonal (infinite eigenvalues), all with
T and Q, Z.  Compared on what a generalized Schur form
fixes: the finite eigenvalues (matched, within 1e-9 of the larger magnitude),
the number of infinite eigenvalues, backward errors of both factors and
orthogonality of Q and Z within 100 n u, exact structure (S quasi
triangular with 2x2 blocks only for complex pairs, T triangular)."""
import sys

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle

pytestmark = pytest.mark.gpu
U = 2.0 ** -52


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def pencil(n, seed, nzero=0):
    g = np.random.default_rng(seed)
    H = np.triu(g.standard_normal((n, n)), -1)
    T = np.triu(g.standard_normal((n, n)))
    if nzero and n > 0:
        for k in g.choice(n, size=min(nzero, n), replace=False):
            T[k, k] = 0.0
    return H, T


def match(a, b):
    if len(a) == 0:
        return 0.0
    C = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(C)
    return C[r, c].max()


def check_pair(H, T, S, Tt, Q, Z, alpha, beta, tag):
    n = H.shape[0]
    assert np.all(np.tril(Tt, -1) == 0.0), tag
    assert np.all(np.tril(S, -2) == 0.0), tag
    bs = np.linalg.norm(Q.T @ H @ Z - S)
    bt = np.linalg.norm(Q.T @ T @ Z - Tt)
    assert bs <= 100 * n * U * max(np.linalg.norm(H), 1e-300), (tag, bs)
    assert bt <= 100 * n * U * max(np.linalg.norm(T), 1e-300), (tag, bt)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 100 * n * U, tag
    assert np.linalg.norm(Z.T @ Z - np.eye(n)) <= 100 * n * U, tag
    k = 0
    while k < n:
        if k + 1 < n and S[k + 1, k] != 0.0:
            assert alpha[k].imag > 0 and alpha[k + 1].imag < 0 and beta[k] > 0, tag
            k += 2
        else:
            assert alpha[k].imag == 0.0 and beta[k] >= 0.0, tag
            k += 1
    _, _, _, _, ao, bo, oi = oracle.qz(H, T, want_qz=False)
    assert oi == 0
    assert int((beta == 0).sum()) == int((bo == 0).sum()), tag
    lam = alpha[beta > 0] / beta[beta > 0]
    lo = ao[bo > 0] / bo[bo > 0]
    assert len(lam) == len(lo), tag
    scale = max(1.0, float(np.abs(lo).max())) if len(lo) else 1.0
    assert match(lam, lo) <= 1e-9 * scale, (tag, match(lam, lo))


def run(pairs):
    import torch
    import paper_2007_03576_amd as hq
    Hs = [torch.from_numpy(np.ascontiguousarray(H)).cuda() for H, _ in pairs]
    Ts = [torch.from_numpy(np.ascontiguousarray(T)).cuda() for _, T in pairs]
    S, Tt, Q, Z, alpha, beta, info = hq.qz_batched(Hs, Ts)
    torch.cuda.synchronize()
    return ([s.cpu().numpy() for s in S], [t.cpu().numpy() for t in Tt], [q.cpu().numpy() for q in Q],
            [z.cpu().numpy() for z in Z], [a.cpu().numpy() for a in alpha], [b.cpu().numpy() for b in beta],
            info.cpu().numpy())


def test_qz_batched_matches_oracle(gpu):
    sizes = [1, 2, 3, 5, 8, 13, 21, 34, 47, 55, 64, 2, 30, 64]
    _say(f"case QZ batched orders {sizes}")
    pairs = [pencil(n, 900 + i) for i, n in enumerate(sizes)]
    S, Tt, Q, Z, alpha, beta, info = run(pairs)
    assert np.all(info == 0), info
    for i, (H, T) in enumerate(pairs):
        check_pair(H, T, S[i], Tt[i], Q[i], Z[i], alpha[i], beta[i], f"pair{i}_n{sizes[i]}")


def test_qz_batched_infinite_eigenvalues(gpu):
    spec = [(6, 1), (10, 2), (17, 3), (32, 1), (40, 4), (64, 2), (3, 3), (1, 1)]
    _say(f"case QZ batched infinite eigenvalues {spec}")
    pairs = [pencil(n, 1700 + i, nz) for i, (n, nz) in enumerate(spec)]
    S, Tt, Q, Z, alpha, beta, info = run(pairs)
    assert np.all(info == 0), info
    for i, (H, T) in enumerate(pairs):
        check_pair(H, T, S[i], Tt[i], Q[i], Z[i], alpha[i], beta[i], f"inf{i}")
        assert int((beta[i] == 0).sum()) >= 1
        assert np.all(np.diag(Tt[i])[beta[i] == 0] == 0.0)


def test_qz_identity_T_and_rejections(gpu):
    import ctypes
    import torch
    from paper_2007_03576_amd._lib import lib
    _say("case QZ with T = I, and a negative order through the C-ABI")
    H, _ = pencil(40, 77)
    S, Tt, Q, Z, alpha, beta, info = run([(H, np.eye(40))])
    assert info[0] == 0
    lam = alpha[0] / beta[0]
    assert match(lam, np.linalg.eigvals(H)) <= 1e-10 * max(1.0, np.abs(lam).max())
    d = torch.zeros(16, dtype=torch.float64, device="cuda")
    offs = torch.zeros(2, dtype=torch.int64, device="cuda")
    nn = torch.tensor([-1, 0], dtype=torch.int32, device="cuda")
    info = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = lib().hqr_qz_batched(P(d), P(d), None, None, P(offs), P(nn), 2, P(d), P(d), P(d), P(offs), P(info), None)
    torch.cuda.synchronize()
    assert rc == 0
    assert info.cpu().tolist() == [-1, 0]


def test_qz_global_memory_orders(gpu):
    sizes = [65, 80, 100, 128, 150, 200, 3, 64]
    nzero = [0, 2, 0, 1, 0, 3, 0, 1]
    _say(f"case QZ orders above the LDS limit {sizes}")
    pairs = [pencil(n, 2600 + i, nz) for i, (n, nz) in enumerate(zip(sizes, nzero))]
    S, Tt, Q, Z, alpha, beta, info = run(pairs)
    assert np.all(info == 0), info
    for i, (H, T) in enumerate(pairs):
        check_pair(H, T, S[i], Tt[i], Q[i], Z[i], alpha[i], beta[i], f"global{i}_n{sizes[i]}")
        if nzero[i]:
            assert int((beta[i] == 0).sum()) >= 1


def test_qz_global_memory_without_factors(gpu):
    import torch
    import paper_2007_03576_amd as hq
    sizes = [90, 33, 140]
    _say(f"case QZ without Q and Z {sizes}")
    pairs = [pencil(n, 3100 + i, 1) for i, n in enumerate(sizes)]
    Hs = [torch.from_numpy(np.ascontiguousarray(H)).cuda() for H, _ in pairs]
    Ts = [torch.from_numpy(np.ascontiguousarray(T)).cuda() for _, T in pairs]
    S, Tt, Q, Z, alpha, beta, info = hq.qz_batched(Hs, Ts, want_qz=False)
    torch.cuda.synchronize()
    assert Q is None and Z is None
    assert np.all(info.cpu().numpy() == 0)
    for i, (H, T) in enumerate(pairs):
        a, b = alpha[i].cpu().numpy(), beta[i].cpu().numpy()
        assert np.all(np.tril(Tt[i].cpu().numpy(), -1) == 0.0)
        assert np.all(np.tril(S[i].cpu().numpy(), -2) == 0.0)
        _, _, _, _, ao, bo, oi = oracle.qz(H, T, want_qz=False)
        assert oi == 0
        assert int((b == 0).sum()) == int((bo == 0).sum())
        lam, lo = a[b > 0] / b[b > 0], ao[bo > 0] / bo[bo > 0]
        assert match(lam, lo) <= 1e-9 * max(1.0, float(np.abs(lo).max()))
