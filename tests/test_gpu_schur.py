"""GPU parity tests of hqr_schur (C-ABI through the thin torch binding) against the oracle.

A real Schur form is unique only up to the order of the eigenvalues along the
diagonal, the signs of Q's columns and a rotation inside each 2x2 block, so the
GPU result and the oracle's are compared on what is unique:
  * eigenvalue multisets (optimal matching), within 1e-10 * kappa_i * ||H||_F
    (kappa_i from LAPACK left/right eigenvectors), or against the prescribed
    spectrum for the normal test matrices (kappa = 1);
  * backward error ||Q^T H Q - T||_F / ||H||_F <= 100 n u and orthogonality
    ||Q^T Q - I||_F <= 100 n u;
  * exact quasi-triangular structure with standardized 2x2 blocks.
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
    return (T.cpu().numpy(), None if Q is None else Q.cpu().numpy(), w.cpu().numpy(), info,
            hq.last_stats())


def assert_schur(H, T, Q, w, ref_eigs=None, kappa_tol=True, tag=""):
    n = H.shape[0]
    ok, msg = checks.structure_ok(T, w)
    assert ok, f"{tag}: {msg}"
    be = checks.rel_backward(H, T, Q)
    ob = checks.orth(Q)
    _say(f"{tag}: n={n} backward={be:.3e} ({be / U:.1f} u) orth={ob:.3e}")
    assert be <= 100 * n * U, f"{tag}: backward error {be}"
    assert ob <= 100 * n * U, f"{tag}: orthogonality {ob}"
    # oracle eigenvalues for the same input
    To, Qo, wo, info, _ = oracle.schur(H)
    assert info == 0
    hn = np.linalg.norm(H)
    if ref_eigs is not None:
        r, c, d = checks.match(w, ref_eigs)
        assert d.max() <= 1e-10 * max(hn, 1.0), f"{tag}: max |dl| vs prescribed {d.max()}"
    lam, kap = checks.eig_condition(H)
    r, c, d = checks.match(w, wo)
    r2, c2, _ = checks.match(wo, lam)
    kap_o = np.empty(n)
    kap_o[r2] = kap[c2]
    tol = 1e-10 * np.maximum(kap_o[c], 1.0) * max(hn, 1.0)
    assert np.all(d <= tol), f"{tag}: eigenvalue mismatch vs oracle, worst {np.max(d / tol)} x tol"


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 50, 75, 96])
def test_small_block_solver(gpu, n):
    _say(f"case small n={n}")
    H = hi.gaussian_hessenberg(n, seed=100 + n)
    T, Q, w, info, st = run_gpu(H)
    assert info == 0
    assert_schur(H, T, Q, w, tag=f"small{n}")


@pytest.mark.parametrize("n,params", [(150, None), (256, None), (300, {"ns": 16, "nw": 48}),
                                      (400, {"ns": 32, "nw": 96, "nmin": 40})])
def test_aed_and_sweeps(gpu, n, params):
    _say(f"case aed n={n} params={params}")
    H = hi.hessrand(n, seed=7 + n)
    T, Q, w, info, st = run_gpu(H, params)
    _say(f"stats {st}")
    assert info == 0
    assert_schur(H, T, Q, w, tag=f"hessrand{n}")


def test_prescribed_config0(gpu):
    _say("case prescribed n=256 (config 0 recipe)")
    H, ev = hi.prescribed_hessenberg(256, seed=2020)
    T, Q, w, info, st = run_gpu(H)
    _say(f"stats {st}")
    assert info == 0
    assert_schur(H, T, Q, w, ref_eigs=ev, tag="cfg0")


def test_big_aed_window(gpu):
    _say("case big AED window n=600 nw=160 ns=32")
    H = hi.gaussian_hessenberg(600, seed=11)
    T, Q, w, info, st = run_gpu(H, {"ns": 32, "nw": 160})
    _say(f"stats {st}")
    assert info == 0
    assert st["deflation_windows"] > 0
    assert_schur(H, T, Q, w, tag="bigaed600")


def test_big_aed_reordering_chains(gpu):
    # large windows on matrices where an early deflation window fails for
    # more than half (and at most two thirds) of its candidates: a chain of
    # reordering windows carries the failures to the top of the AED window;
    # every run must be a correct Schur form, and the chains must have run
    total = 0
    for n, seed, nw in [(700, 12, 320), (700, 13, 320), (640, 14, 256), (800, 15, 400)]:
        _say(f"case big AED window reordering chains n={n} nw={nw} seed={seed}")
        H = hi.hessrand(n, seed=seed)
        T, Q, w, info, st = run_gpu(H, {"ns": 48, "nw": nw})
        _say(f"stats {st}")
        assert info == 0
        assert_schur(H, T, Q, w, tag=f"reorder{n}_{seed}")
        total += st["reordering_windows"]
    assert total > 0


def test_large_window_factor(gpu):
    # an AED window of 1024: its factor (order 1024) is applied out of place
    # by the tiled MFMA product and copied back
    _say("case AED window 1024 n=1300 ns=64")
    H = hi.gaussian_hessenberg(1300, seed=31)
    T, Q, w, info, st = run_gpu(H, {"ns": 64, "nw": 1024})
    _say(f"stats {st}")
    assert info == 0
    assert_schur(H, T, Q, w, tag="win1024")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_aed_modes(gpu, mode):
    # Sec. 3.5, adaptive approach: AED windows above 96 run sequentially (one
    # workgroup reduces the window, tests every candidate and reorders the
    # failures) or in parallel (recursive solve, chains of deflation and
    # reordering windows); 0 decides per window from the queued update work
    total = {"sequential_aeds": 0, "parallel_aeds": 0}
    for n, seed, nw in [(600, 21, 192), (500, 22, 128), (700, 23, 320)]:
        _say(f"case AED mode {mode} n={n} nw={nw} seed={seed}")
        H = hi.hessrand(n, seed=seed)
        T, Q, w, info, st = run_gpu(H, {"ns": 32, "nw": nw, "aed_mode": mode})
        _say(f"stats {st}")
        assert info == 0
        assert_schur(H, T, Q, w, tag=f"aedmode{mode}_{n}")
        for k in total:
            total[k] += st[k]
    assert total["sequential_aeds"] + total["parallel_aeds"] > 0
    if mode == 1:
        assert total["parallel_aeds"] == 0
    if mode == 2:
        assert total["sequential_aeds"] == 0


def test_sequential_aed_size_limit(gpu):
    # windows above aed_seq_max go to the parallel AED even when the
    # sequential one is requested (the smaller windows of a nearly deflated
    # active block may still run sequentially)
    _say("case sequential AED limit n=600 nw=192 aed_seq_max=160")
    H = hi.hessrand(600, seed=24)
    T, Q, w, info, st = run_gpu(H, {"ns": 32, "nw": 192, "aed_mode": 1, "aed_seq_max": 160})
    _say(f"stats {st}")
    assert info == 0
    assert_schur(H, T, Q, w, tag="seqlimit")
    assert st["parallel_aeds"] > 0


@pytest.mark.parametrize("nsmall", [8, 16])
@pytest.mark.parametrize("n,params", [(90, {}), (300, {"ns": 16, "nw": 80})])
def test_multishift_small_solver(gpu, n, params, nsmall):
    _say(f"case multishift small solver n={n} small_shifts={nsmall} params={params}")
    H = hi.hessrand(n, seed=70 + n)
    p = dict(params)
    p["small_shifts"] = nsmall
    T, Q, w, info, st = run_gpu(H, p)
    _say(f"stats {st}")
    assert info == 0
    assert_schur(H, T, Q, w, tag=f"ms{nsmall}_{n}")


def test_single_stream_matches_two_streams(gpu):
    _say("case streams=1 vs streams=2 (bitwise identical: same kernels, same order per element)")
    H = hi.hessrand(350, seed=3)
    T1, Q1, w1, i1, _ = run_gpu(H, {"ns": 16, "nw": 64, "streams": 1})
    T2, Q2, w2, i2, _ = run_gpu(H, {"ns": 16, "nw": 64, "streams": 2})
    assert i1 == 0 and i2 == 0
    assert np.array_equal(T1, T2) and np.array_equal(Q1, Q2)


def test_syn_matrix(gpu):
    _say("case syn_n n=320")
    H, ev = hi.syn_matrix(320, seed=5)
    T, Q, w, info, st = run_gpu(H, {"ns": 24, "nw": 64})
    assert info == 0
    assert_schur(H, T, Q, w, tag="syn320")
