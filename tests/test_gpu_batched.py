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


def _packed_case(lo, hi_, count, seed):
    import torch
    sizes = hi.batched_sizes(count, lo, hi_, seed=seed)
    mats = [hi.gaussian_hessenberg(int(n), seed=seed * 1000 + i) for i, n in enumerate(sizes)]
    return mats, [torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats]


@pytest.mark.skip(reason="per-bucket shift counts (bulge chains in the batched kernels) did not finish on the "
                         "GPU, cause not found; the table was removed and the batched kernels run double shifts")
def test_batched_shift_table_both_tiers(gpu):
    """Per-bucket shift counts (multishift bulge chains in the LDS and the
    global-memory tiers), longest-first queue over mixed orders incl. 0."""
    import torch
    import paper_2007_03576_amd as hq
    _say("case batched shift table 32:2,64:4,96:6,160:8,256:12 sizes 0..200")
    hq.set_batched_shifts([32, 64, 96, 160, 256], [2, 4, 6, 8, 12])  # entry point removed
    try:
        mats, _ = _packed_case(1, 200, 24, 11)
        mats = mats[:12] + [np.zeros((0, 0))] + mats[12:]
        dev = [torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats]
        Ts, Qs, ws, info = hq.schur_batched(dev)
        torch.cuda.synchronize()
        info = info.cpu().numpy()
        for i, H in enumerate(mats):
            if H.shape[0] == 0:
                assert info[i] == 0
                continue
            check_one(H, Ts[i].cpu().numpy(), Qs[i].cpu().numpy(), ws[i].cpu().numpy(), int(info[i]),
                      f"t{i} n={H.shape[0]}")
    finally:
        hq.set_batched_shifts([], [])


@pytest.mark.skip(reason="per-bucket shift counts (bulge chains in the batched kernels) did not finish on the "
                         "GPU, cause not found; the table was removed and the batched kernels run double shifts")
def test_batched_shift_table_lds_tier(gpu):
    """Per-bucket shift counts in the LDS tier (bulge chains of 2..6 bulges),
    double shifts above it, longest-first queue over mixed orders incl. 0."""
    import torch
    import paper_2007_03576_amd as hq
    _say("case batched shift table 24:2,48:4,72:8,96:12 sizes 1..160 plus an empty matrix")
    hq.set_batched_shifts([24, 48, 72, 96], [2, 4, 8, 12])
    try:
        mats, _ = _packed_case(1, 160, 24, 13)
        mats = mats[:12] + [np.zeros((0, 0))] + mats[12:]
        dev = [torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats]
        Ts, Qs, ws, info = hq.schur_batched(dev)
        torch.cuda.synchronize()
        info = info.cpu().numpy()
        for i, H in enumerate(mats):
            if H.shape[0] == 0:
                assert info[i] == 0
                continue
            check_one(H, Ts[i].cpu().numpy(), Qs[i].cpu().numpy(), ws[i].cpu().numpy(), int(info[i]),
                      f"t{i} n={H.shape[0]}")
    finally:
        hq.set_batched_shifts([], [])


def test_batched_graph_replays_match_eager(gpu):
    """The batched solve captured into a HIP graph: three replays on new
    inputs, eager work and synchronizations between them, each bit-identical
    to an eager solve of the same input."""
    import torch
    import paper_2007_03576_amd as hq
    from paper_2007_03576_amd.api import pack
    _say("case batched graph replay sizes 16..140 count 40")
    sizes = hi.batched_sizes(40, 16, 140, seed=21)
    g = hq.BatchedGraph([int(n) for n in sizes])
    for rep in range(3):
        mats = [hi.gaussian_hessenberg(int(n), seed=7000 + 100 * rep + i) for i, n in enumerate(sizes)]
        packed = pack([torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats])
        Ts, Qs, ws, info = g.run(packed)
        torch.cuda.synchronize()
        got_T = g.prob.H.clone()
        got_Q = g.prob.Q.clone()
        got_w = (g.prob.wr.clone(), g.prob.wi.clone())
        assert int(info.abs().max()) == 0
        eager = hq.BatchedProblem([int(n) for n in sizes])
        eager.load(packed)
        eager.solve()
        torch.cuda.synchronize()
        assert torch.equal(eager.H, got_T), f"replay {rep}: T differs from eager"
        assert torch.equal(eager.Q, got_Q), f"replay {rep}: Q differs from eager"
        assert torch.equal(eager.wr, got_w[0]) and torch.equal(eager.wi, got_w[1])
        k = rep * 7 % len(mats)
        check_one(mats[k], Ts[k].cpu().numpy(), Qs[k].cpu().numpy(), ws[k].cpu().numpy(), 0, f"rep{rep} m{k}")



def test_batched_orders_above_320_on_half_grid(gpu):
    """Orders above 320 are taken by the lower half of the global grid first;
    the rest of the global tier and the LDS tier follow (all against the
    oracle)."""
    import torch
    import paper_2007_03576_amd as hq
    sizes = [400, 340, 330, 321, 320, 200, 97, 96, 50, 5]
    _say(f"case batched orders {sizes}")
    mats = [hi.gaussian_hessenberg(n, seed=900 + i) for i, n in enumerate(sizes)]
    Ts, Qs, ws, info = hq.schur_batched([torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats])
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    for i, H in enumerate(mats):
        check_one(H, Ts[i].cpu().numpy(), Qs[i].cpu().numpy(), ws[i].cpu().numpy(), int(info[i]), f"w{i} n={H.shape[0]}")


def test_autotune_launch_shape_installed_and_results_unchanged(gpu):
    """The launch-shape tuner installs one of its candidates; the solve under
    the tuned shape is bit-identical to the default shape (one workgroup per
    matrix either way, only the grid and queue split change)."""
    import torch
    import paper_2007_03576_amd as hq
    from paper_2007_03576_amd import autotune
    _say("case autotune launch shape orders 97..360 count 64")
    prev = hq.batched_launch()
    try:
        tab = autotune.tune(97, 360, count=64, seed=5)
        assert (tab["wg_per_cu"], tab["wide_n"]) in autotune.CANDIDATES
        assert hq.batched_launch() == {"wg_per_cu": tab["wg_per_cu"], "wide_n": tab["wide_n"]}
        sizes, packed = autotune.sample(90, 400, 12, 6, "cuda")
        outs = []
        for wg, wide in [(2, 320), (1, 4095), (3, 200)]:
            hq.set_batched_launch(wg, wide)
            p = hq.BatchedProblem(sizes)
            p.load(packed)
            p.solve()
            torch.cuda.synchronize()
            assert int(p.info.abs().max()) == 0
            outs.append((p.H.clone(), p.Q.clone()))
        for H, Q in outs[1:]:
            assert torch.equal(H, outs[0][0]) and torch.equal(Q, outs[0][1])
    finally:
        hq.set_batched_launch(prev["wg_per_cu"], prev["wide_n"])


@pytest.mark.parametrize("table", [
    {"upper": [4095], "nw": [32], "ns": [16]},
    {"upper": [128, 192, 4095], "nw": [24, 48, 64], "ns": [12, 24, 48]},
    {"upper": [150, 4095], "nw": [0, 40], "ns": [0, 40]},
])
def test_batched_aed_table(gpu, table):
    """Per-bucket AED windows and shift counts for orders above 96 (H and Q
    in global memory, the AED window in LDS), mixed with double shifts below
    and in buckets without AED; every matrix against the oracle."""
    import torch
    import paper_2007_03576_amd as hq
    _say(f"case batched AED table {table}")
    hq.set_batched_table(table["upper"], table["nw"], table["ns"])
    try:
        mats, _ = _packed_case(1, 260, 30, 17)
        mats = mats[:10] + [np.zeros((0, 0))] + mats[10:]
        dev = [torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats]
        Ts, Qs, ws, info = hq.schur_batched(dev)
        torch.cuda.synchronize()
        info = info.cpu().numpy()
        for i, H in enumerate(mats):
            if H.shape[0] == 0:
                assert info[i] == 0
                continue
            check_one(H, Ts[i].cpu().numpy(), Qs[i].cpu().numpy(), ws[i].cpu().numpy(), int(info[i]),
                      f"t{i} n={H.shape[0]}")
        # prescribed spectra through the AED path
        for i, n in enumerate([120, 200, 256]):
            H, ev = hi.prescribed_hessenberg(n, seed=900 + i)
            Tl, Ql, wl, inf = hq.schur_batched([torch.from_numpy(np.ascontiguousarray(H)).cuda()])
            w = wl[0].cpu().numpy()
            _, _, d = checks.match(w, ev)
            assert d.max() <= 1e-10 * np.linalg.norm(H)
            check_one(H, Tl[0].cpu().numpy(), Ql[0].cpu().numpy(), w, int(inf[0]), f"p{n}")
    finally:
        hq.set_batched_table([], [], [])
