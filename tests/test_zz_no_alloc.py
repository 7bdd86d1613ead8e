"""hqr_schur_batched_noalloc (the entry point for callers that cannot
allocate) against hqr_schur_batched on the same inputs: two calls in a row,
the second with a smaller batch, both bit-identical to the allocating entry
point (the same kernels solve each matrix in one workgroup, so the result
does not depend on which workgroup took it)."""
import ctypes
import sys

import numpy as np
import pytest

import hqr_inputs as hi

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _solve(entry, sizes, packed, dev):
    import torch
    from paper_2007_03576_amd._lib import lib
    count = len(sizes)
    offs = np.zeros(count, dtype=np.int64)
    offs[1:] = np.cumsum(np.asarray(sizes, dtype=np.int64)[:-1] ** 2)
    eo = hi.eig_offsets(np.asarray(sizes))
    H = torch.from_numpy(packed).to(dev)
    Q = torch.cat([torch.eye(int(s), dtype=torch.float64, device=dev).reshape(-1) for s in sizes])
    tot = int(np.sum(sizes))
    wr = torch.full((max(tot, 1),), np.nan, dtype=torch.float64, device=dev)
    wi = torch.full_like(wr, np.nan)
    info = torch.full((count,), -7, dtype=torch.int32, device=dev)
    d_off = torch.from_numpy(offs).to(dev)
    d_n = torch.from_numpy(np.asarray(sizes, dtype=np.int32)).to(dev)
    d_eo = torch.from_numpy(np.asarray(eo, dtype=np.int64)).to(dev)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    fn = getattr(lib(), entry)
    rc = fn(P(H), P(Q), P(d_off), P(d_n), count, P(wr), P(wi), P(d_eo), P(info),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == 0, (entry, rc)
    return H.cpu().numpy(), Q.cpu().numpy(), wr.cpu().numpy(), wi.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("count", [3000, 700])
def test_noalloc_matches_allocating_entry(gpu, count):
    # orders across both tiers (LDS <= 96 < global), with empty matrices
    sizes = hi.batched_sizes(count, 0, 180, seed=91 + count)
    packed, _ = hi.batched_gaussian(sizes, seed=91 + count)
    _say(f"case noalloc count={count} max order {int(np.max(sizes))}")
    a = _solve("hqr_schur_batched", sizes, packed, gpu)
    b = _solve("hqr_schur_batched_noalloc", sizes, packed, gpu)
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True)
    assert np.all(b[4] == 0)


def test_noalloc_twice_second_smaller(gpu):
    big = hi.batched_sizes(2500, 1, 200, seed=5)
    small = hi.batched_sizes(400, 1, 120, seed=6)
    pb, _ = hi.batched_gaussian(big, seed=5)
    ps, _ = hi.batched_gaussian(small, seed=6)
    _say("case noalloc two calls in a row, the second smaller")
    r1 = _solve("hqr_schur_batched_noalloc", big, pb, gpu)
    r2 = _solve("hqr_schur_batched_noalloc", small, ps, gpu)
    e1 = _solve("hqr_schur_batched", big, pb, gpu)
    e2 = _solve("hqr_schur_batched", small, ps, gpu)
    for x, y in zip(r1, e1):
        assert np.array_equal(x, y, equal_nan=True)
    for x, y in zip(r2, e2):
        assert np.array_equal(x, y, equal_nan=True)


def test_noalloc_rejects_oversized_batch(gpu):
    from paper_2007_03576_amd._lib import lib
    buf = ctypes.c_void_p(1)
    assert lib().hqr_schur_batched_noalloc(buf, None, buf, buf, (1 << 20) + 1, buf, buf, buf, buf, None) == -5
