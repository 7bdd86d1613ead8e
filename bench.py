"""Benchmark: Hessenberg -> real Schur form (multishift QR + AED) on one MI355X.

One step = one full hqr_schur call (T and Q) on the benchmark matrix, with the
input already resident in HBM.  The default workload is the paper-scale
configuration: n = 16384 with a prescribed spectrum (8192 real eigenvalues
and 4096 conjugate pairs, Haar orthogonal similarity reduced to Hessenberg
form on the GPU, seed 2020), 256 shifts per sweep and an AED window of 1024,
Q accumulated from I.  The n = 4096 Gaussian Hessenberg configuration (64
shifts, window 256), the batched and the differentiated forms are reported
beside it.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    "gaussian_hessenberg_n4096": dict(n=4096, gen="gaussian", ns=64, nw=256),
    "prescribed_hessenberg_n256": dict(n=256, gen="prescribed", ns=0, nw=0),
    "prescribed_hessenberg_n16384": dict(n=16384, gen="prescribed", ns=256, nw=1024),
    "hessrand_n4096": dict(n=4096, gen="hessrand", ns=64, nw=256),
}


def make_input(spec, seed, dev, cache=None, name=""):
    """(device tensor holding H column-major (row-major storage of H^T), the
    prescribed eigenvalues or None).  With a cache directory the input is
    read from there when present, else generated and written there (so that
    a profiled run need not execute the generator's library kernels)."""
    import numpy as np
    import torch
    import hqr_inputs as hi
    n = spec["n"]
    if cache:
        path = os.path.join(cache, f"{name}_{seed}.npz")
        if os.path.exists(path):
            z = np.load(path)
            ev = z["ev"] if z["ev"].size else None
            return torch.from_numpy(z["Ht"]).to(dev), ev
        Ht, ev = make_input(spec, seed, dev)
        os.makedirs(cache, exist_ok=True)
        np.savez(path, Ht=Ht.cpu().numpy(), ev=np.zeros(0) if ev is None else np.asarray(ev))
        return Ht, ev
    if spec["gen"] == "prescribed" and n > 4096:
        H, ev = hi.prescribed_hessenberg_device(n, seed=seed, device=dev)  # host reduction would take minutes
        return H.t().contiguous(), ev
    ev = None
    if spec["gen"] == "gaussian":
        H = hi.gaussian_hessenberg(n, seed=seed)
    elif spec["gen"] == "hessrand":
        H = hi.hessrand(n, seed=seed)
    else:
        H, ev = hi.prescribed_hessenberg(n, seed=seed)
    return torch.from_numpy(np.ascontiguousarray(H.T)).to(dev), ev


def measured_traffic(kernel, workload="gaussian_hessenberg_n4096"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary
    of the workload (FETCH_SIZE and WRITE_SIZE, calibrated with a plain copy),
    or None when there is none or the HIP sources changed since the counters
    were taken."""
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_iter_{workload}.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("pmc-json:"):
            rec = json.loads(line.split(":", 1)[1])
    if rec is None or rec.get("kernel") != kernel:
        return None
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2007_03576_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h")):
            h.update(open(f, "rb").read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def batched_run(seed):
    """Batched form: 20000 Gaussian Hessenberg matrices with orders drawn from
    16..256, packed, T and Q for each.  The per-bucket AED window and shift
    count (orders 97..128, 129..192, 193..256) and the launch shape of the
    global grid come from the autotuners (their own seeded samples); the
    solve (order sort, two persistent grids draining a longest-first queue)
    is captured once into a HIP graph and the second of two replays is timed.
    The plain solver (one hqr_schur call per matrix) is timed on a seeded
    sample of 64 matrices of the same batch for comparison."""
    import numpy as np
    import torch
    import hqr_inputs as hi
    import paper_2007_03576_amd as hq
    dev = torch.device("cuda:0")
    count = 20000
    sizes = hi.batched_sizes(count, 16, 256, seed=seed)
    packed, _ = hi.batched_gaussian(sizes, seed=seed)
    H0 = torch.from_numpy(packed).to(dev)
    from paper_2007_03576_amd import autotune
    t0 = time.perf_counter()
    table = autotune.tune_table(seed=seed + 7)  # per-bucket (nw, ns), own seeded samples
    shape = autotune.tune(97, 256, seed=seed + 1)  # the global grid's orders, own seeded sample
    tune_s = time.perf_counter() - t0
    g = hq.BatchedGraph([int(n) for n in sizes])
    dt = None
    for _ in range(2):
        g.prob.load(H0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.graph.replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    info_max = int(g.prob.info.abs().max())
    # accuracy of a seeded sample (outside the timed region)
    pick = np.random.default_rng(seed).choice(count, size=32, replace=False)
    worst_be = worst_orth = 0.0
    for i in pick:
        n, o = int(sizes[i]), g.prob.offs[i]
        A = H0[o:o + n * n].reshape(n, n).t()
        T = g.prob.H[o:o + n * n].reshape(n, n).t()
        Q = g.prob.Q[o:o + n * n].reshape(n, n).t()
        worst_be = max(worst_be, float(torch.linalg.norm(Q.t() @ A @ Q - T) / torch.linalg.norm(A)))
        worst_orth = max(worst_orth, float(torch.linalg.norm(Q.t() @ Q - torch.eye(n, dtype=Q.dtype, device=dev))))
    # the plain solver, one call per matrix, on the same sample's first 64 matrices
    pick = np.random.default_rng(seed + 2).choice(count, size=64, replace=False)
    mats = [H0[g.prob.offs[i]:g.prob.offs[i] + int(sizes[i]) ** 2].reshape(int(sizes[i]), int(sizes[i])).t()
            for i in pick]
    hq.schur(mats[0].t().contiguous().t())  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for A in mats:
        hq.schur(A)
    torch.cuda.synchronize()
    plain_dt = time.perf_counter() - t0
    plain_rate = len(mats) / plain_dt
    return {"workload": "20000 Gaussian Hessenberg matrices, orders U{16..256} (seeded), T and Q, one graph replay",
            "s": dt, "solves_per_s": count / dt, "info_max": info_max,
            "accuracy_sample32": {"backward_rel_max": worst_be, "orth_max": worst_orth},
            "launch_shape": {"wg_per_cu": shape["wg_per_cu"], "wide_n": shape["wide_n"], "tune_s": tune_s},
            "bucket_table": {"upper": table["upper"], "nw": table["nw"], "ns": table["ns"],
                             "seconds": table["seconds"]},
            "plain_per_matrix": {"sample": "64 matrices of the batch, one hqr_schur call each",
                                 "solves_per_s": plain_rate},
            "speedup_vs_plain": (count / dt) / plain_rate}


def grad_run(seed):
    """Differentiation form: 512 matrices of order 512 with well-separated
    prescribed spectra, L = sum softplus(Re l) + 0.1 sum |l|^2, forward Schur
    solve and backward dL/dH (the second of two timed)."""
    import torch
    import hqr_inputs as hi
    import paper_2007_03576_amd as hq
    from paper_2007_03576_amd import autotune
    H, _ = hi.prescribed_batch_device(512, 512, seed=seed, device="cuda")
    # AED window / shifts and launch shape for 512 matrices of order 512, tuned
    # on 512 other matrices of the same kind: prescribed spectra converge far
    # more slowly than Gaussian Hessenberg matrices, so a Gaussian sample would
    # pick other settings, and a sample smaller than the batch cannot tell one
    # workgroup per CU from two (measured on the batch: 1.02 s against 1.29 s)
    Ht, _ = hi.prescribed_batch_device(512, 512, seed=seed + 9, device="cuda")
    packed_t = Ht.transpose(1, 2).contiguous().reshape(-1)

    def same_kind(lo, hi_, count, sd, dev):
        return [512] * Ht.shape[0], packed_t

    table = autotune.tune_table(buckets=((512, 512),), seed=seed + 9, sampler=same_kind)
    shape = autotune.tune(512, 512, seed=seed + 3, sampler=same_kind,
                          candidates=((1, 4095), (2, 4095), (2, 320), (3, 320), (4, 320)))
    del Ht, packed_t
    fw = bw = None
    X = None
    for _ in range(2):
        X = H.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam = hq.eigvals(X)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = torch.nn.functional.softplus(lam.real).sum() + 0.1 * (lam.abs() ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fw, bw = t1 - t0, t2 - t1
    # accuracy (outside the timed region): central differences of the same
    # batched forward along two seeded unit directions on the Hessenberg
    # pattern of all 512 matrices, against <dL/dH, D>
    def loss_of(M):
        with torch.no_grad():
            lm = hq.eigvals(M)
            return float(torch.nn.functional.softplus(lm.real).sum() + 0.1 * (lm.abs() ** 2).sum())

    gen = torch.Generator(device=H.device)
    gen.manual_seed(seed + 5)
    fd_checks = []
    h = 1e-5
    for _ in range(2):
        D = torch.randn(H.shape, generator=gen, dtype=H.dtype, device=H.device).triu(-1)
        D /= torch.linalg.norm(D)
        fd = (loss_of(H + h * D) - loss_of(H - h * D)) / (2 * h)
        an = float((X.grad * D).sum())
        fd_checks.append({"fd": fd, "analytic": an, "rel_diff": abs(fd - an) / max(abs(an), 1e-300)})
    # the plain solver, one hqr_schur call per matrix (forward only), on 8 of the matrices
    hq.schur(H[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(8):
        hq.schur(H[b])
    torch.cuda.synchronize()
    plain_rate = 8 / (time.perf_counter() - t0)
    return {"workload": "512 matrices n=512, separated prescribed spectra, L = sum softplus(Re l) + 0.1 sum |l|^2",
            "forward_s": fw, "backward_s": bw, "solves_per_s": 512 / (fw + bw),
            "accuracy_fd": {"h": h, "directions": fd_checks},
            "launch_shape": {"wg_per_cu": shape["wg_per_cu"], "wide_n": shape["wide_n"]},
            "bucket_table": {"nw": table["nw"], "ns": table["ns"], "seconds": table["seconds"]},
            "plain_per_matrix": {"sample": "8 of the matrices, one hqr_schur call each, forward only",
                                 "solves_per_s": plain_rate},
            "speedup_vs_plain": (512 / (fw + bw)) / plain_rate}


def next_rows_run(seed):
    """The phases around the Schur reduction and the QZ variant, each timed
    (second of two calls) with its accuracy: the Householder Hessenberg
    reduction of a dense Gaussian n = 4096 matrix with Q (nominal 10/3 n^3 +
    4/3 n^3 flops), the eigenvectors of an n = 2048 matrix from its Schur form
    (residual ||A X - X L|| / (||A|| ||X||)), and the batched QZ variant on
    2048 random pairs of orders 16..64 (in LDS) and 256 pairs of order 256
    (global memory), Python packing of the pair lists included."""
    import numpy as np
    import torch
    import hqr_inputs as hi
    import paper_2007_03576_amd as hq
    dev = torch.device("cuda:0")
    out = {}
    g = torch.Generator(device=dev).manual_seed(seed)
    n = 4096
    A = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H, Q = hq.hessenberg(A)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    an = float(torch.linalg.norm(A))
    be = float(torch.linalg.norm(Q.t() @ A @ Q - H)) / an
    orth = float(torch.linalg.norm(Q.t() @ Q - torch.eye(n, dtype=Q.dtype, device=dev)))
    out["hessenberg"] = {"n": n, "s": dt, "tflops_nominal": (14.0 / 3.0) * n ** 3 / dt / 1e12,
                         "backward_rel": be, "orth": orth, "below_subdiag_zero": bool((torch.tril(H, -2) == 0).all())}
    del A, H, Q
    n = 2048
    Hn = hi.gaussian_hessenberg(n, seed=seed)
    Hd = torch.from_numpy(np.ascontiguousarray(Hn)).to(dev)
    T, Q, w, info = hq.schur(Hd)
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X = hq.eigenvectors(T, Q, w)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    Hc = Hd.to(torch.complex128)
    res = float(torch.linalg.norm(Hc @ X - X * w[None, :])) / (float(torch.linalg.norm(Hd)) *
                                                            float(torch.linalg.norm(X)))
    out["eigenvectors"] = {"n": n, "s": dt, "residual_rel": res, "schur_info": info}
    del Hd, T, Q, X, Hc
    rng = np.random.default_rng(seed)
    for name, count, lo, hi_ in (("qz_orders16_64", 2048, 16, 64), ("qz_order256", 256, 256, 256)):
        sizes = rng.integers(lo, hi_ + 1, size=count)
        Hs = [torch.from_numpy(np.triu(rng.standard_normal((k, k)), -1)).to(dev) for k in sizes]
        Ts = [torch.from_numpy(np.triu(rng.standard_normal((k, k)))).to(dev) for k in sizes]
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res_qz = hq.qz_batched(Hs, Ts)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        info_qz = res_qz[-1].cpu().numpy()
        # backward error of the first pair
        S0, T0, Q0, Z0 = res_qz[0][0], res_qz[1][0], res_qz[2][0], res_qz[3][0]
        bh = float(torch.linalg.norm(Q0.t() @ Hs[0] @ Z0 - S0)) / float(torch.linalg.norm(Hs[0]))
        bt = float(torch.linalg.norm(Q0.t() @ Ts[0] @ Z0 - T0)) / float(torch.linalg.norm(Ts[0]))
        out[name] = {"pairs": count, "orders": [lo, hi_], "s": dt, "pairs_per_s": count / dt,
                     "info_max": int(info_qz.max()), "first_pair_backward": [bh, bt]}
    torch.cuda.empty_cache()
    return out


def solve_line(workload, seed, steps, warmup, streams=2, small_shifts=0, cache=None):
    """`warmup` untimed and `steps` timed hqr_schur calls on the workload's
    matrix (one staged copy of H and of Q = I per call, so the timed region is
    solves only), then the accuracy of the last solve (backward error,
    orthogonality, and for a prescribed spectrum the distance of every
    computed eigenvalue to it and back), the run statistics, the kernel-class
    split and the roofline entries of the dominant kernel and of the
    FP64-MFMA update kernel."""
    import numpy as np
    import torch
    import paper_2007_03576_amd as hq
    from paper_2007_03576_amd import profiling
    spec = WORKLOADS[workload]
    n = spec["n"]
    dev = torch.device("cuda:0")
    H0d, ev = make_input(spec, seed, dev, cache, workload)  # row-major of H^T = column-major H
    params = {"ns": spec["ns"], "nw": spec["nw"], "streams": streams, "small_shifts": small_shifts}
    nsteps = warmup + steps
    Hs = [H0d.clone() for _ in range(nsteps)]
    Qs = [torch.eye(n, dtype=torch.float64, device=dev) for _ in range(nsteps)]
    wr = torch.empty(n, dtype=torch.float64, device=dev)
    wi = torch.empty_like(wr)
    infos = []
    for i in range(warmup):
        infos.append(hq.schur_colmajor(Hs[i].t(), Qs[i].t(), wr, wi, params=params))
    torch.cuda.synchronize()
    profiling.enable(True)
    profiling.reset()
    t0 = time.perf_counter()
    for i in range(warmup, nsteps):
        infos.append(hq.schur_colmajor(Hs[i].t(), Qs[i].t(), wr, wi, params=params))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = profiling.read()
    split = profiling.lds_split()
    profiling.enable(False)
    stats = hq.last_stats()
    dt = (t1 - t0) / steps
    assert all(i == 0 for i in infos), infos
    # accuracy of the last solve (outside the timed region)
    for i in range(nsteps - 1):
        Hs[i] = Qs[i] = None
    torch.cuda.empty_cache()
    T, Q, H0 = Hs[-1].t(), Qs[-1].t(), H0d.t()
    u = 2.0 ** -52
    hn = float(torch.linalg.norm(H0))
    be = float(torch.linalg.norm(Q.t() @ H0 @ Q - T)) / hn
    orth = float(torch.linalg.norm(Q.t() @ Q - torch.eye(n, dtype=Q.dtype, device=dev)))
    acc = {"backward_rel": be, "backward_u": be / u, "orth": orth, "bound_100nu": 100 * n * u}
    if ev is not None:
        from scipy.spatial import cKDTree
        w = wr.cpu().numpy() + 1j * wi.cpu().numpy()
        P, R = np.c_[w.real, w.imag], np.c_[np.real(ev), np.imag(ev)]
        acc["eig_dist_max_rel"] = max(cKDTree(R).query(P)[0].max(), cKDTree(P).query(R)[0].max()) / hn
    roof = profiling.roofline(prof, steps)
    roof["traffic"] = measured_traffic(roof["kernel"], workload)
    times = profiling.summary(prof, steps)
    times["lds_iteration"]["split"] = split
    out = {"workload": workload, "n": n, "ns": spec["ns"], "nw": spec["nw"], "steps": steps, "warmup": warmup,
           "ms_per_step": dt * 1e3, "value": 10.0 * n ** 3 / dt / 1e12, "unit": "TFLOP/s (10n^3 nominal)",
           "solves_per_s": 1.0 / dt, "accuracy": acc, "run_stats": stats, "roofline": roof, "kernel_times": times}
    del Hs, Qs, H0d, T, Q, H0
    torch.cuda.empty_cache()
    return out


def host_sample(spec, seed, target_n):
    """The workload's generator at order target_n, on the host."""
    import hqr_inputs as hi
    if spec["gen"] == "gaussian":
        return hi.gaussian_hessenberg(target_n, seed=seed)
    if spec["gen"] == "hessrand":
        return hi.hessrand(target_n, seed=seed)
    return hi.prescribed_hessenberg(target_n, seed=seed)[0]


def cpu_baseline(spec, H):
    """The oracle on a bounded sample of the same workload (same generator at
    a smaller order, the workload's shift count and window when they fit the
    sample, else the oracle's automatic ones), single thread; returns nominal
    TFLOP/s."""
    import oracle
    n = H.shape[0]
    ns, nw = (spec["ns"], spec["nw"]) if spec["nw"] <= n // 4 else (0, 0)
    t0 = time.perf_counter()
    T, Q, w, info, st = oracle.schur(H, want_q=True, ns=ns, nw=nw)
    dt = time.perf_counter() - t0
    assert info == 0
    par = f"ns={ns}, nw={nw}" if ns else "automatic ns and nw (the workload's window exceeds a quarter of the sample)"
    return {"value": 10.0 * n ** 3 / dt / 1e12, "unit": "TFLOP/s (10n^3 nominal)", "cores": 1,
            "kind": "oracle", "host_cpus": os.cpu_count(),
            "sample": f"one full solve of the workload's generator at n={n} ({par}, Q accumulated): {dt:.2f} s "
                      f"on one thread of a host with {os.cpu_count()} logical CPUs (the oracle is single-threaded C)"}


def lapack_context(H):
    """Context, not the oracle: the host's LAPACK real Schur driver (dgees
    through scipy, OpenBLAS on all its threads) on the same bounded sample as
    cpu_baseline.  dgees also runs the Hessenberg reduction and forms its
    orthogonal factor (on an input that is already Hessenberg), so it does
    more than the Schur phase alone."""
    import scipy
    import scipy.linalg as sl
    from threadpoolctl import threadpool_info
    n = H.shape[0]
    t0 = time.perf_counter()
    sl.schur(H, output="real")
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
    return {"value": 10.0 * n ** 3 / dt / 1e12, "unit": "TFLOP/s (10n^3 nominal)", "threads": threads,
            "kind": "LAPACK dgees (scipy %s, OpenBLAS)" % scipy.__version__,
            "sample": f"one real Schur decomposition of the same matrix as the oracle's sample (n={n}): {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="prescribed_hessenberg_n16384", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=2020)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other configuration and the batched, differentiation and next-row lines")
    ap.add_argument("--cpu-n", type=int, default=2048)
    ap.add_argument("--streams", type=int, default=2)
    ap.add_argument("--small-shifts", type=int, default=0)
    ap.add_argument("--extra-only", nargs="?", const="all", default=None, choices=["all", "batched", "grad", "next"],
                    help="only the batched and/or differentiation lines (for profiling those kernels)")
    ap.add_argument("--input-cache", default=None,
                    help="directory for the generated inputs: read when present, else written")
    ap.add_argument("--prepare-only", action="store_true",
                    help="only generate the workload's input into --input-cache")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="only run 5 plain device copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.copy_calib:
        import torch
        nel = args.copy_calib // 8
        a = torch.ones(nel, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": nel * 8, "copies": 5}))
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.extra_only:
        out = {}
        if args.extra_only in ("all", "batched"):
            out["batched"] = batched_run(args.seed)
        if args.extra_only in ("all", "grad"):
            out["grad"] = grad_run(args.seed)
        if args.extra_only in ("all", "next"):
            out["next_rows"] = next_rows_run(args.seed)
        print(json.dumps(out))
        return

    spec = WORKLOADS[args.workload]
    if args.prepare_only:
        import torch
        if not args.input_cache:
            print("--prepare-only needs --input-cache", file=sys.stderr)
            sys.exit(2)
        make_input(spec, args.seed, torch.device("cuda:0"), args.input_cache, args.workload)
        print(json.dumps({"prepared": args.workload, "cache": args.input_cache}))
        return
    line = solve_line(args.workload, args.seed, args.steps, args.warmup, args.streams, args.small_shifts,
                      args.input_cache)
    out = {
        "metric": "FP64 TFLOP/s (10n^3 nominal) & Schur solves/sec, batched+grad vs plain, 1 MI355X",
        "value": line["value"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": line["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": spec["n"], "ns": spec["ns"], "nw": spec["nw"],
                   "want_q": True, "seed": args.seed, "streams": args.streams,
                   "small_shifts": args.small_shifts or 2},
        "solves_per_s": line["solves_per_s"],
        "accuracy": line["accuracy"],
        "run_stats": line["run_stats"],
        "roofline": line["roofline"],
        "kernel_times": line["kernel_times"],
    }
    if not args.no_extra:
        # the other single-matrix configuration, then the batched and differentiated forms
        other = "gaussian_hessenberg_n4096" if args.workload != "gaussian_hessenberg_n4096" \
            else "prescribed_hessenberg_n16384"
        steps2, warm2 = (3, 1) if other == "gaussian_hessenberg_n4096" else (1, 0)
        out["other_config"] = solve_line(other, args.seed, steps2, warm2, args.streams, args.small_shifts)
        out["plain_solves_per_s"] = line["solves_per_s"]
        out["batched"] = batched_run(args.seed)
        out["grad"] = grad_run(args.seed)
        out["next_rows"] = next_rows_run(args.seed)
    if not args.no_cpu_baseline:
        H = host_sample(spec, args.seed, args.cpu_n)
        out["cpu_baseline"] = cpu_baseline(spec, H)
        out["lapack_context"] = lapack_context(H)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
