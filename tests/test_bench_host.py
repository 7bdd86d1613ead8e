"""Host-side checks of bench.py's contract (no GPU needed): the multi-GPU
refusal, and the HBM-traffic figure read from the committed rocprofv3
summary, which is valid only while the HIP sources match its hash."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_measured_traffic_follows_the_source_hash():
    """Bytes per launch while the summary's hash matches the HIP sources,
    None otherwise (then the bench reports traffic as null)."""
    import glob
    import hashlib
    import json
    import bench
    path = os.path.join(ROOT, "profiles", "k_iter_gaussian_hessenberg_n4096.md")
    rec = [json.loads(l.split(":", 1)[1]) for l in open(path) if l.startswith("pmc-json:")][-1]
    assert rec["read_bytes_per_launch"] > 0 and rec["write_bytes_per_launch"] > 0
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2007_03576_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h")):
            h.update(open(f, "rb").read())
    t = bench.measured_traffic("k_iter")
    if h.hexdigest() == rec["sources_sha256"]:
        assert t == rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
    else:
        assert t is None
    assert bench.measured_traffic("k_update") is None


def test_profile_summaries_name_their_commands():
    prof = os.path.join(ROOT, "profiles")
    names = [f for f in os.listdir(prof) if f.endswith(".md")]
    assert names
    for f in names:
        text = open(os.path.join(prof, f)).read()
        assert "rocprofv3 --kernel-trace --stats" in text, f
        assert "python3 bench.py" in text, f


def test_input_cache_round_trip(tmp_path):
    """--input-cache: the first call generates and writes the input, the
    second reads back the same matrix and spectrum (host tensors here)."""
    import numpy as np
    import torch
    import bench
    spec = bench.WORKLOADS["prescribed_hessenberg_n256"]
    a, ev = bench.make_input(spec, 11, torch.device("cpu"), str(tmp_path), "prescribed_hessenberg_n256")
    assert (tmp_path / "prescribed_hessenberg_n256_11.npz").exists()
    b, ev2 = bench.make_input(spec, 11, torch.device("cpu"), str(tmp_path), "prescribed_hessenberg_n256")
    assert torch.equal(a, b)
    assert np.array_equal(np.asarray(ev), np.asarray(ev2))
    c, ev3 = bench.make_input(spec, 11, torch.device("cpu"))
    assert torch.equal(a, c)
    # Gaussian inputs carry no spectrum
    g, gev = bench.make_input(bench.WORKLOADS["gaussian_hessenberg_n4096"], 3, torch.device("cpu"), str(tmp_path), "g")
    g2, gev2 = bench.make_input(bench.WORKLOADS["gaussian_hessenberg_n4096"], 3, torch.device("cpu"), str(tmp_path), "g")
    assert gev is None and gev2 is None and torch.equal(g, g2)
