"""CPU checks of bench.py's host-side helpers: the committed counter record
is used only for the kernel source and launch parameters it was taken with,
the probe summary is parsed, the roofline arithmetic follows its
definitions, and a multi-GPU request is refused."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_probe_summary_is_parsed():
    assert bench.probe_ceiling("copy", 27, "GB_per_s") > 1000
    assert bench.probe_ceiling("gather") > 1e10
    assert bench.probe_ceiling("no-such-probe") is None


def test_traffic_record_needs_matching_source_and_parameters():
    import hashlib
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_2e24.json")))["kernels"]
    for kernel, r in rec.items():
        t = bench.measured_traffic(kernel, r["launch_params"])
        current = hashlib.sha256(open(os.path.join(ROOT, r["source"]), "rb").read()).hexdigest() == r["sha256"]
        want = r["read_bytes"] + r["write_bytes"]
        assert t == (want if current else None), kernel
        # the bytes are the request counts times the request sizes
        q = r["requests"]
        assert r["read_bytes"] == 32 * q["rd32"] + 64 * q["rd64"] + 128 * q["rd128"], kernel
        assert r["write_bytes"] == 32 * (q["wr"] - q["wr64"]) + 64 * q["wr64"], kernel
        other = dict(r["launch_params"] or {}, lr_per_wave1=12345)
        assert bench.measured_traffic(kernel, other) is None, kernel
    assert bench.measured_traffic("k_not_profiled", None) is None


def test_kernel_roofline_arithmetic():
    work = {"n": 1 << 24, "q": 1 << 24, "graph_n": 1 << 22, "graph_nnz": 1 << 26, "graph_m": 1 << 25}
    r = bench.kernel_roofline("k_walk1<true>", 1.0, 3.0, work, None)
    bpu, _, units = bench.ALG_BYTES["k_walk1<true>"]
    assert r["units_per_launch"] == units(work) == 1 << 25
    assert abs(r["achieved"] - bpu * (1 << 25) / 1e-3 / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / bench.HBM_PEAK_GBS) < 1e-12
    assert abs(r["random_frac"] - (1 << 25) / 1e-3 / r["random_ceiling_per_s"]) < 1e-12
    assert bench.kernel_roofline("k_unknown", 1.0, 1.0, work, None)["achieved"] is None


def test_multi_gpu_request_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def test_small_first_moves_whole_trees():
    """The 4096-tree batch handed over with its small trees first: every
    tree keeps its parents and its queries, only the tree order changes."""
    import numpy as np
    import gen
    b = gen.forest_batch(120, seed=3, log2_min=6, log2_max=14, qlog2_min=0, qlog2_max=6)
    limit = 4096
    r = bench._small_first(b, limit)
    order = np.argsort(b["sizes"] > limit, kind="stable")
    k = int(np.sum(b["sizes"] <= limit))
    assert 0 < k < len(order)
    assert (r["sizes"][:k] <= limit).all() and (r["sizes"][k:] > limit).all()
    assert r["offsets"][0] == 0 and r["offsets"][-1] == b["offsets"][-1]
    qs = np.searchsorted(b["qtree"], np.arange(len(order) + 1))
    rqs = np.searchsorted(r["qtree"], np.arange(len(order) + 1))
    for i, t in enumerate(order):
        assert np.array_equal(r["parent"][r["offsets"][i]:r["offsets"][i + 1]],
                              b["parent"][b["offsets"][t]:b["offsets"][t + 1]])
        assert np.array_equal(r["qx"][rqs[i]:rqs[i + 1]], b["qx"][qs[t]:qs[t + 1]])
        assert np.array_equal(r["qy"][rqs[i]:rqs[i + 1]], b["qy"][qs[t]:qs[t + 1]])
