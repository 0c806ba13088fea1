"""Host-side logic of bench.py (no GPU): the k-set size, the counter lookup
tied to the kernel source, the isolated-time lookup in the autotune cache and
the one-GPU guard."""
import json
import os
import subprocess
import sys

import bench


def test_half_space_size():
    # |n_a| <= m without the origin, one of each +-n pair
    for m in (1, 5, 24):
        assert bench.n_half_space((m, m, m)) == ((2 * m + 1) ** 3 - 1) // 2
    assert bench.n_half_space((2, 3, 4)) == (5 * 7 * 9 - 1) // 2
    assert bench.n_half_space((24, 24, 24)) == 58824
    # brute force on a small grid: one of each +-n pair, origin excluded
    pts = {(a, b, c) for a in range(-2, 3) for b in range(-3, 4) for c in range(-1, 2)} - {(0, 0, 0)}
    half = {p for p in pts if p > (0, 0, 0)}
    assert len(half) == len(pts) // 2 == bench.n_half_space((2, 3, 1))


def test_traffic_only_for_the_profiled_source():
    h = bench.kernel_source_hash()
    with open(os.path.join(bench.PROFILES, "traffic_c3.json")) as f:
        d = json.load(f)
    got = bench.traffic_from_profiles("force_mm", h)
    if d.get("kernel_source_hash") == h:
        assert got == d["kernels"]["force_mm"]["hbm_bytes_per_launch"] and got > 0
    else:
        assert got is None
    assert bench.traffic_from_profiles("force_mm", "0" * 16) is None
    assert bench.traffic_from_profiles("no_such_kernel", h) is None


def test_isolated_time_from_the_autotune_cache(tmp_path):
    cache = tmp_path / "tune.jsonl"
    times = {"bwd6_kc3_x1": 294.6, "bwd6_kc3_x0": 295.0, "bwd6_kc6_x1": 292.0, "bwd3_kc4": 340.0,
             "fwd_mfma_ct2_1024_x1": 161.5, "fwd_mfma_ct2_768_x1": 159.0}
    cache.write_text(json.dumps({"key": "k0", "times_us": {"bwd6_kc3_x1": 1.0}}) + "\n" +
                     json.dumps({"key": "k1", "times_us": times}) + "\n")
    desc = "fwd=mfma-fold ct=2 nt=3 xcd=1 blocks~1024 bwd=mfma-fold-eyl xcd=1 kc=3 kgrid=25x49x49 precision=fp64"
    # the last line is the plan's; the adjoint entry matches block order and chunking
    assert bench._isolated_us(str(cache), desc, "force_mm") == 294.6
    assert bench._isolated_us(str(cache), desc, "sfac_mm") == 161.5
    # automatic chunking: the best of that block order
    auto = desc.replace("kc=3", "kc=auto")
    assert bench._isolated_us(str(cache), auto, "force_mm") == 292.0
    # a plan on other kernels, or no cache
    assert bench._isolated_us(str(cache), desc.replace("bwd=mfma-fold-eyl", "bwd=mfma-fold-16"),
                              "force_mm") is None
    assert bench._isolated_us(str(tmp_path / "missing.jsonl"), desc, "force_mm") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
