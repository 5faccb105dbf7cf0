"""Host-side checks of the benchmark script (no GPU): the counter figures it
reports belong to the kernel sources in the tree, the stored full-size digests
parse and cover every benchmarked workload, and a request for more than one
GPU is refused before anything touches a device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2604_06947_amd import plans  # noqa: E402


@pytest.mark.parametrize("key", sorted(plans.COUNTERS))
def test_counter_figures_belong_to_the_current_sources(key):
    """The bench reports a kernel's counter figures only while its sources hash
    to the value recorded with them; every recorded entry must be current, so
    that no figure on the bench line is silently dropped."""
    c = plans.COUNTERS[key]
    assert c["sources_sha"] == bench.kernel_sources_sha(c["sources"]), key


def test_counter_fields_follow_the_hash():
    f = bench.counter_fields(plans, "w2", 11.0e-6)
    assert f["traffic"] == plans.COUNTERS["w2"]["traffic_bytes"]
    assert 0.0 < f["valu_issue_frac"] < 1.0 and 0.0 < f["hbm_counter_frac"] < 1.0
    saved = plans.COUNTERS["w2"]["sources_sha"]
    try:
        plans.COUNTERS["w2"]["sources_sha"] = "0" * 16
        g = bench.counter_fields(plans, "w2", 11.0e-6)
        assert g["traffic"] is None and g["valu_issue_frac"] is None
    finally:
        plans.COUNTERS["w2"]["sources_sha"] = saved


def test_roofline_constants():
    # 256 CUs x 64 lanes x 2.4 GHz: one integer operation per lane and cycle
    assert abs(bench.ALU_PEAK_TOPS - 39.3216) < 1e-9
    assert bench.SIMDS == 1024 and bench.CLOCK_HZ == 2.4e9
    assert bench.HBM_PEAK_GBS == 8000.0 and bench.FP64_PEAK_TFLOPS == 78.6


def test_golden_digests_cover_the_benchmarked_workloads():
    G = bench.golden()
    for key in ("w1", "w2", "w3_r0.01", "w3_r0.001", "w3_r0.0001", "w6"):
        assert key in G, key
    assert sum(1 for k in G if k.startswith("w4_")) == 4096
    w5 = [k for k in G if k.startswith("w5_")]
    assert len(w5) == 533
    for n, steps, _, sha in G.values():
        assert n > 0 and steps >= 0 and len(sha) == 64


def test_percentiles_with_and_without_service_times():
    import numpy as np
    lat = np.arange(1, 101, dtype=float)
    out = bench._pct(lat, lat / 2)
    assert out["p50_latency_s"] == np.percentile(lat, 50)
    assert out["p99_service_s"] == np.percentile(lat / 2, 99)
    assert set(bench._pct(lat)) == {"p50_latency_s", "p99_latency_s"}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
