"""bench.py's host side, without a GPU: the one-GPU refusal, the roofline arithmetic and the
HBM-traffic table's link to the committed counter summaries."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_pair_roofline_arithmetic():
    pairs, ms = 133859 * 1070872, 99.0
    out = bench.pair_roofline("mixed", True, pairs, ms, "no-such-workload")
    assert out["achieved"] == pytest.approx(58 * pairs / (ms * 1e-3) / 1e12)
    assert out["frac"] == pytest.approx(out["achieved"] / 157.3)
    # the mix-adjusted ceiling of the probe summary: 256 CUs x 2.4 GHz over the CU clocks of a
    # pair (58 flops at 256 per clock, one exp and one rsqrt at 256 / cycles results per clock)
    clk = 58 / 256 + 8.19 / 256 + 8.32 / 256
    assert out["mix_adjusted"]["pairs_per_s_ceiling"] == pytest.approx(256 * 2.4e9 / clk, rel=2e-3)
    assert out["mix_adjusted"]["frac"] == pytest.approx(pairs / (ms * 1e-3) / out["mix_adjusted"]["pairs_per_s_ceiling"])
    assert out["traffic"] is None          # no counter run for this key
    assert out["kernel_sources_sha16"] == bench.kernel_sources_hash()
    f64 = bench.pair_roofline("fp64", True, pairs, 2 * ms, "no-such-workload")
    assert f64["frac"] == pytest.approx(58 * pairs / (2 * ms * 1e-3) / 1e12 / 78.6)
    assert "mix_adjusted" not in f64


def test_traffic_entries_name_their_counter_summary():
    """Each stored traffic figure is the one its committed summary states, for the sources
    hash the summary was taken on."""
    assert bench.PAIR_TRAFFIC
    for (workload, precision, sha), (nbytes, path) in bench.PAIR_TRAFFIC.items():
        text = open(os.path.join(ROOT, path)).read()
        assert sha in text, (path, sha)
        assert f"{nbytes} bytes" in text, (path, nbytes)
