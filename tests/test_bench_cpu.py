"""Host-side logic of bench.py (CPU only): the one-GPU contract, and the
lookup of the stored HBM counter summary that fills roofline.traffic."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def _stored():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        return json.load(f)


def test_traffic_lookup_follows_the_kept_variant():
    t = _stored()
    from paper_2512_16889_amd.build import source_hash
    if t["kernel_source_sha256"] != source_hash():
        pytest.skip("the committed counters were taken from other kernel sources")
    k = t["kernels"]

    def mean_row(real, v):
        names = [f"void swf::row_d_kernel<{real}, 320, {v}, {s}>(swf::PassArgs)" for s in range(4)]
        return sum(k[n]["fetch_bytes"] + k[n]["write_bytes"] for n in names) / 4

    # the cached choice (row, y, z variants) of an autotuner cache line
    assert bench.stored_traffic(0, "mixed", 320, "deriv f32 ...: cached 3 0 0", None) == pytest.approx(mean_row("float", 3))
    assert bench.stored_traffic(0, "fp64", 320, "deriv f64 ...: cached 2 0 0", None) == pytest.approx(mean_row("double", 2))
    # or the fastest variant the autotuner timed
    report = "row v0 74.3 ms\nrow v1 72.2 ms\nrow v2 36.9 ms\nrow v3 36.1 ms\ncol1 v0 13.4 ms"
    assert bench.stored_traffic(0, "mixed", 320, report, None) == pytest.approx(mean_row("float", 3))
    col = k["void swf::col_d_kernel<float, 320, 0, 1, 0>(swf::PassArgs)"]
    assert bench.stored_traffic(1, "mixed", 320, report, None) == pytest.approx(col["fetch_bytes"] + col["write_bytes"])
    # a kernel that was never measured gives no traffic
    assert bench.stored_traffic(0, "mixed", 48, "cached 0 0 0", None) is None


def test_traffic_is_dropped_when_the_sources_change(monkeypatch):
    import paper_2512_16889_amd.build as b
    monkeypatch.setattr(b, "source_hash", lambda: "0" * 64)
    assert bench.stored_traffic(0, "mixed", 320, "cached 3 0 0", None) is None
