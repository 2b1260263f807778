"""Host-side logic of bench.py (no GPU): the one-GPU guard, the roofline
arithmetic, and the rule that counter traffic is reported only for the stencil
sources it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_roofline_arithmetic():
    # 10 launches, 2 ms in all, 6.6e8 algorithmic bytes each, 65536 sites x 64 RHS
    r = bench.stencil_roofline("k_dslash_eo<IOBF>", 10, 2.0, 10 * 6.6e8, 65536, 64, "no such entry")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(6.6e9 / 2e-3 / 1e9, rel=1e-6)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["avg_launch_ms"] == pytest.approx(0.2)
    assert r["flop_per_launch"] == 1872 * 65536 * 64
    assert r["alu_tflops"] == pytest.approx(1872 * 65536 * 64 / 0.2e-3 / 1e12, rel=1e-3)
    assert r["traffic"] is None and r["traffic_gbps"] is None


def _tiles(L_x, slab):
    """The site-order tiles the autotuner may pick (its candidates and the default)."""
    out = set()
    for y in (1, 2, 3, 4, 6, 8):
        for t in (slab, slab // 2):
            if L_x % y == 0 and t >= 1 and slab % t == 0 and y * t * L_x <= 1024:
                out.add((y, t))
    return out


def test_committed_counters_belong_to_the_current_stencil():
    """profiles/stencil_traffic.json holds the calibrated FETCH_SIZE + WRITE_SIZE
    bytes of the dominant stencil for every tile the autotuner can pick at the
    two benchmark lattices; they must have been taken on the stencil sources as
    they are now (else the bench reports null traffic)."""
    d = json.load(open(os.path.join(ROOT, "profiles", "stencil_traffic.json")))
    keys = [bench.traffic_key("k_dslash_eo<IOBF>", 64, "24x24x24x48", t) for t in _tiles(24, 6) | {(2, 6)}]
    keys += [bench.traffic_key("k_dslash_eo<IOBF>", 64, "16x16x16x32", t) for t in _tiles(16, 4) | {(4, 4)}]
    for key in keys:
        assert d[key]["source_hash"] == bench.stencil_hash(), key
        t = bench.load_traffic(key)
        assert t == d[key]["bytes_per_launch"]
        assert t == pytest.approx(d[key]["read_bytes"] + d[key]["write_bytes"], abs=2)
        assert d[key]["fetch_factor"] > 0 and d[key]["write_factor"] > 0


def test_traffic_is_null_when_the_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "stencil_hash", lambda: "0000000000000000")
    key = bench.traffic_key("k_dslash_eo<IOBF>", 64, "24x24x24x48", (2, 6))
    assert bench.load_traffic(key) is None
    r = bench.stencil_roofline("k_dslash_eo<IOBF>", 1, 1.0, 1e9, 65536, 64, key)
    assert r["traffic"] is None and r["traffic_gbps"] is None
