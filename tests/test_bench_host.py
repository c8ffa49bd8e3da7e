"""Host-side checks of bench.py (no GPU): its flop constants are the CPU
oracle's own operation counts, and it refuses more than one GPU."""
import os
import subprocess
import sys

import pytest

from paper_1307_6488_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("index", [2, 3])
def test_rhs_flop_constants_match_oracle_count(orc, index):
    w = I.workload(index, n_override=12)
    counts = orc.count_rhs_flops(w.params, w.grid, w.make_state(), (4, 5, 6))
    assert sum(counts) == bench.RHS_FLOPS[w.params.fd_order]


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_null_once_kernel_sources_change(monkeypatch):
    w = "brill-lindquist-128^3-o4-upwind"
    for tile, m in bench.MEASURED_TRAFFIC[w].items():
        monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: m["sources_sha256"])
        assert bench.measured_traffic(w, tile) == pytest.approx((m["fetch_kib"] * 2.0 + m["write_kib"]) * 1024)
        assert bench.measured_traffic(w, "64x64") is None
        assert bench.measured_traffic("no-such-workload", tile) is None
        monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
        assert bench.measured_traffic(w, tile) is None


def test_profile_summaries_cite_the_recorded_counters():
    """Each recorded traffic entry has a rocprofv3 summary under profiles/
    that names the same kernel-sources hash and the same counter readings."""
    prof = os.path.join(ROOT, "profiles")
    texts = [open(os.path.join(prof, f)).read() for f in os.listdir(prof) if f.endswith(".md")]
    for w, recs in bench.MEASURED_TRAFFIC.items():
        for tile, m in recs.items():
            hits = [t for t in texts if m["sources_sha256"] in t and tile in t]
            assert hits, f"no profile names the hash recorded for {w} {tile}"
            fetch = f"{int(m['fetch_kib'] / 1e3):,}".replace(",", " ")        # thousands of KiB, e.g. "1 164"
            write = f"{int(m['write_kib'] / 1e3):,}".replace(",", " ")
            assert any(fetch in t and write in t for t in hits), (w, tile, fetch, write)
