"""Host logic of bench.py (no GPU): the counter-table lookup behind
roofline.traffic and the ALU roofline, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _table(tmp_path, rows):
    p = tmp_path / "stage_counters.md"
    head = ["| workload | precision | tiles | source | fetch KiB | write KiB | f64 | f32 | valu |",
            "|---|---|---|---|---|---|---|---|---|"]
    p.write_text("\n".join(["# test table", ""] + head + rows) + "\n")
    return str(p)


def test_stage_counters_lookup(tmp_path, monkeypatch):
    key = bench.kernel_source_hash()
    rows = ["| wl | fp64 | x64/y16x16/plain | %s | 100 | 28 | 1900 | 10 | 2000 |" % key,
            "| wl | fp64 | x128/y16x16/xcd | 0000000000000000 | 300 | 50 | 1800 | 9 | 1950 |",
            "| wl | mixed | x64/y16x16/plain | %s | 90 | 20 | 1500 | 360 | 2100 |" % key]
    monkeypatch.setattr(bench, "COUNTER_TABLE", _table(tmp_path, rows))
    # exact row of this source: traffic = (fetch + write) KiB in bytes
    c = bench.stage_counters("wl", "fp64", "x64/y16x16/plain")
    assert c["traffic"] == (100 + 28) * 1024.0
    assert (c["flops64"], c["flops32"], c["valu"]) == (1900.0, 10.0, 2000.0)
    # a row of other sources: its flops may serve, its traffic never
    c = bench.stage_counters("wl", "fp64", "x128/y16x16/xcd")
    assert c["traffic"] is None and c["flops64"] == 1800.0
    # no row for the tiles: the workload's flops, no traffic
    c = bench.stage_counters("wl", "fp64", "x256/y16x24/plain")
    assert c["traffic"] is None and c["flops64"] is not None
    # unknown workload or precision: nothing
    c = bench.stage_counters("other", "fp64", "x64/y16x16/plain")
    assert c == {"traffic": None, "flops64": None, "flops32": None, "valu": None}
    c = bench.stage_counters("wl", "mixed", "x64/y16x16/plain")
    assert c["flops32"] == 360.0 and c["traffic"] == (90 + 20) * 1024.0


def test_stage_counters_without_table(monkeypatch, tmp_path):
    monkeypatch.setattr(bench, "COUNTER_TABLE", str(tmp_path / "missing.md"))
    assert bench.stage_counters("wl", "fp64", "x64/y16x16/plain")["traffic"] is None


def test_source_hash_tracks_the_kernel_sources():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert h == bench.kernel_source_hash()


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
