"""Host logic of bench.py (no GPU): the counter-table lookup behind
roofline.traffic and the ALU roofline, the state-difference metric of the
precision comparison, and the one-GPU guard."""
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
    # a row of other sources: nothing from it (the counters describe that code)
    c = bench.stage_counters("wl", "fp64", "x128/y16x16/xcd")
    assert c == {"traffic": None, "flops64": None, "flops32": None, "valu": None}
    # no row for the tiles: nothing
    c = bench.stage_counters("wl", "fp64", "x256/y16x24/plain")
    assert c["traffic"] is None and c["flops64"] is None
    # unknown workload or precision: nothing
    c = bench.stage_counters("other", "fp64", "x64/y16x16/plain")
    assert c == {"traffic": None, "flops64": None, "flops32": None, "valu": None}
    c = bench.stage_counters("wl", "mixed", "x64/y16x16/plain")
    assert c["flops32"] == 360.0 and c["traffic"] == (90 + 20) * 1024.0


def test_tiles_key_and_env():
    """The tile choice as the bench line reports it and as --tiles takes it:
    one entry when every group agrees, else one per group of (d, N) in
    ascending order (the library's group order), whatever the instance
    order."""
    import numpy as np
    from types import SimpleNamespace as NS
    ws = [NS(ndim=2, N=3), NS(ndim=1, N=2), NS(ndim=2, N=2), NS(ndim=2, N=3)]
    args = NS(tiles=None)
    same = np.array([[128, 16, 16, 1]] * 3 + [[128, 16, 16, 1]])
    same[1] = [128, 0, 0, 1]
    # a 1D group has no y tile (0 x 0)
    assert bench.tiles_key(args, ws, same) == "x128/y0x0/xcd,x128/y16x16/xcd,x128/y16x16/xcd"
    t = np.array([[64, 32, 8, 0], [256, 0, 0, 1], [128, 16, 24, 1], [64, 32, 8, 0]])
    key = bench.tiles_key(args, ws, t)
    assert key == "x256/y0x0/xcd,x128/y16x24/xcd,x64/y32x8/plain"
    env = bench.tiles_env(key)
    assert env == {"MPWENO_XSHAPE": "0,1,2", "MPWENO_YSHAPE": "0,2,1",
                   "MPWENO_XCD_SWIZZLE": "1,1,0"}
    two = [NS(ndim=2, N=2), NS(ndim=2, N=3)]
    assert bench.tiles_key(args, two, np.array([[128, 16, 16, 1]] * 2)) == "x128/y16x16/xcd"
    assert bench.tiles_env("x128/y16x16/xcd") == {
        "MPWENO_XSHAPE": "1", "MPWENO_YSHAPE": "0", "MPWENO_XCD_SWIZZLE": "1"}
    assert bench.tiles_key(NS(tiles="x64/y16x16/plain"), two, None) == "x64/y16x16/plain"
    assert bench.tiles_key(args, two, None) == "default"


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


def test_state_difference_metric():
    """L1 and Linf per kind of component over uneven instances."""
    import numpy as np
    from paper_2608_00746_amd import inputs as I
    ws = [I.random_state((12, 10), nphase=2, seed=1), I.random_state((9, 7), nphase=3, seed=2)]
    a = [w.U.copy() for w in ws]
    b = [w.U.copy() for w in ws]
    d = bench.state_difference(ws, a, b)
    assert all(v == 0.0 for v in d["L1_rel"].values())
    # perturb the energy of one cell of the second instance by 1e-9 of it
    w = ws[1]
    a[1].reshape(w.nU, -1)[w.N + w.ndim, 5] *= 1 + 1e-9
    d = bench.state_difference(ws, a, b)
    assert d["L1_rel"]["m"] == 0.0 and d["L1_rel"]["alpha"] == 0.0
    E = [x.reshape(v.nU, -1)[v.N + v.ndim] for x, v in zip(b, ws)]
    vol = [float(np.prod(v.dx)) for v in ws]
    ref = 1e-9 * abs(E[1][5]) * vol[1] / sum(np.abs(e).sum() * v for e, v in zip(E, vol))
    assert abs(d["L1_rel"]["rho_E"] - ref) <= 1e-6 * ref
    assert abs(d["Linf_rel"]["rho_E"] - 1e-9 * abs(E[1][5]) / max(np.abs(e).max() for e in E)) \
        <= 1e-6 * d["Linf_rel"]["rho_E"]
