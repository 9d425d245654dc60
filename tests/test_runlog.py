"""The JSON-lines run log (host logic; a stand-in context on the CPU)."""
import json

import numpy as np

from paper_2608_00746_amd import inputs as I
from paper_2608_00746_amd import runlog


class _FakeSolver:
    """Advance moves time and steps and perturbs the energy total by a known
    relative amount; diag returns rows in the library's slot layout."""

    def __init__(self, ws):
        self.w = ws
        self.opts = ws[0].opts
        self.steps = 0

    def advance(self, n):
        self.steps += n

    def diag(self):
        d = np.zeros((len(self.w), 40))
        for i, w in enumerate(self.w):
            U = w.U.reshape(w.nU, -1)
            vol = float(np.prod(w.dx))
            d[i, :w.nU] = U.sum(axis=1) * vol
            d[i, w.N + w.ndim] *= 1.0 + 1e-9 * self.steps
            d[i, 32] = 0.25
            d[i, 33] = 0.5 / min(w.dx)
            d[i, 26] = 1e-3 * self.steps
            d[i, 27] = self.steps
        return d


def test_run_writes_a_line_per_block(tmp_path):
    ws = [I.random_state((12, 10), nphase=2, seed=1), I.random_state((9,), nphase=3, seed=2)]
    s = _FakeSolver(ws)
    path = tmp_path / "run.jsonl"
    recs = runlog.run(s, 25, 10, str(path), extra=lambda sv, k: {"probe": k}, sync=lambda: None)
    lines = [json.loads(l) for l in open(path)]
    assert len(lines) == len(recs) == 4          # before, 10, 20, 25
    assert [l["step"] for l in lines] == [0, 10, 20, 25]
    assert [l["probe"] for l in lines] == [0, 10, 20, 25]
    assert "cell_updates_per_s" not in lines[0]
    for l in lines[1:]:
        assert l["cell_updates_per_s"] > 0 and l["ms_per_step"] > 0
        assert l["hbm_frac_algorithmic"] > 0
    last = lines[-1]
    assert last["precision"] == "fp64" and last["N"] == [2, 3] and last["d"] == [1, 2]
    assert last["cells"] == 12 * 10 + 9 and last["instances"] == 2
    for i, w in enumerate(ws):
        r = last["instances_diag"][i]
        assert r["steps"] == 25 and abs(r["t"] - 0.025) < 1e-15
        # energy total drifted by 25e-9 relative, nothing else
        cons = r["conservation_rel"]
        assert len(cons) == w.N + w.ndim + 1
        assert abs(cons[w.N + w.ndim] - 25e-9) < 1e-15
        assert all(c == 0.0 for c in cons[:w.N + w.ndim])
        # N_I = out[32] / (min dx * out[33]) = 0.25 / 0.5
        assert abs(r["interface_thickness"] - 0.5) < 1e-15


def test_run_rejects_bad_blocks(tmp_path):
    ws = [I.random_state((8,), nphase=2, seed=3)]
    import pytest
    with pytest.raises(ValueError):
        runlog.run(_FakeSolver(ws), 10, 0, str(tmp_path / "x.jsonl"), sync=lambda: None)
