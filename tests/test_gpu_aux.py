"""Checkpoint and resume, the interface-thickness diagnostics and the run
log, on the GPU.

* Checkpoint: K steps, save (U and t per instance, to a file), K more steps;
  a fresh context restored from the file and run K steps reproduces the
  second half bitwise (states and times), because a step reads nothing but
  U and t (the CFL step, the time clip and instance retirement derive from
  them) and every reduction has a fixed order.  FP64 and mixed, a batch of
  1D and 2D instances of two and three phases, graph replay on.
* With the Phase-Field step the solve of Eq. (4) starts from the previous
  step's Q, which the checkpoint does not hold: a resumed run matches to
  the solver's tolerance (the bar of the Phase-Field parity, 1e-9 of the
  component scale), not bitwise.
* N_I of Eq. (30) from the diagnostics' two integrals against the oracle's
  definition on the same states (1e-12: the sums are taken in another order).
"""
import json

import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I
from test_gpu_parity import _scales

pytestmark = pytest.mark.gpu


def _solver(ws, graph=True):
    import torch
    from paper_2608_00746_amd.binding import Solver
    return Solver(ws, use_graph=graph, stream=torch.cuda.Stream())


def _batch(prec):
    o = I.Options(flux=I.FLUX_HLL, cfl=0.2, precision=prec)
    ws = I.batched(count=6, opts=o, select=[0, 1, 2])
    ws += [I.advection_1d(200, opts=o), I.shock_interface_n3(72, opts=o)]
    return ws


@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED], ids=["fp64", "mixed"])
def test_checkpoint_resume_bitwise(tmp_path, prec):
    K = 20
    ws = _batch(prec)
    a = _solver(ws)
    a.advance(K)
    path = str(tmp_path / "ck.npz")
    ck = a.checkpoint(path)
    a.advance(K)
    da = a.diag()
    Ua = [a.host(i).copy() for i in range(len(ws))]
    a.close()

    b = _solver(_batch(prec))
    b.restore(path)
    db0 = b.diag()
    assert np.array_equal(db0[:, 26], ck["t"])
    b.advance(K)
    db = b.diag()
    for i in range(len(ws)):
        assert np.array_equal(b.host(i), Ua[i]), i
    assert np.array_equal(db[:, 26], da[:, 26])
    # the step count is the context's own
    assert np.array_equal(db[:, 27], da[:, 27] - ck["steps"])
    b.close()


def test_checkpoint_resume_with_phase_field(tmp_path):
    K = 4
    w = I.pf_bubble((48, 40), 2, width=1.5)
    a = _solver([w], graph=False)
    for _ in range(K):
        a.step()
    path = str(tmp_path / "pf.npz")
    a.checkpoint(path)
    for _ in range(K):
        a.step()
    Ua = a.host(0).reshape(w.nU, -1).copy()
    a.close()
    b = _solver([I.pf_bubble((48, 40), 2, width=1.5)], graph=False)
    b.restore(path)
    for _ in range(K):
        b.step()
    Ub = b.host(0).reshape(w.nU, -1)
    b.close()
    err = np.abs(Ua - Ub).max(axis=1) / _scales(w, Ua)
    print("PF resume err", np.array2string(err, precision=2))
    assert (err <= 1e-9).all(), err


def test_restore_rejects_a_foreign_checkpoint(tmp_path):
    ws = _batch(I.PREC_FP64)
    a = _solver(ws[:2])
    ck = a.checkpoint()
    a.close()
    b = _solver(ws)
    with pytest.raises(ValueError):
        b.restore(ck)
    b.close()


@pytest.mark.parametrize("make", [
    lambda: I.pf_bubble((96,), 2, width=2.0),
    lambda: I.pf_bubble((64, 48), 3, width=1.5),
    lambda: I.shock_vessel_bubble_3d(40, 20, 20),
], ids=["1d", "2d", "3d"])
def test_interface_thickness_vs_oracle(oracle, make):
    w = make()
    w.opts.phase_field = 0
    s = _solver([w], graph=False)
    for _ in range(3):
        s.step()
    ni = s.interface_thickness()[0]
    U = s.host(0).reshape(w.nU, -1)
    s.close()
    ref = oracle.interface_thickness(U[w.N + w.ndim + 1], w.n, w.dx)
    print(w.name, "N_I", ni, ref)
    assert ref > 0.5
    assert abs(ni - ref) <= 1e-12 * ref


def test_run_log_on_the_gpu(tmp_path):
    from paper_2608_00746_amd import runlog
    ws = _batch(I.PREC_MIXED)
    s = _solver(ws)
    path = tmp_path / "run.jsonl"
    runlog.run(s, 48, 16, str(path))
    s.close()
    lines = [json.loads(l) for l in open(path)]
    assert [l["step"] for l in lines] == [0, 16, 32, 48]
    for l in lines[1:]:
        assert l["cell_updates_per_s"] > 0 and 0 < l["hbm_frac_algorithmic"] < 1
        for w, r in zip(ws, l["instances_diag"]):
            assert r["steps"] == l["step"] and r["nonfinite"] == 0
            assert r["sum_alpha_err"] <= 1e-8
            if all(b == (I.BC_PERIODIC, I.BC_PERIODIC) for b in w.bc):
                assert max(r["conservation_rel"][:w.N]) <= 1e-12   # phase masses
