"""Tile shapes and the autotuner: every x-strip width and y-tile shape (one
for all groups of instances, or one per group) gives the same states bitwise (a shape changes which workgroup computes a cell,
never its arithmetic), and mp_weno_autotune keeps the states, the time and
the step count, returns valid shapes, and the tuned solver reproduces the
untuned one bitwise."""
import os

import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I

pytestmark = pytest.mark.gpu


def _solver(ws, **kw):
    from paper_2608_00746_amd.binding import Solver
    return Solver(ws if isinstance(ws, list) else [ws], **kw)


def _cases():
    o = I.Options(flux=I.FLUX_HLL, cfl=0.2)
    return [I.random_state((45, 301), nphase=2, seed=81, lowp=0.0, opts=o),
            I.random_state((23, 130), nphase=3, seed=82, bc=1, lowp=0.0, opts=o),
            I.random_state((257,), nphase=2, seed=83, lowp=0.0, opts=o)]


def _run(ws, K, env):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        s = _solver(ws)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    for _ in range(K):
        s.step()
    out = [s.host(i).copy() for i in range(len(ws))]
    s.close()
    return out


@pytest.mark.parametrize("xs,ys", [(1, 0), (0, 1), (1, 1), (2, 2), ("2,1,0", "1,2")])
@pytest.mark.parametrize("precision", [I.PREC_FP64, I.PREC_MIXED])
def test_tile_shapes_bitwise(xs, ys, precision):
    ws = _cases()
    for w in ws:
        w.opts.precision = precision
    ref = _run(ws, 3, {"MPWENO_XSHAPE": 0, "MPWENO_YSHAPE": 0})
    env = {"MPWENO_XSHAPE": xs, "MPWENO_YSHAPE": ys}
    if isinstance(xs, str):
        # one entry per group ((d, N) = (1, 2), (2, 2), (2, 3)), a short list
        # repeating its last entry, and the tile order per group too
        env["MPWENO_XCD_SWIZZLE"] = "1,0"
    got = _run(ws, 3, env)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_autotune_keeps_state_and_results():
    ws = _cases()
    a = _solver(ws)
    b = _solver(ws)
    before = [a.host(i).copy() for i in range(len(ws))]
    ch = a.autotune(reps=2)
    assert ch.shape == (len(ws), 4)
    for i, w in enumerate(ws):
        assert np.array_equal(a.host(i), before[i])
        assert ch[i, 0] in (256, 128, 64)
        if w.ndim == 2:
            assert (ch[i, 1], ch[i, 2]) in ((16, 16), (32, 8), (16, 24))
        else:
            assert ch[i, 1] == 0 and ch[i, 2] == 0
        assert ch[i, 3] in (0, 1)
    assert (a.diag()[:, 27] == 0).all() and (a.diag()[:, 26] == 0).all()
    for _ in range(3):
        a.step()
        b.step()
    for i in range(len(ws)):
        assert np.array_equal(a.host(i), b.host(i)), i
    a.close()
    b.close()


def test_autotune_then_graph_replay():
    import torch
    ws = _cases()[:2]
    st = torch.cuda.Stream()
    a = _solver(ws, stream=st, use_graph=True)
    b = _solver(ws, stream=st)
    a.step()
    b.step()
    a.autotune(reps=1)          # drops the captured graph
    for _ in range(3):
        a.step()
        b.step()
        torch.cuda.synchronize()
    for i in range(len(ws)):
        assert np.array_equal(a.host(i), b.host(i)), i
    a.close()
    b.close()
