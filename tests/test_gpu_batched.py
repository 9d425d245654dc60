"""Many uneven instances in one context: every sweep, reduction and RK stage
is one launch per (N, d) group over the tiles of all its instances.

* L(U) of every instance of a mixed batch (1D and 2D, N = 2 and 3, uneven
  sizes, ragged tiles) matches the oracle to the FP64 bar;
* a batched run reproduces solo runs of the same instances bitwise (states,
  CFL steps, diagnostics): batching changes which workgroup computes a tile,
  never the arithmetic of a cell or the order of a reduction;
* per-instance external time steps and per-instance end times;
* the CFL step a step takes from its first x sweep equals mp_weno_dt's;
* the 256-instance shock-bubble sweep stays finite and admissible, and its
  sampled instances match their solo runs bitwise.
"""
import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I
from conftest import oracle_problem
from test_gpu_parity import TOL, TOL_RAW_RHS, _rel_err, _scales

pytestmark = pytest.mark.gpu


def _batch_fp64():
    o = I.Options(flux=I.FLUX_HLL, cfl=0.2)
    ws = [
        I.random_state((300,), nphase=2, seed=71, lowp=0.0, opts=o),
        I.random_state((24, 280), nphase=2, seed=72, lowp=0.0, opts=o),
        I.random_state((137,), nphase=3, seed=73, bc=1, lowp=0.0, opts=o),
        I.random_state((40, 100), nphase=3, seed=74, lowp=0.0, opts=o),
        I.random_state((7, 9), nphase=2, seed=75, bc=1, lowp=0.0, opts=o),
        I.batched_instance(64, 3, 0.15, 1.5e9, opts=o),
        I.random_state((5,), nphase=2, seed=76, lowp=0.0, opts=o),
        I.batched_instance(96, 2, 0.1, 8e8, opts=o),
    ]
    for w in ws:
        w.t_end = 0.0
    return ws


def _solver(ws, **kw):
    from paper_2608_00746_amd.binding import Solver
    return Solver(ws, **kw)


def test_batched_rhs_vs_oracle(oracle):
    ws = _batch_fp64()
    s = _solver(ws)
    L = [x.cpu().numpy().reshape(-1) for x in s.rhs()]
    s.close()
    for w, Lg in zip(ws, L):
        pb = oracle_problem(oracle, w)
        U = w.U.reshape(-1)
        Lo = pb.rhs(U)
        dt = pb.dt(U, 0.0)
        sc = _scales(w)
        inc = dt * np.abs((Lg - Lo).reshape(w.nU, -1)).max(axis=1) / sc
        Lmax = np.abs(Lo.reshape(w.nU, -1)).max(axis=1)
        raw = _rel_err(Lg, Lo, w.nU)
        significant = dt * Lmax > 1e-10 * sc
        print(w.name, w.n, "batched rhs dt-scaled err:", np.array2string(inc, precision=2))
        assert np.isfinite(Lg).all()
        assert (inc <= TOL).all(), (w.name, inc)
        assert (raw[significant] <= TOL_RAW_RHS).all(), (w.name, raw)


@pytest.mark.parametrize("precision", [I.PREC_FP64, I.PREC_MIXED])
@pytest.mark.parametrize("graph", [False, True])
def test_batched_bitwise_vs_solo(precision, graph):
    import torch
    ws = _batch_fp64()
    for w in ws:
        w.opts.precision = precision
    st = torch.cuda.Stream()
    b = _solver(ws, stream=st, use_graph=graph)
    solos = [_solver([w], stream=st) for w in ws]
    K = 5
    for k in range(K):
        db = b.dt()
        for i, s in enumerate(solos):
            assert db[i] == s.dt()[0], (k, i)
        b.step()
        for s in solos:
            s.step()
    dg = b.diag()
    for i, (w, s) in enumerate(zip(ws, solos)):
        assert np.array_equal(b.host(i), s.host(0)), (w.name, i)
        ds = s.diag()[0]
        assert np.array_equal(dg[i], ds), (w.name, i)
        assert dg[i][27] == K and dg[i][25] == 0
    b.close()
    for s in solos:
        s.close()


@pytest.mark.parametrize("graph", [False, True])
def test_cfl_step_of_the_first_sweep_equals_the_cfl_pass(graph):
    """In 2D and 3D a step takes its CFL step from the rates its first x
    sweep reduces (no pass of its own over U^n); mp_weno_dt takes it from a
    pass over U^n.  Both evaluate the same rate per cell and a maximum, so a
    run on its own steps and a run fed mp_weno_dt's steps agree bitwise
    (states and times), over 16 steps (one captured run with graphs)."""
    import torch
    ws = _batch_fp64() + [I.shock_vessel_bubble_3d(40, 20, 20)]
    ws[-1].t_end = 0.0
    st = torch.cuda.Stream()
    a = _solver(ws, stream=st, use_graph=graph)
    b = _solver(ws, stream=st)
    K = 16
    t = np.zeros(len(ws))
    a.advance(K)
    for _ in range(K):
        dt = b.dt()
        t = t + dt
        b.step(dt)
    da = a.diag()
    assert np.array_equal(da[:, 26], t)
    for i, w in enumerate(ws):
        assert np.array_equal(a.host(i), b.host(i)), (w.name, i)
    assert (da[:, 27] == K).all()
    a.close()
    b.close()


def test_batched_external_dt_and_end_time():
    ws = _batch_fp64()
    n = len(ws)
    b = _solver(ws)
    solos = [_solver([w]) for w in ws]
    dts = np.array([s.dt()[0] for s in solos]) * np.linspace(0.5, 0.9, n)
    b.step(dts)
    for i, s in enumerate(solos):
        s.step(float(dts[i]))
        assert np.array_equal(b.host(i), s.host(0)), i
    d = b.diag()
    assert np.array_equal(d[:, 26], dts)
    for s in solos:
        s.close()
    b.close()
    # per-instance end times clip the CFL step of each instance on its own
    ws = _batch_fp64()
    dcfl = _solver(ws).dt()
    for i, w in enumerate(ws):
        w.t_end = dcfl[i] * (0.25 if i % 2 else 4.0)
    b = _solver(ws)
    got = b.dt()
    want = np.where(np.arange(n) % 2 == 1, dcfl * 0.25, dcfl)
    assert np.allclose(got, want, rtol=1e-15, atol=0.0)
    b.close()


def test_batched_sweep_256():
    """The 256-instance sweep (64..512 cells a side, N = 2 or 3, mixed
    precision): a few steps of the whole batch; the smallest instances are
    rerun alone and compared bitwise."""
    ws = I.batched()
    cells = sum(w.ncells for w in ws)
    assert len(ws) == 256 and cells > 2.5e7
    b = _solver(ws, use_graph=False)
    K = 3
    for _ in range(K):
        b.step()
    d = b.diag()
    assert (d[:, 25] == 0).all()
    assert (d[:, 27] == K).all()
    eps = np.finfo(float).eps
    assert (d[:, 21] >= 0).all() and (d[:, 22] >= 0).all()
    assert (d[:, 23] <= 1 + 1e-12).all() and (d[:, 24] > 0).all()
    assert (d[:, 20] <= 64 * eps).all()
    n = np.array([w.n[0] for w in ws])
    for i in list(np.argsort(n)[:3]) + [int(np.argmax(n))]:
        s = _solver([ws[i]])
        for _ in range(K):
            s.step()
        assert np.array_equal(b.host(i), s.host(0)), ws[i].name
        s.close()
    b.close()
