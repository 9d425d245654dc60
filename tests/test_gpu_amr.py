"""GPU two-level coupling (mp_weno_amr_link) against the oracle's composite
step (oracle/amr.py) on the same seeded smooth states:
* states of the coarse grid and of the block (interior and ring) after
  three steps with a common external dt, at the FP64 window bar of the
  parity suite (2D N = 2 HLL, 2D N = 3 HLLC, 1D N = 2);
* with the CFL step: linked instances take one dt, the composite totals of
  m_p, rho u, rho E hold to rounding over 40 steps, sum alpha stays 1;
* captured 16-step graphs reproduce eager steps bitwise;
* a block too close to the coarse boundary is rejected."""
import numpy as np
import pytest

from oracle import amr
from paper_2608_00746_amd import inputs as I
from amr_states import two_level
from conftest import oracle_problem

pytestmark = pytest.mark.gpu


def _solver(ws, links, use_graph=False):
    import torch
    from paper_2608_00746_amd.binding import Solver
    s = Solver(ws, use_graph=use_graph, stream=torch.cuda.Stream())
    s.amr_link(links)
    return s


def _one_d(nc=40, lo=12, W=12, flux=1):
    h = 1.0 / nc
    g = np.array([1.5, 1.01]); pi = np.array([0.0, 0.02]); D = np.array([0.0, 3.0])
    def st(x0, n, dx):
        f = lambda x: 0.2 * (3.0 + np.sin(2 * np.pi * x))
        a1 = I.cell_average_1d(f, n, x0, x0 + n * dx)
        alpha = np.stack([a1, 1.0 - a1])
        m = np.array([2.0, 1.0])[:, None] * alpha
        u = (1.0 + 0.3 * I.cell_average_1d(lambda x: np.cos(2 * np.pi * x), n, x0, x0 + n * dx))[None]
        return I._to4d(I.conserved(alpha, m, u, np.ones(n), g, pi, D), 1)
    o = I.Options(flux=flux, cfl=0.4)
    pmin = I.default_pmin(pi, 1.0)
    wc = I.Workload("c1", 1, (nc,), (h,), ((0, 0),), g, pi, D, pmin, np.zeros(2), st(0.0, nc, h), opts=o)
    wf = I.Workload("f1", 1, (2 * W + 6,), (h / 2,), ((1, 1),), g, pi, D, pmin, np.zeros(2),
                    st((lo - 1.5) * h, 2 * W + 6, h / 2), opts=o)
    return wc, wf, amr.Block((lo,), W, 1), (lo,)


def _scales(U, nU):
    U = U.reshape(nU, -1)
    return np.maximum(np.abs(U).max(axis=1), 1e-300)


@pytest.mark.parametrize("case", ["2d_n2_hll", "2d_n3_hllc", "1d_n2_hll"])
def test_coupled_steps_vs_oracle(oracle, case):
    if case == "1d_n2_hll":
        wc, wf, b, lo = _one_d()
    else:
        N, flux = (2, 1) if case == "2d_n2_hll" else (3, 0)
        lo, W, H = (7, 6), 8, 10
        wc, wf = two_level(24, lo, W, H, N=N, opts=I.Options(flux=flux, cfl=0.4))
        b = amr.Block(lo, W, H)
    pbc, pbf = oracle_problem(oracle, wc), oracle_problem(oracle, wf)
    dt = 0.4 * wf.dx[0] / 3.0
    s = _solver([wc, wf], [(1, 0, lo)])
    for _ in range(3):
        s.step(dt=dt)
    Gc, Gf = s.host(0).reshape(-1), s.host(1).reshape(-1)
    s.close()
    Uc, Uf = wc.U.reshape(-1).copy(), wf.U.reshape(-1).copy()
    for _ in range(3):
        Uc, (Uf,) = amr.composite_step(pbc, [pbf], Uc, [Uf], [b], dt)
    for G, U, w in ((Gc, Uc, wc), (Gf, Uf, wf)):
        err = np.abs(G.reshape(w.nU, -1) - U.reshape(w.nU, -1)).max(axis=1) / _scales(U, w.nU)
        print(case, w.name, np.array2string(err, precision=2))
        assert (err <= 1e-12).all(), err


def test_coupled_cfl_steps_conserve(oracle):
    lo, W, H = (7, 6), 8, 10
    wc, wf = two_level(24, lo, W, H, N=3, opts=I.Options(flux=1, cfl=0.4))
    pbc, pbf = oracle_problem(oracle, wc), oracle_problem(oracle, wf)
    b = amr.Block(lo, W, H)
    t0 = amr.composite_totals(pbc, [pbf], wc.U.reshape(-1), [wf.U.reshape(-1)], [b])
    s = _solver([wc, wf], [(1, 0, lo)], use_graph=True)
    dts = s.dt()
    assert dts[0] == dts[1]
    s.advance(40)
    d = s.diag()
    assert d[0, 26] == d[1, 26] and d[0, 27] == d[1, 27] == 40
    Gc, Gf = s.host(0).reshape(-1), s.host(1).reshape(-1)
    s.close()
    t1 = amr.composite_totals(pbc, [pbf], Gc, [Gf], [b])
    cons = slice(0, wc.N + 3)
    err = np.abs(t1[cons] - t0[cons]) / np.abs(t0[cons]).max()
    assert err.max() <= 1e-13, err
    for G, w in ((Gc, wc), (Gf, wf)):
        a = G.reshape(w.nU, -1)[w.N + w.ndim + 1:]
        assert np.abs(a.sum(axis=0) - 1.0).max() <= 1e-13


def test_coupled_graph_replay_equals_eager():
    lo = (7, 6)
    outs = []
    for graph in (False, True):
        wc, wf = two_level(24, lo, 8, 10, N=2, opts=I.Options(flux=1, cfl=0.4))
        s = _solver([wc, wf], [(1, 0, lo)], use_graph=graph)
        if graph:
            s.advance(32)
        else:
            for _ in range(32):
                s.step()
        outs.append((s.host(0).copy(), s.host(1).copy()))
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_coupling_geometry_rejected():
    from paper_2608_00746_amd.binding import MpWenoError
    wc, wf = two_level(24, (7, 6), 8, 10, N=2)
    s = _solver([wc, wf], [])
    with pytest.raises(MpWenoError) as e:
        s.amr_link([(1, 0, (1, 6))])             # block 1 coarse cell from the boundary
    assert e.value.status == -1
    with pytest.raises(MpWenoError):
        s.amr_link([(0, 1, (7, 6))])             # roles swapped: sizes do not fit
    s.close()
