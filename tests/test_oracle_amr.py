"""Pins of the oracle's two-level coupling (oracle/amr.py; refinement by 2
of uniform levels, Sec. 3.4.2):
* the composite grid conserves m_p, rho u and rho E to rounding over steps
  of a flow with non-uniform velocity through the block edges;
* uniform velocity and pressure stay uniform on both levels (equilibrium),
  and sum_p alpha_p stays 1 in the refluxed coarse cells;
* inside the block, farther from its ring than one step's domain of
  dependence (3 cells per RK stage), the fine cells equal those of the same
  step on the uniformly refined grid: the coupling touches nothing it should
  not."""
import numpy as np
import pytest

from oracle import amr
from amr_states import two_level, state
from conftest import oracle_problem


def _setup(oracle, nc=24, lo=(7, 6), W=8, H=10, N=2, flow=True, flux=1):
    from paper_2608_00746_amd import inputs as I
    wc, wf = two_level(nc, lo, W, H, N, flow, opts=I.Options(flux=flux, cfl=0.4))
    return (oracle_problem(oracle, wc), oracle_problem(oracle, wf), wc.U.reshape(-1).copy(),
            wf.U.reshape(-1).copy(), amr.Block(lo, W, H))


@pytest.mark.parametrize("N,flux", [(2, 1), (3, 0)])
def test_composite_conservation(oracle, N, flux):
    pbc, pbf, Uc, Uf, b = _setup(oracle, N=N, flux=flux)
    dt = 0.4 * pbf.dx[0] / 3.0
    t0 = amr.composite_totals(pbc, [pbf], Uc, [Uf], [b])
    for _ in range(3):
        Uc, (Uf,) = amr.composite_step(pbc, [pbf], Uc, [Uf], [b], dt)
    t1 = amr.composite_totals(pbc, [pbf], Uc, [Uf], [b])
    cons = slice(0, N + 3)                         # m_p, rho u, rho v, rho E
    err = np.abs(t1[cons] - t0[cons]) / np.abs(t0[cons]).max()
    assert err.max() <= 1e-14, err
    # without the flux correction the same steps do not conserve
    pbc2, pbf2, Uc2, Uf2, b2 = _setup(oracle, N=N, flux=flux)
    saved = amr.stage_correction
    try:
        amr.stage_correction = lambda *a, **k: {}
        for _ in range(3):
            Uc2, (Uf2,) = amr.composite_step(pbc2, [pbf2], Uc2, [Uf2], [b2], dt)
    finally:
        amr.stage_correction = saved
    t2 = amr.composite_totals(pbc2, [pbf2], Uc2, [Uf2], [b2])
    assert (np.abs(t2[cons] - t0[cons]) / np.abs(t0[cons]).max()).max() > 1e-9


def test_composite_equilibrium_and_volume_sum(oracle):
    pbc, pbf, Uc, Uf, b = _setup(oracle, flow=False)
    dt = 0.4 * pbf.dx[0] / 3.0
    for _ in range(3):
        Uc, (Uf,) = amr.composite_step(pbc, [pbf], Uc, [Uf], [b], dt)
    for pb, U in ((pbc, Uc), (pbf, Uf)):
        V = U.reshape(pb.nU, -1)
        for i in range(V.shape[1]):
            P, u = pb.pressure(V[:, i])
            assert abs(P - 1.0) <= 1e-12 and abs(u[0] - 1.0) <= 1e-12 and abs(u[1] - 0.5) <= 1e-12
        a = V[pb.N + pb.ndim + 1:]
        assert np.abs(a.sum(axis=0) - 1.0).max() <= 1e-14


def test_block_interior_equals_uniform_refinement(oracle):
    nc, lo, W = 32, (6, 6), 20
    pbc, pbf, Uc, Uf, b = _setup(oracle, nc=nc, lo=lo, W=W, H=W)
    # the uniformly refined grid and its step (same RK expressions)
    from paper_2608_00746_amd import inputs as I
    U2, g, pi, D = state(((0, 1), (0, 1)), 2 * nc, 2 * nc)
    pbu = oracle.Problem(2, (2 * nc, 2 * nc), (0.5 / nc, 0.5 / nc), ((0, 0), (0, 0)),
                         list(g), list(pi), list(D), list(I.default_pmin(pi, 1.0)), flux=1)
    dt = 0.4 * pbf.dx[0] / 3.0
    Uu, _ = amr.composite_step(pbu, [], U2.reshape(-1), [], [], dt)
    Uc, (Uf,) = amr.composite_step(pbc, [pbf], Uc, [Uf], [b], dt)
    F = Uf.reshape(pbf.nU, 2 * W + 6, 2 * W + 6)
    G = Uu.reshape(pbu.nU, 2 * nc, 2 * nc)
    reach = 9                                       # 3 cells per stage, 3 stages
    h = amr.HALO
    sl = slice(h + reach, h + 2 * W - reach)
    fx0 = 2 * lo[0]
    blockF = F[:, sl, sl]
    blockU = G[:, 2 * lo[1] + reach:2 * lo[1] + 2 * W - reach, fx0 + reach:fx0 + 2 * W - reach]
    assert blockF.shape == blockU.shape and blockF.shape[1] >= 20
    rel = np.abs(blockF - blockU).max(axis=(1, 2)) / np.abs(blockU).max(axis=(1, 2))
    assert rel.max() <= 1e-14, rel
    # next to the ring the coarse data enter: the fine cells there differ,
    # by the size of the coarse-fine truncation difference
    # (piecewise-constant ghost cells: first order in the coarse spacing)
    edge = np.abs(F[:, h:h + 3, h:-h] - G[:, 2 * lo[1]:2 * lo[1] + 3, fx0:fx0 + 2 * W]).max(
        axis=(1, 2)) / np.abs(G).max(axis=(1, 2))
    assert 1e-8 < edge.max() < 5e-2, edge
