"""The mixed-precision path (FP32 smoothness indicators, weights, u/P face
increments, sound speeds, wave speeds and HLL coefficients; FP64 everything
that decides consistency, bounds and equilibrium) against the FP64 oracle.

Stated accuracy (measured on the paper-shaped workloads; the FP32 weights
move a face value by ~1e-7 of its stencil's variation):
* L(U): max |L_mixed - L_orc| <= 1e-4 max |L_orc| per significant component;
* states after a window of steps: per-component L1 and max error relative
  to the component scale <= 1e-6.
Exact invariants (FP64 round-off, as on the FP64 path): uniform velocity and
pressure stay uniform across a translating interface, sum_p alpha_p = 1,
bounds, an absent phase stays exactly zero and N = 3 with an absent phase
reproduces N = 2 bitwise.
"""
import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I
from conftest import oracle_problem
from test_gpu_parity import _scales, _solver

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps
TOL_RHS = 1e-4
TOL_STATE = 1e-6


def _mixed(w):
    w.opts.precision = I.PREC_MIXED
    return w


@pytest.mark.parametrize("make", [
    lambda: I.shock_bubble_2d(256, 128), lambda: I.shock_interface_n3(128),
    lambda: I.advection_2d(64), lambda: I.batched_instance(160, 3, 0.15, 1.5e9),
    lambda: I.paper_five_phase(50), lambda: I.air_helium_shock_tube(0.01),
    # Kapila model: the sound speed (Wood) and 1 + K_p in the mixed sweeps
    lambda: I.random_state((40, 130), nphase=3, seed=21, lowp=0.0,
                           opts=I.Options(flux=1, model=I.MODEL_KAPILA))])
def test_rhs_mixed_vs_oracle(oracle, make):
    w = _mixed(make())
    s = _solver(w)
    Lg = s.rhs()[0].cpu().numpy().reshape(w.nU, -1)
    s.close()
    pb = oracle_problem(oracle, w)
    U = w.U.reshape(-1)
    Lo = pb.rhs(U).reshape(w.nU, -1)
    dt = pb.dt(U, 0.0)
    sc = _scales(w)
    Lmax = np.abs(Lo).max(axis=1)
    raw = np.abs(Lg - Lo).max(axis=1) / np.where(Lmax > 0, Lmax, 1.0)
    significant = dt * Lmax > 1e-10 * sc
    print(w.name, "mixed rhs rel err:", np.array2string(raw, precision=2))
    assert np.isfinite(Lg).all()
    assert (raw[significant] <= TOL_RHS).all(), raw


@pytest.mark.parametrize("make,K", [
    (lambda: I.shock_bubble_2d(256, 128), 10), (lambda: I.shock_interface_n3(128), 10),
    (lambda: I.advection_2d(64), 10), (lambda: I.air_helium_shock_tube(0.01), 40)])
def test_window_mixed_vs_oracle(oracle, make, K):
    w = _mixed(make())
    w.t_end = 0.0
    pb = oracle_problem(oracle, w, t_end=0.0)
    s = _solver(w)
    U = w.U.reshape(-1).copy()
    for _ in range(K):
        dt = pb.dt(U, 0.0)
        U = pb.step(U, dt)
        s.step(dt)
    Ug = s.host(0).reshape(w.nU, -1)
    Uo = U.reshape(w.nU, -1)
    sc = _scales(w, U)
    linf = np.abs(Ug - Uo).max(axis=1) / sc
    l1 = np.abs(Ug - Uo).mean(axis=1) / sc
    print(w.name, "mixed after", K, "steps: Linf", np.array2string(linf, precision=2),
          "L1", np.array2string(l1, precision=2))
    assert (linf <= TOL_STATE).all() and (l1 <= TOL_STATE).all()
    s.close()


@pytest.mark.parametrize("flux", [I.FLUX_HLLC, I.FLUX_HLL])
def test_mixed_equilibrium(flux):
    """Sec. 2.2.2: uniform u and P across the translating air-water slab stay
    uniform on the mixed path within the FP64 pressure floor (c_R = 1 - c_L
    is exact, u/P increments of uniform stencils are exactly zero)."""
    w = _mixed(I.advection_1d(200, opts=I.Options(flux=flux, cfl=0.5)))
    s = _solver(w)
    steps = 200
    for _ in range(steps):
        s.step()
    U = s.host(0).reshape(w.nU, -1)
    N = 2
    rho = U[:N].sum(0)
    u = U[N] / rho
    A = 1.0 / (w.gamma - 1.0)
    B = w.gamma * w.pinf / (w.gamma - 1.0)
    a = U[-N:]
    P = (U[N + 1] - 0.5 * U[N] ** 2 / rho - (B[:, None] * a).sum(0)) / (A[:, None] * a).sum(0)
    gP = 1e5 + (w.gamma * w.pinf).max()
    assert np.abs(P - 1e5).max() <= 64 * EPS * gP * np.sqrt(steps)
    assert np.abs(u - 1.0).max() <= 64 * EPS * 1500.0 * np.sqrt(steps)
    assert np.abs(a.sum(0) - 1).max() <= 16 * N * EPS * np.sqrt(steps)
    # averages: bounds to round-off (the CFL here is above the sufficient 1/12)
    tau = 1e-12
    assert (U[:N] >= -tau * U[:N].max()).all() and (a >= -tau).all() and (a <= 1 + tau).all()
    s.close()


def test_mixed_reduction_bitwise():
    w3 = _mixed(I.random_state((30, 270), nphase=3, seed=41, absent=(2,), lowp=0.0,
                               opts=I.Options(flux=1, cfl=0.2)))
    keep = [0, 1, 3, 4, 5, 6, 7]
    w2 = w3.copy()
    w2.gamma, w2.pinf, w2.D, w2.pmin, w2.cT = (x[:2] for x in
                                               (w3.gamma, w3.pinf, w3.D, w3.pmin, w3.cT))
    w2.U = w3.U[keep].copy()
    s3, s2 = _solver(w3), _solver(w2)
    for _ in range(3):
        s3.step()
        s2.step()
    a, b = s3.host(0), s2.host(0)
    assert (a[2] == 0).all() and (a[-1] == 0).all()
    assert np.array_equal(a[keep], b)
    s3.close(); s2.close()


def test_mixed_bounds_shock_interface():
    w = _mixed(I.shock_interface_n3(256))
    s = _solver(w)
    for _ in range(30):
        s.step()
    d = s.diag()[0]
    assert d[25] == 0
    assert d[21] >= 0 and d[22] >= 0 and d[23] <= 1 and d[20] <= 16 * 3 * EPS
    s.close()
