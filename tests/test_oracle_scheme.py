"""Whole-scheme pins of the oracle (Sec. 4.1): conservation, equilibrium,
volume-fraction sum, consistency of reduction, thermal equilibrium, design
order on smooth advection, bounds under the sufficient CFL, symmetry, and the
CFL time step.
"""
import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I
from conftest import oracle_problem

EPS = np.finfo(float).eps


def _run(pb, U, dt, steps):
    U = U.reshape(-1).copy()
    for _ in range(steps):
        U = pb.step(U, dt)
    return U


@pytest.mark.parametrize("N,flux,recon", [(2, 0, 0), (3, 1, 0), (3, 0, 1)])
def test_conservation_periodic(oracle, N, flux, recon):
    w = I.random_state((24, 32), nphase=N, seed=N + flux, lowp=0.0,
                       opts=I.Options(flux=flux, recon=recon, cfl=0.2))
    pb = oracle_problem(oracle, w)
    U0 = w.U.reshape(-1).copy()
    d0 = pb.diag(U0)
    dt = pb.dt(U0)
    U = _run(pb, U0, dt, 3)
    d1 = pb.diag(U)
    nU = w.nU
    # masses, momenta, energy (the alpha are not conserved quantities)
    for c in list(range(N)) + list(range(N, N + 3)):
        scale = np.abs(w.U[c]).sum() * np.prod(w.dx)
        assert abs(d1[c] - d0[c]) <= 1e-13 * scale, (c, d1[c], d0[c])
    assert d1[nU + 0] <= 16 * N * EPS              # sum alpha = 1


@pytest.mark.parametrize("flux", [0, 1])
def test_equilibrium_advection_1d(oracle, flux):
    """Uniform u and P across the translating air-water slab stay uniform
    (Sec. 2.2.2, equilibrium), within the pressure floor of Eq. (27)."""
    w = I.advection_1d(100, opts=I.Options(flux=flux, cfl=0.5))
    pb = oracle_problem(oracle, w)
    U = w.U.reshape(-1).copy()
    dt = pb.dt(U)
    steps = 200
    U = _run(pb, U, dt, steps)
    Uc = U.reshape(w.nU, -1)
    Ps, us = [], []
    for i in range(Uc.shape[1]):
        P, u = pb.pressure(Uc[:, i].copy())
        Ps.append(P)
        us.append(u[0])
    Ps, us = np.array(Ps), np.array(us)
    gP = 1e5 + (w.gamma * w.pinf).max()
    assert np.abs(Ps - 1e5).max() <= 64 * EPS * gP * np.sqrt(steps)
    c = 1449.1
    assert np.abs(us - 1.0).max() <= 64 * EPS * (1 + c) * np.sqrt(steps)
    # the slab moved: alpha_1 is no longer the initial profile
    assert np.abs(Uc[-2] - w.U.reshape(w.nU, -1)[-2]).max() > 1e-3


def test_reduction_n3_equals_n2_over_steps(oracle):
    """Sec. 3.4 / 4.1.2: an absent phase stays exactly zero and an N = 3 run
    with phase 3 absent reproduces the N = 2 run bitwise."""
    w3 = I.random_state((20, 24), nphase=3, seed=9, absent=(2,), lowp=0.0,
                        opts=I.Options(flux=1, cfl=0.2))
    pb3 = oracle_problem(oracle, w3)
    keep = [0, 1, 3, 4, 5, 6, 7]
    U3 = w3.U.reshape(w3.nU, -1)
    U2 = U3[keep].copy()
    pb2 = oracle.Problem(2, w3.n, w3.dx, w3.bc, list(w3.gamma[:2]), list(w3.pinf[:2]),
                         list(w3.D[:2]), list(w3.pmin[:2]), flux=1, cfl=0.2)
    dt = pb3.dt(U3.reshape(-1))
    assert dt == pb2.dt(U2.reshape(-1))
    a = _run(pb3, U3, dt, 3).reshape(w3.nU, -1)
    b = _run(pb2, U2, dt, 3).reshape(7, -1)
    assert (a[2] == 0).all() and (a[-1] == 0).all()
    assert np.array_equal(a[keep], b)


def test_reduction_n8_equals_n7_over_steps(oracle):
    """The widest phase count of the boundary: N = 8 with phase 8 absent
    reproduces the N = 7 run bitwise over steps, and the absent phase stays
    exactly zero (every per-phase loop of the scheme runs over eight
    phases)."""
    N = 8
    w8 = I.random_state((14, 18), nphase=N, seed=17, absent=(N - 1,), lowp=0.0,
                        opts=I.Options(flux=1, cfl=0.2))
    pb8 = oracle_problem(oracle, w8)
    keep = [c for c in range(w8.nU) if c not in (N - 1, w8.nU - 1)]
    U8 = w8.U.reshape(w8.nU, -1)
    U7 = U8[keep].copy()
    pb7 = oracle.Problem(2, w8.n, w8.dx, w8.bc, list(w8.gamma[:N - 1]), list(w8.pinf[:N - 1]),
                         list(w8.D[:N - 1]), list(w8.pmin[:N - 1]), flux=1, cfl=0.2)
    dt = pb8.dt(U8.reshape(-1))
    assert dt == pb7.dt(U7.reshape(-1))
    a = _run(pb8, U8, dt, 3).reshape(w8.nU, -1)
    b = _run(pb7, U7, dt, 3).reshape(w8.nU - 2, -1)
    assert (a[N - 1] == 0).all() and (a[-1] == 0).all()
    assert np.array_equal(a[keep], b)


def test_thermal_and_consistency_errors_roundoff(oracle):
    """Sec. 4.1.1 with WENO-C: temperature and the consistency error
    (alpha_1 rho_1)/rho_1 - alpha_1 stay at round-off."""
    w = I.paper_two_phase_advection(40)
    pb = oracle_problem(oracle, w)
    U = _run(pb, w.U, w.dt_fixed, 20).reshape(w.nU, -1)
    rho1 = 1.204e-3
    cons = np.abs(U[0] / rho1 - U[-2]).max()
    assert cons < 1e-13
    T = np.array([pb.temperature(U[:, i].copy()) for i in range(0, U.shape[1], 7)])
    assert np.abs(T - 300.0).max() / 300.0 < 1e-10


@pytest.mark.slow
def test_fifth_order_smooth_advection(oracle):
    """Sec. 4.1.4: L1 error of alpha_1 at t = 1 with dt = dx^(5/3) converges at
    fifth order."""
    errs, hs = [], []
    for n in (20, 40, 80):
        w = I.smooth_1d(n)
        pb = oracle_problem(oracle, w)
        steps = int(np.ceil(1.0 / w.dt_fixed))
        dt = 1.0 / steps
        U = _run(pb, w.U, dt, steps).reshape(w.nU, -1)
        ex = I.smooth_1d_exact_alpha(n, 1.0)
        errs.append(np.abs(U[-2] - ex).sum() / n)
        hs.append(1.0 / n)
    rates = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert rates[-1] > 4.5, (errs, rates)


@pytest.mark.parametrize("recon", [0, 1])
def test_bounds_under_sufficient_cfl(oracle, recon):
    """Sec. 4.2: with HLL and CFL <= 1/12 the update stays admissible."""
    w = I.random_state((200,), nphase=3, seed=12, lowp=0.05,
                       opts=I.Options(flux=1, cfl=1.0 / 12.0, recon=recon))
    pb = oracle_problem(oracle, w)
    U = w.U.reshape(-1).copy()
    for _ in range(5):
        U = pb.step(U, pb.dt(U))
        d = pb.diag(U)
        nU = w.nU
        scale = np.abs(U).max()
        assert d[nU + 1] >= -1e-12 * scale          # min m_p
        assert d[nU + 2] >= -1e-12 and d[nU + 3] <= 1 + 1e-12
        assert d[nU + 4] >= -1e-9 * np.abs(U.reshape(nU, -1)[3]).max()
        assert d[nU + 5] == 0


def test_xy_symmetry(oracle):
    """Transposing a 2D state transposes L(U) with the velocity components
    swapped (catches index errors in the second direction)."""
    w = I.random_state((16, 16), nphase=2, seed=2, lowp=0.0, opts=I.Options(flux=1))
    pb = oracle_problem(oracle, w)
    U = w.U[:, 0]
    L = pb.rhs(U.reshape(-1)).reshape(U.shape)
    Ut = np.transpose(U, (0, 2, 1)).copy()
    Ut[[2, 3]] = Ut[[3, 2]]
    Lt = pb.rhs(Ut.reshape(-1)).reshape(U.shape)
    Lt[[2, 3]] = Lt[[3, 2]]
    Lt = np.transpose(Lt, (0, 2, 1))
    for c in range(w.nU):
        sc = np.abs(L[c]).max() + 1e-300
        assert np.abs(L[c] - Lt[c]).max() <= 1e-12 * sc


def test_dt_cfl(oracle):
    """The CFL step against max_i sum_d (|u_d| + c)/dx_d computed here from
    primitives (pure phases: textbook stiffened-gas sound speed)."""
    w = I.shock_bubble_2d(64, 32)
    pb = oracle_problem(oracle, w)
    U = w.U[:, 0]
    N = 2
    rho = U[:N].sum(0)
    ux, uy = U[N] / rho, U[N + 1] / rho
    pure = (U[-2] == 0) | (U[-1] == 0) | (U[-2] < 1e-30) | (U[-1] < 1e-30)
    dt = pb.dt(U.reshape(-1))
    # only the pure-water post-shock cells and pure water at rest matter for
    # the maximum; compute c there from the stiffened-gas formula
    P = np.where(ux > 0, 1e9, 1e5)
    c = np.sqrt(6.12 * (P + 3.43e8) / rho)
    s = ((np.abs(ux) + c) / w.dx[0] + (np.abs(uy) + c) / w.dx[1])[pure & (U[-1] > 0.99)]
    assert abs(dt - 0.2 / s.max()) < 1e-9 * dt
    pb.__dict__  # noqa
    # clipping to t_end
    pb2 = oracle_problem(oracle, w, t_end=1e-9)
    assert pb2.dt(U.reshape(-1), 0.0) == 1e-9


def test_alpha_source_forms(oracle):
    """The alpha source of Eq. (3), alpha_p (1 + K_p) times the u-hat
    difference over dx, at the cell average alphabar_p (the default, the
    equation as written) or at alphabar_p / S, S = sum_q alphabar_q (the
    same for a consistent state).  Rough 1D states whose volume fractions
    sum to 1 + 1e-6, random (compressing and expanding) velocities:
    * only the alpha rates differ between the forms, and for the Allaire
      model (K_p = 0) by alphabar_p (1 - 1/S) times one per-cell factor, the
      u-hat difference over dx;
    * with alphabar_p / S the sources sum to the u-hat difference that the
      fluxes' alpha parts sum to (faces closed to sum 1), so sum_p L(alpha_p)
      stays at rounding in every cell, both models, while the cell form
      leaves (S - 1) times that difference.  (A cell limited by theta_i or
      theta^psi, or falling back to first order, has faces
      alphabar + theta (alpha^face - alphabar) whose alphas sum to
      S + theta (1 - S), so there the cancellation needs S = 1; such cells
      are absent from this state.)"""
    N = 3
    for model in (0, 1):
        w = I.random_state((64,), nphase=N, seed=7, lowp=0.0,
                           opts=I.Options(flux=1, model=model))
        U = w.U.reshape(w.nU, -1).copy()
        ia = slice(N + w.ndim + 1, N + w.ndim + 1 + N)
        U[ia] *= 1.0 + 1e-6
        S = U[ia].sum(axis=0)
        Ln = oracle_problem(oracle, w, alpha_source=oracle.SRC_NORMALIZED).rhs(
            U.reshape(-1)).reshape(w.nU, -1)
        Lc = oracle_problem(oracle, w, alpha_source=oracle.SRC_CELL).rhs(
            U.reshape(-1)).reshape(w.nU, -1)
        La = Ln[ia]
        assert np.abs(La.sum(axis=0)).max() <= 1e-14 * np.abs(La).max()
        assert np.abs(La).max() > 0.0
        assert np.array_equal(Ln[:ia.start], Lc[:ia.start])
        d = Lc[ia] - Ln[ia]
        assert np.abs(d).max() > 0.0
        if model == 0:
            # the u-hat difference over dx, from every phase present in a cell
            pres = U[ia] > 1e-3
            with np.errstate(divide="ignore", invalid="ignore"):
                f = np.where(pres, d / (U[ia] * (1.0 - 1.0 / S)), np.nan)
            fmax, fmin = np.nanmax(f, axis=0), np.nanmin(f, axis=0)
            big = np.abs(fmax) > 1e-3 * np.nanmax(np.abs(f))
            assert big.sum() > 10
            spread = (fmax - fmin)[big] / np.abs(fmax)[big]
            assert spread.max() <= 1e-6, spread.max()
            # the cell form's alpha rates sum to (S - 1) times it
            sc = Lc[ia].sum(axis=0)[big]
            assert np.allclose(sc, ((S - 1.0) * fmax)[big], rtol=1e-5,
                               atol=1e-12 * np.abs(Lc[ia]).max())
