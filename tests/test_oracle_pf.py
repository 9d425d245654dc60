"""Pins of the oracle's Phase-Field step (Sec. 2.2.1, Eqs. (4)-(5);
Sec. 4, Eq. (28)) against what the model and the mathematics fix:

* g'(phi) against a numerical derivative of g and its three zeros;
* [div J_p]: sum over phases vanishes pointwise, the integral of each phase
  vanishes (the multipliers B), N = 2 antisymmetry, zero for a uniform
  mixture of any composition and for a fluid at rest (M = 0), and a small
  residual on the equilibrium kink phi = 1/(1 + exp(-sqrt(2) x/eta)) that
  falls at second order as eta/dx grows;
* Eq. (4): the 1D face fluxes k dQ/dx equal the exact prefix sums of
  [div J] dx; a 2D problem that varies in x only reproduces the 1D
  gradients; the constant-coefficient operator is the five-point Laplacian;
* the PF flux: zero without gradient, no transfer out of an empty donor or
  into a full receiver, sum_p F^alpha_p = 0, m_p = rho_p alpha_p carried
  consistently, uniform u and P carried exactly, the cap at k_f |G|;
* the PF step: periodic totals conserved, sum alpha = 1, bounds, uniform u
  and P preserved, an absent phase stays zero and N = 3 with an absent
  phase reproduces N = 2 bitwise.
"""
import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I
from conftest import oracle_problem

EPS = np.finfo(float).eps


def _pb(oracle, w, **kw):
    return oracle_problem(oracle, w, **kw)


def test_gprime_pins(oracle):
    g = lambda x: x * x * (1 - x) ** 2
    for x in (0.0, 0.5, 1.0):
        assert oracle.pf_gprime(x) == 0.0
    rng = np.random.default_rng(0)
    for x in rng.uniform(-0.2, 1.2, 50):
        h = 1e-5
        fd = (g(x + h) - g(x - h)) / (2 * h)
        assert abs(oracle.pf_gprime(x) - fd) <= 1e-9


@pytest.mark.parametrize("shape,N,bc", [((96,), 2, 0), ((96,), 3, 1), ((40, 32), 2, 1),
                                        ((36, 30), 3, 0)])
def test_divj_sums(oracle, shape, N, bc):
    w = I.pf_bubble(shape, N, width=1.5, bc=bc)
    pb = _pb(oracle, w)
    eta = w.dx[0]
    r, info = pb.pf_divj(w.U.reshape(-1), eta)
    M = info["M"]
    assert M == pytest.approx(0.5 * eta * np.linalg.norm([1.0, 0.5][:w.ndim]), rel=1e-14)
    scale = np.abs(r).max()
    assert scale > 0
    # sum over phases vanishes pointwise (sum_p W_pq = 0, sum_p R_p = 0, sum_p lap phi_p = 0)
    assert np.abs(r.sum(axis=0)).max() <= 64 * EPS * scale
    # each phase's integral vanishes (the multipliers enforce it)
    vol = np.prod(w.dx)
    assert (np.abs(r.sum(axis=1)) * vol <= 1e-13 * scale * vol * w.ncells).all()
    if N == 2:
        assert np.abs(r[0] + r[1]).max() <= 64 * EPS * scale


def test_divj_uniform_and_rest(oracle):
    # a uniform mixture of any composition: the multipliers cancel the
    # double-well term exactly in exact arithmetic
    n = 24
    g, pi, D = I._eos([I.AIR_SI, I.WATER_SI, I.CAVITY_WATER_SI])
    for comp in ([0.3, 0.7, 0.0], [0.2, 0.5, 0.3], [0.5, 0.5, 0.0]):
        a = np.array(comp)[:, None] * np.ones((3, n))
        m = np.array([1.0, 1000.0, 1030.0])[:, None] * a
        U = I.conserved(a, m, np.ones((1, n)), 1e5, g, pi, D)
        w = I.Workload("u", 1, (n,), (1.0 / n,), ((0, 0),), g, pi, D,
                       I.default_pmin(pi, 1e5), np.zeros(3), I._to4d(U, 1))
        r, info = _pb(oracle, w).pf_divj(w.U.reshape(-1), 1.0 / n)
        assert info["M"] > 0
        assert np.abs(r).max() <= 1e-12 * info["M"] * n * n
    # at rest: M = 0 and nothing moves
    w = I.pf_bubble((48,), 2, u=(0.0, 0.0))
    r, info = _pb(oracle, w).pf_divj(w.U.reshape(-1), w.dx[0])
    assert info["M"] == 0.0 and np.abs(r).max() == 0.0


def _kink(n, eta_cells):
    """Equilibrium profile of Eq. (28) in 1D, eta^2 phi'' = g'(phi):
    phi = 1 / (1 + exp(-sqrt(2) x / eta)), point values at the centres."""
    g, pi, D = I._eos([I.AIR_SI, I.WATER_SI])
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx - 0.5
    eta = eta_cells * dx
    a1 = 1.0 / (1.0 + np.exp(-np.sqrt(2.0) * x / eta))
    a = np.stack([a1, 1.0 - a1])
    m = np.array([1.0, 1000.0])[:, None] * a
    U = I.conserved(a, m, np.ones((1, n)), 1e5, g, pi, D)
    w = I.Workload("kink", 1, (n,), (dx,), ((1, 1),), g, pi, D, I.default_pmin(pi, 1e5),
                   np.zeros(2), I._to4d(U, 1))
    return w, eta


def test_divj_equilibrium_kink(oracle):
    errs = []
    for ec in (2.0, 4.0, 8.0):
        w, eta = _kink(400, ec)
        r, info = _pb(oracle, w).pf_divj(w.U.reshape(-1), eta)
        # scale of the individual terms: M |phi''| ~ M / eta^2
        errs.append(np.abs(r).max() * eta * eta / info["M"])
    # second-order truncation error of the Laplacian, nothing else
    assert errs[0] < 0.05
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0, errs


def test_q_equation_prefix_sum_1d(oracle):
    """1D, outflow: k_{i+1/2} (Q_{i+1} - Q_i)/dx = dx sum_{j<=i} [div J]_j
    (the discrete Eq. (4) summed from the left end, where the flux is 0)."""
    for N, width in ((2, 1.0), (3, 2.0)):
        w = I.pf_bubble((128,), N, width=width, bc=I.BC_OUTFLOW)
        pb = _pb(oracle, w)
        U = w.U.reshape(-1)
        r, _ = pb.pf_divj(U, w.dx[0])
        G, res = pb.pf_gradients(U, r)
        assert (res <= 1e-12).all()
        K = pb.pf_k(U)
        for p in range(N):
            k = K[p]
            kf = 0.5 * (k[:-1] + k[1:])
            J = w.dx[0] * np.cumsum(r[p])[:-1]
            Jd = kf * G[0, p, :-1]
            assert np.abs(J - Jd).max() <= 1e-12 * np.abs(J).max()
            assert G[0, p, -1] == 0.0          # outflow end: no face


def test_q_equation_2d_reduces_to_1d(oracle):
    n = 64
    w1 = I.pf_bubble((n,), 2, width=1.5, bc=I.BC_OUTFLOW)
    pb1 = _pb(oracle, w1)
    U1 = w1.U.reshape(w1.nU, -1)
    r1, _ = pb1.pf_divj(U1.reshape(-1), w1.dx[0])
    G1, _ = pb1.pf_gradients(U1.reshape(-1), r1)
    # the same slab, uniform in y (periodic), velocity along x only
    ny = 6
    N = 2
    U2 = np.zeros((2 * N + 3, ny, n))
    for c in range(N):
        U2[c] = U1[c]
    U2[N] = U1[N]
    U2[N + 2] = U1[N + 1]
    for p in range(N):
        U2[N + 3 + p] = U1[N + 2 + p]
    w2 = I.Workload("slab2d", 2, (n, ny), (1.0 / n, 1.0 / n), ((1, 1), (0, 0)),
                    w1.gamma, w1.pinf, w1.D, w1.pmin, w1.cT, U2[:, None])
    pb2 = _pb(oracle, w2)
    r2, info2 = pb2.pf_divj(U2.reshape(-1), 1.0 / n)
    # M is the same (|u| identical), the y Laplacian vanishes
    assert np.abs(r2.reshape(N, ny, n) - r1[:, None, :]).max() <= 1e-12 * np.abs(r1).max()
    G2, res = pb2.pf_gradients(U2.reshape(-1), r2)
    G2 = G2.reshape(2, N, ny, n)
    K = pb1.pf_k(U1.reshape(-1))
    for p in range(N):
        k = K[p]
        kf = np.append(0.5 * (k[:-1] + k[1:]), 0.0)
        J1 = kf * G1[0, p]
        J2 = kf[None, :] * G2[0, p]
        assert np.abs(J2 - J1[None, :]).max() <= 1e-11 * np.abs(J1).max()
        assert np.abs(G2[1, p] * kf[None, :]).max() <= 1e-11 * np.abs(J1).max()


def test_q_operator_constant_k(oracle):
    """phi = 1/2 everywhere (k = 1/4): the operator is k times the standard
    five-point Laplacian; on Q = x^2 + 3 y^2 its interior rows give
    k (2 + 6)."""
    nx, ny = 12, 10
    w = I.pf_bubble((nx, ny), 2, bc=I.BC_OUTFLOW)
    pb = _pb(oracle, w)
    A = pb.q_operator(np.full(nx * ny, 0.5))
    dx = w.dx[0]
    X, Y = np.meshgrid((np.arange(nx) + 0.5) * dx, (np.arange(ny) + 0.5) * dx)
    Q = (X ** 2 + 3 * Y ** 2).reshape(-1)
    AQ = (A @ Q).reshape(ny, nx)
    assert np.allclose(AQ[1:-1, 1:-1], 0.25 * 8.0, rtol=1e-9, atol=0)
    # symmetric, rows sum to zero
    assert abs(A - A.T).max() == 0.0
    assert np.abs(np.asarray(A.sum(axis=1))).max() <= 1e-12 * abs(A).max()


def _prim(pb, N, d, m, u, P, a):
    return np.concatenate([m, u, [P], a])


def test_pf_flux_pins(oracle):
    w = I.pf_bubble((8,), 3)
    pb = _pb(oracle, w)
    N, d = 3, 1
    rho = np.array([1.0, 1000.0, 1030.0])
    rng = np.random.default_rng(5)
    g, pi = w.gamma, w.pinf
    A = 1 / (g - 1)
    B = g * pi / (g - 1)
    for _ in range(200):
        aL = rng.dirichlet(np.ones(N))
        aR = rng.dirichlet(np.ones(N))
        u = rng.uniform(-3, 3)
        P = rng.uniform(1e4, 1e6)
        VL = _prim(pb, N, d, rho * aL, [u], P, aL)
        VR = _prim(pb, N, d, rho * aR, [u], P, aR)
        G = rng.normal(size=N)
        F = pb.pf_flux(VL, VR, G)
        Fa, Fm = F[N + 2:], F[:N]
        sc = np.abs(G).max()
        assert abs(Fa.sum()) <= 16 * EPS * sc
        assert np.allclose(Fm, rho * Fa, rtol=0, atol=64 * EPS * sc * rho.max())
        assert F[N] == pytest.approx(u * Fm.sum(), abs=64 * EPS * sc * 1e3 * 3)
        E = Fm.sum() * 0.5 * u * u + (Fa * (A * P + B)).sum()
        assert F[N + 1] == pytest.approx(E, abs=1e-12 * sc * (A * P + B).max())
        assert (pb.pf_flux(VL, VR, np.zeros(N)) == 0).all()
        # the cap: no volume flux beyond k_f |G| of Eq. (4)
        kf = rng.uniform(0, 0.05, N)
        Fc = pb.pf_flux(VL, VR, G, kf)
        S = (np.abs(G) * kf).sum()
        for p in range(N):
            assert abs(Fc[N + 2 + p]) <= abs(G[p]) * kf[p] + S * 1.01 + 1e-300
    # an empty donor gives nothing, a full receiver takes nothing
    aL = np.array([1.0, 0.0, 0.0])
    aR = np.array([0.0, 1.0, 0.0])
    VL = _prim(pb, N, d, rho * aL, [0.0], 1e5, aL)
    VR = _prim(pb, N, d, rho * aR, [0.0], 1e5, aR)
    F = pb.pf_flux(VL, VR, np.array([1.0, -1.0, 1.0]))
    assert (F == 0).all()


def test_pf_step_invariants(oracle):
    w = I.pf_bubble((40, 32), 3, width=1.5, bc=I.BC_PERIODIC)
    pb = _pb(oracle, w)
    U = w.U.reshape(-1)
    dt = pb.dt(U)
    U2, info = pb.pf_step(U, dt, w.dx[0])
    assert (info["residual"] <= 1e-12).all()
    d0, d1 = pb.diag(U), pb.diag(U2)
    nU, N = w.nU, 3
    for c in range(nU):
        sc = np.abs(w.U.reshape(nU, -1)[c]).max() * np.prod(w.dx) * w.ncells
        assert abs(d1[c] - d0[c]) <= 1e-13 * sc, c
    assert d1[nU] <= 16 * N * EPS                     # sum alpha = 1
    assert d1[nU + 1] >= 0 and d1[nU + 2] >= 0 and d1[nU + 3] <= 1 + 1e-14
    V = U2.reshape(nU, -1)
    rho = V[:N].sum(0)
    # uniform u = (1, 0.5) and P = 1e5 carried exactly up to round-off
    assert np.abs(V[N] / rho - 1.0).max() <= 1e-12
    assert np.abs(V[N + 1] / rho - 0.5).max() <= 1e-12
    for i in range(0, w.ncells, 37):
        P, _ = pb.pressure(V[:, i])
        assert abs(P - 1e5) <= 64 * EPS * (1e5 + 6.12 * 3.43e8)
    # the step changed something
    assert np.abs(U2 - U).max() > 0


def test_pf_absent_phase_and_reduction(oracle):
    w3 = I.pf_bubble((48, 40), 3, width=1.5)
    U3 = w3.U.reshape(w3.nU, -1).copy()
    N = 3
    # remove phase 3: its volume goes to phase 2, mass and energy rebuilt
    a = U3[-N:].copy()
    a[1] += a[2]
    a[2] = 0.0
    m = np.array([1.0, 1000.0, 1030.0])[:, None] * a
    u = np.stack([U3[N] / U3[:N].sum(0), U3[N + 1] / U3[:N].sum(0)])
    # same EOS for the absent slot as the reduced problem does not see it
    Ua = I.conserved(a, m, u, 1e5, w3.gamma, w3.pinf, w3.D)
    w3.U = Ua.reshape(w3.U.shape)
    keep = [0, 1, 3, 4, 5, 6, 7]
    w2 = w3.copy()
    w2.gamma, w2.pinf, w2.D, w2.pmin, w2.cT = (x[:2] for x in
                                               (w3.gamma, w3.pinf, w3.D, w3.pmin, w3.cT))
    w2.U = w3.U[[0, 1, 3, 4, 5, 6, 7]].copy()
    pb3, pb2 = _pb(oracle, w3), _pb(oracle, w2)
    U = w3.U.reshape(-1)
    dt = pb3.dt(U)
    A, _ = pb3.pf_step(U, dt, w3.dx[0])
    B, _ = pb2.pf_step(w2.U.reshape(-1), dt, w2.dx[0])
    A = A.reshape(9, -1)
    assert (A[2] == 0).all() and (A[-1] == 0).all()
    assert np.array_equal(A[keep], B.reshape(7, -1))
