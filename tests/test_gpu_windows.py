"""The benchmark configurations as written, on the GPU (full sizes).

Always run:
* C4, 2D N = 3 shock-interface at 1024^2: phase 3 stays exactly 0 in the
  strip x >= 0.85 beyond its stencils' reach (3 cells per RK stage), and
  the problem with an absent third phase equals its N = 2 version bitwise
  (FP64 and mixed);
* C5, the 256-instance batch: 8 seeded instances after 20 steps of the
  batched FP64 run against the oracle run of each alone, at the window bar;
  and the benchmark's own configuration (mixed, autotuned, graphs): L(U)
  and 10 steps of sampled instances against the oracle at the mixed bars.
With MPWENO_LONG=1 (minutes; measured figures in the design notes):
* C1 for the full period (t = 1, 580 024 steps): invariants and the L1
  error of alpha_1 against the translated initial state, plus the first
  5 800 steps against the oracle;
* C2a, 1 000 steps at 512^2 against the oracle;
* C2b, the smooth 2D problem to t = 1 at 128^2 .. 1024^2: design order;
* C3, the first 100 FP64 steps at 2048 x 1024 against the oracle;
* C5 end to end: every instance to its own t_end = (1 - x_s)/S, finished
  instances retired (bitwise frozen while the others run).
"""
import os

import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I
from conftest import oracle_problem
from test_gpu_parity import _scales

pytestmark = pytest.mark.gpu
LONG = pytest.mark.skipif(os.environ.get("MPWENO_LONG") != "1",
                          reason="long run (minutes): set MPWENO_LONG=1")


def _solver(ws, graph=True):
    import torch
    from paper_2608_00746_amd.binding import Solver
    return Solver(ws, use_graph=graph, stream=torch.cuda.Stream())


def _window(oracle, w, steps, tol=None):
    """GPU and oracle from the same state, each with its own CFL steps.  The
    bar: 1e-12 of the component scale up to 20 steps, then growing as
    sqrt(steps / 20): two correct FP64 evaluation orders differ per step by
    rounding, and on the SI air-water states the pressure recovered from
    rho E amplifies that by (P + gamma Pinf) / P ~ 2e4 (its ulp floor), so
    the differences add up as a random walk over a long window."""
    if tol is None:
        tol = 1e-12 * max(1.0, np.sqrt(steps / 20.0))
    s = _solver([w])
    s.advance(steps)
    G = s.host(0).reshape(w.nU, -1)
    s.close()
    pb = oracle_problem(oracle, w)
    U = w.U.reshape(-1).copy()
    t = 0.0
    for _ in range(steps):
        dt = pb.dt(U, t)
        U = pb.step(U, dt)
        t += dt
    U = U.reshape(w.nU, -1)
    err = np.abs(G - U).max(axis=1) / _scales(w, U)
    print(w.name, steps, "steps: window err", np.array2string(err, precision=2))
    assert (err <= tol).all(), (err, tol)
    return err


@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED], ids=["fp64", "mixed"])
def test_c4_strip_stays_free_of_phase_3(prec):
    n, steps = 1024, 5
    w = I.shock_interface_n3(n, opts=I.Options(flux=I.FLUX_HLL, cfl=0.2, precision=prec))
    s = _solver([w])
    s.advance(steps)
    U = s.host(0).reshape(w.nU, n, n)
    s.close()
    reach = 3 * 3 * steps
    i0 = int(np.ceil(0.85 * n)) + reach
    assert i0 < n - 50
    N, d = w.N, w.ndim
    assert np.all(U[2, :, i0:] == 0.0) and np.all(U[N + d + 1 + 2, :, i0:] == 0.0)
    # and phase 3 did move into the first cells of the strip
    assert np.abs(U[N + d + 1 + 2, :, int(np.ceil(0.85 * n)):i0]).max() > 0.0


def _absent_third(n, N, prec):
    """Gas bubble in the (4.4, 6e8) liquid with a right-moving 1e9 Pa shock,
    as two phases or as three with the third (6.12, 3.43e8) absent."""
    g, pi, D = I._eos([I.AIR_SI, I.CAVITY_WATER_SI, I.WATER_SI][:N])
    rho = np.array([1.0, 1000.0])
    dx = 1.0 / n
    box = ((0, 1), (0, 1))
    a1 = np.clip(I.cell_average_2d(lambda X, Y: I._tanh_disc(X, Y, 0.5, 0.5, 0.12, dx),
                                   n, n, box), 0.0, 1.0)
    alpha = [a1, 1.0 - a1] + [np.zeros((n, n))] * (N - 2)
    r2, u2, S = I.rh_post_shock(g[1], pi[1], rho[1], 1e5, 1e9)
    xc = (np.arange(n) + 0.5) * dx
    post = np.broadcast_to(xc < 0.25, (n, n))
    m = [rho[0] * a1, np.where(post, r2, rho[1]) * alpha[1]] + [np.zeros((n, n))] * (N - 2)
    u = np.zeros((2, n, n))
    u[0] = np.where(post, u2, 0.0)
    P = np.where(post, 1e9, 1e5)
    U = I.conserved(np.stack(alpha), np.stack(m), u, P, g, pi, D)
    return I.Workload("absent_%d_N%d" % (n, N), 2, (n, n), (dx, dx), ((1, 1), (1, 1)), g, pi,
                      D, I.default_pmin(pi, 1e5), np.zeros(N), I._to4d(U, 2),
                      opts=I.Options(flux=I.FLUX_HLL, cfl=0.2, precision=prec))


@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED], ids=["fp64", "mixed"])
def test_c4_absent_third_phase_equals_two_phases_bitwise(prec):
    n, steps = 1024, 40
    out = {}
    for N in (2, 3):
        w = _absent_third(n, N, prec)
        s = _solver([w])
        s.advance(steps)
        out[N] = (s.host(0).reshape(w.nU, -1), s.diag()[0])
        s.close()
    U2, d2 = out[2]
    U3, d3 = out[3]
    # components: m1 m2 | (m3) | mom x2, E | a1 a2 | (a3)
    assert np.array_equal(U3[[0, 1, 3, 4, 5, 6, 7]], U2) and d2[26] == d3[26]
    assert np.all(U3[2] == 0.0) and np.all(U3[8] == 0.0)


def test_c5_sampled_instances_vs_oracle(oracle):
    steps = 20
    ws = I.batched(opts=I.Options(flux=I.FLUX_HLL, cfl=0.2, precision=I.PREC_FP64))
    s = _solver(ws)
    s.advance(steps)
    pick = np.random.default_rng(5).choice(len(ws), 8, replace=False)
    G = {int(k): s.host(int(k)).reshape(ws[k].nU, -1).copy() for k in pick}
    s.close()
    for k in pick:
        w = ws[int(k)]
        pb = oracle_problem(oracle, w)
        U = w.U.reshape(-1).copy()
        t = 0.0
        for _ in range(steps):
            dt = pb.dt(U, t)
            U = pb.step(U, dt)
            t += dt
        U = U.reshape(w.nU, -1)
        err = np.abs(G[int(k)] - U).max(axis=1) / _scales(w, U)
        print(w.name, np.array2string(err, precision=2))
        assert (err <= 1e-12).all(), (w.name, err)


def test_c5_headline_configuration_sampled_vs_oracle(oracle):
    """The benchmark's own launch configuration (the 256-instance batch,
    mixed precision, autotuned tile shapes, captured 16-step graphs):
    L(U) of 10 sampled instances (seeded, plus the smallest and the largest)
    against the oracle at the mixed bar (1e-4 of max |L| per significant
    component), then 10 steps of the whole batch against each sampled
    instance's oracle run alone at the mixed window bar (1e-6 of the
    component scale)."""
    from test_gpu_mixed import TOL_RHS, TOL_STATE
    ws = I.batched(opts=I.Options(flux=I.FLUX_HLL, cfl=0.2, precision=I.PREC_MIXED))
    s = _solver(ws)
    s.autotune()
    L = s.rhs()
    n = np.array([w.ncells for w in ws])
    pick = sorted(set(np.random.default_rng(7).choice(len(ws), 8, replace=False).tolist()
                      + [int(np.argmin(n)), int(np.argmax(n))]))
    Lg = {k: L[k].cpu().numpy().reshape(ws[k].nU, -1) for k in pick}
    del L
    steps = 10
    s.advance(steps)
    G = {k: s.host(k).reshape(ws[k].nU, -1).copy() for k in pick}
    d = s.diag()
    s.close()
    assert (d[:, 27] == steps).all() and (d[:, 25] == 0).all()
    for k in pick:
        w = ws[k]
        pb = oracle_problem(oracle, w)
        U = w.U.reshape(-1).copy()
        Lo = pb.rhs(U).reshape(w.nU, -1)
        dt = pb.dt(U, 0.0)
        sc = _scales(w)
        Lmax = np.abs(Lo).max(axis=1)
        raw = np.abs(Lg[k] - Lo).max(axis=1) / np.where(Lmax > 0, Lmax, 1.0)
        significant = dt * Lmax > 1e-10 * sc
        t = 0.0
        for _ in range(steps):
            dtk = pb.dt(U, t)
            U = pb.step(U, dtk)
            t += dtk
        U = U.reshape(w.nU, -1)
        err = np.abs(G[k] - U).max(axis=1) / _scales(w, U)
        print(w.name, "rhs", np.array2string(raw, precision=2), "| 10 steps",
              np.array2string(err, precision=2))
        assert (raw[significant] <= TOL_RHS).all(), (w.name, raw)
        assert (err <= TOL_STATE).all(), (w.name, err)


@LONG
def test_c1_full_period(oracle):
    w = I.advection_1d(200)
    _window(oracle, w, 5800)
    s = _solver([w])
    n_steps = 0
    while True:
        s.advance(1000)
        n_steps += 1000
        if s.diag()[0, 26] >= 1.0 - 1e-15:
            break
    d = s.diag()[0]
    G = s.host(0).reshape(w.nU, -1)
    s.close()
    U0 = w.U.reshape(w.nU, -1)
    assert abs(d[26] - 1.0) <= 1e-12
    a = G[w.N + 2]
    l1 = np.abs(a - U0[w.N + 2]).sum() * w.dx[0]
    tot0 = U0.sum(axis=1) * w.dx[0]
    tot1 = G.sum(axis=1) * w.dx[0]
    print("C1: steps", int(d[27]), "L1(alpha_1) vs translated IC", l1,
          "conservation", np.abs(tot1 - tot0) / np.abs(tot0).max(), "sum alpha", d[20])
    # after 580 024 steps: sum alpha - 1 and the totals carry the random walk
    # of per-step rounding (measured 1.7e-11 and <= 2.5e-11)
    assert l1 < 0.02
    assert d[20] <= 1e-10
    assert (np.abs(tot1[:w.N + 2] - tot0[:w.N + 2]) / np.abs(tot0[:w.N + 2]) <= 1e-10).all()


@LONG
def test_c2a_1000_steps(oracle):
    """Momentum is the velocity of an advected air-water interface: its
    rounding floor is the equilibrium bound 64 eps (|u| + c) sqrt(steps)
    relative to |u| (c = 1449 m/s in the water); measured 2.8e-11."""
    w = I.advection_2d(512)
    steps = 1000
    tol = np.full(w.nU, 1e-12 * np.sqrt(steps / 20.0))
    tol[w.N:w.N + w.ndim] = 64 * np.finfo(float).eps * (1.0 + 1449.06) * np.sqrt(steps)
    _window(oracle, w, steps, tol=tol)


@LONG
def test_c2b_convergence_to_1024():
    errs = []
    sizes = (128, 256, 512, 1024)
    for n in sizes:
        w = I.smooth_2d(n)
        s = _solver([w])
        dt = np.full(1, w.dt_fixed)
        steps = int(np.ceil(1.0 / w.dt_fixed - 1e-9))
        # the last step lands on t = 1
        for _ in range(steps - 1):
            s.step(dt=dt)
        s.step(dt=np.full(1, 1.0 - (steps - 1) * w.dt_fixed))
        G = s.host(0).reshape(w.nU, -1)
        s.close()
        a = G[w.N + 2]
        a0 = w.U.reshape(w.nU, -1)[w.N + 2]
        errs.append(np.abs(a - a0).sum() / a.size)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("C2b L1(alpha_1):", errs, "rates", rates)
    assert rates[0] > 4.7 and rates[1] > 4.0


@LONG
def test_c3_100_steps_vs_oracle(oracle):
    """The first 100 steps (measured 1.7e-13).  At step 102 the two part by
    2.2e-9 in cell (411, 315), where the air phase holds a denormal mass
    (8.7e-317): the sign of the smallest reconstructed value there, which
    sets theta_p of Eq. (18) and through Eq. (20) the whole cell, is decided
    by the rounding of the interior value; one oracle step from the GPU's
    own state reproduces the GPU's difference."""
    _window(oracle, I.shock_bubble_2d(2048, 1024), 100)


@LONG
def test_c5_end_to_end_with_retirement():
    ws = I.batched(opts=I.Options(flux=I.FLUX_HLL, cfl=0.2, precision=I.PREC_MIXED))
    t_end = np.array([w.t_end for w in ws])
    s = _solver(ws)
    frozen = {}
    steps = 0
    while True:
        s.advance(200)
        steps += 200
        d = s.diag()
        assert (d[:, 25] == 0).all()
        done = np.nonzero(d[:, 26] >= t_end * (1 - 1e-14))[0]
        for k in done:
            k = int(k)
            if k not in frozen:
                frozen[k] = (d[k, 27], s.host(k).copy())
        if len(done) == len(ws):
            break
        assert steps < 100000
    d = s.diag()
    # retired instances kept their state and step count while others ran
    for k, (st, U) in frozen.items():
        assert d[k, 27] == st and np.array_equal(s.host(k), U)
    assert np.allclose(d[:, 26], t_end, rtol=1e-13, atol=0)
    print("C5 end to end: steps", steps, "per-instance steps", d[:, 27].min(), "..",
          d[:, 27].max(), "min alpha", d[:, 22].min(), "max |sum alpha - 1|", d[:, 20].max())
    s.close()
