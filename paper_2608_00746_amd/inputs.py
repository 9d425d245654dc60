"""Seeded synthetic workloads shaped like the paper's problems.

This module builds initial states only: cell-averaged volume fractions,
phase masses, momenta and total energies on uniform grids, plus the per-phase
equation-of-state parameters and scheme switches.  It contains none of the
scheme's arithmetic (no reconstruction, limiter, flux or time update); the
only thermodynamics in it is the stiffened-gas energy closure needed to write
a state in conserved variables (Sec. 2.1 mixture rules with Eq. (26)) and the
Rankine-Hugoniot relations used to seed the shock states of Sec. 4.2.

Both the GPU tests and the oracle tests take their inputs from here; it
imports neither the HIP binding nor the oracle.

Layout of U: float64 array (n_U, nz, ny, nx) with the component order
m_1..m_N, (rho u)_1..(rho u)_d, rho E, alpha_1..alpha_N  (Eq. (1)).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

BC_PERIODIC, BC_OUTFLOW, BC_SYMMETRY = 0, 1, 2
RECON_WENO_C, RECON_WENO_CL, RECON_WENO_JS, RECON_WENO_W = 0, 1, 2, 3
SRC_CELL, SRC_NORMALIZED = 0, 1
FLUX_HLLC, FLUX_HLL = 0, 1
MODEL_ALLAIRE, MODEL_KAPILA = 0, 1
PREC_FP64, PREC_MIXED = 0, 1


@dataclass
class Options:
    recon: int = RECON_WENO_C
    flux: int = FLUX_HLLC
    model: int = MODEL_ALLAIRE
    precision: int = PREC_FP64
    energy_limiter: int = 1
    phase_field: int = 0
    cfl: float = 0.5
    eta_over_dx: float = 1.0
    cg_rtol: float = 1e-12
    cg_maxit: int = 10000
    alpha_source: int = SRC_CELL


@dataclass
class Workload:
    """One uniform-grid instance: grid, EOS, conserved state, switches."""
    name: str
    ndim: int
    n: tuple            # cells per direction (nx[, ny[, nz]])
    dx: tuple
    bc: tuple           # ((lo, hi), ...) per direction
    gamma: np.ndarray
    pinf: np.ndarray
    D: np.ndarray
    pmin: np.ndarray
    cT: np.ndarray
    U: np.ndarray       # (n_U, nz, ny, nx) float64
    t_end: float = 0.0
    opts: Options = field(default_factory=Options)
    dt_fixed: float = 0.0   # a prescribed time step (0: use the CFL)

    @property
    def N(self):
        return len(self.gamma)

    @property
    def nU(self):
        return 2 * self.N + self.ndim + 1

    @property
    def ncells(self):
        return int(np.prod(self.n))

    def copy(self):
        w = dataclasses.replace(self)
        w.U = self.U.copy()
        w.opts = dataclasses.replace(self.opts)
        return w


# ---------------------------------------------------------------------------
# thermodynamic helpers used to *build* states
# ---------------------------------------------------------------------------

def default_pmin(pinf, p_ref):
    """P_min,p is user prescribed (Eq. (9)); reading: just above -Pinf_p."""
    pinf = np.asarray(pinf, dtype=np.float64)
    return -pinf + 1e-6 * (p_ref + pinf)


def conserved(alpha, m, u, P, gamma, pinf, D):
    """Conserved state from cell-averaged alpha_p, m_p, velocity and pressure.

    alpha, m: (N, *shape); u: (d, *shape); P: shape or scalar.
    rho E = rho |u|^2/2 + sum_p alpha_p (P + gamma_p Pinf_p)/(gamma_p - 1)
            + sum_p m_p D_p   (Sec. 2.1 mixture rule with Eq. (26))."""
    alpha = np.asarray(alpha, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    N = alpha.shape[0]
    d = u.shape[0]
    shape = alpha.shape[1:]
    P = np.broadcast_to(np.asarray(P, dtype=np.float64), shape)
    rho = m.sum(axis=0)
    U = np.empty((2 * N + d + 1,) + shape)
    U[:N] = m
    for k in range(d):
        U[N + k] = rho * u[k]
    rhoe = np.zeros(shape)
    for p in range(N):
        g, pi = gamma[p], pinf[p]
        rhoe += alpha[p] * (P + g * pi) / (g - 1.0) + m[p] * D[p]
    U[N + d] = 0.5 * rho * (u ** 2).sum(axis=0) + rhoe
    U[N + d + 1:] = alpha
    return U


def rh_post_shock(gamma, pinf, rho0, p0, p1, u0=0.0, direction=+1):
    """Post-shock state of a stiffened gas at rest ahead of a shock.

    Stiffened-gas Hugoniot (ideal-gas form with P -> P + Pinf).  direction=+1:
    shock moving to +x (post-shock fluid on its left).  Returns
    (rho1, u1, shock_speed)."""
    g = gamma
    a, b = p1 + pinf, p0 + pinf
    rho1 = rho0 * ((g + 1.0) * a + (g - 1.0) * b) / ((g - 1.0) * a + (g + 1.0) * b)
    du = np.sqrt((p1 - p0) * (1.0 / rho0 - 1.0 / rho1))
    S = rho1 * du / (rho1 - rho0)
    return rho1, u0 + direction * du, u0 + direction * S


# ---------------------------------------------------------------------------
# cell averages
# ---------------------------------------------------------------------------

def _gauss(ng):
    x, w = np.polynomial.legendre.leggauss(ng)
    return 0.5 * x, 0.5 * w            # nodes in [-1/2, 1/2], weights sum 1


def cell_average_1d(f, n, x0, x1, ng=8):
    dx = (x1 - x0) / n
    xc = x0 + (np.arange(n) + 0.5) * dx
    g, w = _gauss(ng)
    return sum(wk * f(xc + gk * dx) for gk, wk in zip(g, w))


def cell_average_2d(f, nx, ny, box, ng=4):
    (x0, x1), (y0, y1) = box
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(xc, yc)           # (ny, nx)
    g, w = _gauss(ng)
    out = np.zeros((ny, nx))
    for gi, wi in zip(g, w):
        for gj, wj in zip(g, w):
            out += wi * wj * f(X + gi * dx, Y + gj * dy)
    return out


def cell_average_3d(f, nx, ny, nz, box, ng=3):
    (x0, x1), (y0, y1), (z0, z1) = box
    dx, dy, dz = (x1 - x0) / nx, (y1 - y0) / ny, (z1 - z0) / nz
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    zc = z0 + (np.arange(nz) + 0.5) * dz
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")     # (nz, ny, nx)
    g, w = _gauss(ng)
    out = np.zeros((nz, ny, nx))
    for gi, wi in zip(g, w):
        for gj, wj in zip(g, w):
            for gk, wk in zip(g, w):
                out += wi * wj * wk * f(X + gi * dx, Y + gj * dy, Z + gk * dz)
    return out


def _to4d(U, ndim):
    """(nU, *shape) -> (nU, nz, ny, nx)."""
    if ndim == 1:
        return U[:, None, None, :]
    if ndim == 2:
        return U[:, None, :, :]
    return U


# ---------------------------------------------------------------------------
# materials
# ---------------------------------------------------------------------------
AIR_SI = (1.4, 0.0, 0.0)                  # gamma, Pinf, D
WATER_SI = (6.12, 3.43e8, 0.0)            # Sec. 4.2.2
CAVITY_WATER_SI = (4.4, 6.0e8, 0.0)       # Sec. 4.2.1 water, Pinf x 1e5


def _eos(mats):
    g = np.array([m[0] for m in mats], dtype=np.float64)
    pi = np.array([m[1] for m in mats], dtype=np.float64)
    D = np.array([m[2] for m in mats], dtype=np.float64)
    return g, pi, D


def _tanh_slab(x, lo, hi, w):
    return 0.5 * (np.tanh((x - lo) / w) - np.tanh((x - hi) / w))


def _tanh_disc(X, Y, xc, yc, r, w):
    return 0.5 * (1.0 - np.tanh((np.hypot(X - xc, Y - yc) - r) / w))


def _tanh_ball(X, Y, Z, c, r, w):
    d = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    return 0.5 * (1.0 - np.tanh((d - r) / w))


# ---------------------------------------------------------------------------
# the benchmark configurations
# ---------------------------------------------------------------------------

def advection_1d(n=200, opts=None):
    """1D two-phase advection: periodic [0,1], air slab in water (SI),
    u = 1, P = 1e5, alpha_1 a tanh slab on [0.4, 0.6] of width one cell."""
    g, pi, D = _eos([AIR_SI, WATER_SI])
    rho = np.array([1.0, 1000.0])
    dx = 1.0 / n
    a1 = cell_average_1d(lambda x: _tanh_slab(x, 0.4, 0.6, dx), n, 0.0, 1.0)
    a1 = np.clip(a1, 0.0, 1.0)
    alpha = np.stack([a1, 1.0 - a1])
    m = rho[:, None] * alpha
    U = conserved(alpha, m, np.ones((1, n)), 1e5, g, pi, D)
    return Workload("advection_1d_%d" % n, 1, (n,), (dx,),
                    ((BC_PERIODIC, BC_PERIODIC),), g, pi, D,
                    default_pmin(pi, 1e5), np.zeros(2), _to4d(U, 1), t_end=1.0,
                    opts=opts or Options(cfl=0.5))


def advection_2d(n=512, opts=None):
    """2D two-phase advection: periodic [0,1]^2, air bubble r = 0.15 at the
    centre in water (SI), u = v = 1, P = 1e5, tanh width one cell."""
    g, pi, D = _eos([AIR_SI, WATER_SI])
    rho = np.array([1.0, 1000.0])
    dx = 1.0 / n
    a1 = cell_average_2d(lambda X, Y: _tanh_disc(X, Y, 0.5, 0.5, 0.15, dx), n, n,
                         ((0, 1), (0, 1)))
    a1 = np.clip(a1, 0.0, 1.0)
    alpha = np.stack([a1, 1.0 - a1])
    m = rho[:, None, None] * alpha
    U = conserved(alpha, m, np.ones((2, n, n)), 1e5, g, pi, D)
    return Workload("advection_2d_%d" % n, 2, (n, n), (dx, dx),
                    ((BC_PERIODIC,) * 2,) * 2, g, pi, D, default_pmin(pi, 1e5),
                    np.zeros(2), _to4d(U, 2), t_end=1.0,
                    opts=opts or Options(cfl=0.5))


def smooth_materials():
    """Smooth advection materials of Sec. 4.1.4: (rho, gamma, Pinf, D)."""
    return np.array([2.0, 1.0]), np.array([1.5, 1.01]), np.array([0.0, 0.02]), \
        np.array([0.0, 3.0])


def smooth_1d(n, opts=None):
    """Sec. 4.1.4: alpha_1 = 0.2 (3 + sin 2 pi x), u = 1, P = 1, periodic
    [0,1]; exact cell averages; dt = dx^(5/3)."""
    rho, g, pi, D = smooth_materials()
    dx = 1.0 / n
    xl = np.arange(n) * dx
    xr = xl + dx
    a1 = 0.6 + 0.2 * (np.cos(2 * np.pi * xl) - np.cos(2 * np.pi * xr)) / (2 * np.pi * dx)
    alpha = np.stack([a1, 1.0 - a1])
    m = rho[:, None] * alpha
    U = conserved(alpha, m, np.ones((1, n)), 1.0, g, pi, D)
    return Workload("smooth_1d_%d" % n, 1, (n,), (dx,),
                    ((BC_PERIODIC, BC_PERIODIC),), g, pi, D, default_pmin(pi, 1.0),
                    np.zeros(2), _to4d(U, 1), t_end=1.0,
                    opts=opts or Options(cfl=0.5), dt_fixed=dx ** (5.0 / 3.0))


def smooth_1d_exact_alpha(n, t):
    """Exact cell averages of alpha_1 of smooth_1d after time t (u = 1)."""
    dx = 1.0 / n
    xl = np.arange(n) * dx - t
    xr = xl + dx
    return 0.6 + 0.2 * (np.cos(2 * np.pi * xl) - np.cos(2 * np.pi * xr)) / (2 * np.pi * dx)


def smooth_2d(n, opts=None):
    """2D smooth advection: alpha_1 = 0.2 (3 + sin 2pi x sin 2pi y), u = v = 1,
    P = 1, the Sec. 4.1.4 materials, exact cell averages, dt = dx^(5/3)."""
    rho, g, pi, D = smooth_materials()
    dx = 1.0 / n
    xl = np.arange(n) * dx
    xr = xl + dx
    sx = (np.cos(2 * np.pi * xl) - np.cos(2 * np.pi * xr)) / (2 * np.pi * dx)
    a1 = 0.6 + 0.2 * np.outer(sx, sx)
    alpha = np.stack([a1, 1.0 - a1])
    m = rho[:, None, None] * alpha
    U = conserved(alpha, m, np.ones((2, n, n)), 1.0, g, pi, D)
    return Workload("smooth_2d_%d" % n, 2, (n, n), (dx, dx),
                    ((BC_PERIODIC,) * 2,) * 2, g, pi, D, default_pmin(pi, 1.0),
                    np.zeros(2), _to4d(U, 2), t_end=1.0,
                    opts=opts or Options(cfl=0.5), dt_fixed=dx ** (5.0 / 3.0))


def shock_bubble_2d(nx=2048, ny=1024, p_shock=1e9, opts=None):
    """2D shock-bubble: [0,2]x[0,1], water (SI) at rest with P = 1e5, air
    bubble r = 0.1 at (0.6, 0.5), right-moving shock at x = 0.4 with the
    Rankine-Hugoniot post-shock state for p_shock; outflow on all sides."""
    g, pi, D = _eos([AIR_SI, WATER_SI])
    rho = np.array([1.0, 1000.0])
    dx = 2.0 / nx
    dy = 1.0 / ny
    a1 = cell_average_2d(lambda X, Y: _tanh_disc(X, Y, 0.6, 0.5, 0.1, dx), nx, ny,
                         ((0, 2), (0, 1)))
    a1 = np.clip(a1, 0.0, 1.0)
    alpha = np.stack([a1, 1.0 - a1])
    rho2s, u2s, S = rh_post_shock(g[1], pi[1], rho[1], 1e5, p_shock)
    xc = (np.arange(nx) + 0.5) * dx
    post = np.broadcast_to(xc < 0.4, (ny, nx))
    rho2 = np.where(post, rho2s, rho[1])
    m = np.stack([rho[0] * alpha[0], rho2 * alpha[1]])
    u = np.zeros((2, ny, nx))
    u[0] = np.where(post, u2s, 0.0)
    P = np.where(post, p_shock, 1e5)
    U = conserved(alpha, m, u, P, g, pi, D)
    return Workload("shock_bubble_%dx%d" % (nx, ny), 2, (nx, ny), (dx, dy),
                    ((BC_OUTFLOW,) * 2,) * 2, g, pi, D, default_pmin(pi, 1e5),
                    np.zeros(2), _to4d(U, 2), t_end=(2.0 - 0.4) / S,
                    opts=opts or Options(flux=FLUX_HLL, cfl=0.2))


def shock_interface_n3(n=1024, p_shock=1e9, strip=True, opts=None):
    """2D three-phase shock-interface: [0,1]^2, outflow.  Phase 1 gas
    (1.4, 0, rho 1) bubble r = 0.1 at the centre; phase 2 (4.4, 6e8, 1000)
    shell 0.1 < r < 0.15 and (if strip) the cell-aligned strip x >= 0.85 where
    phase 3 is absent; phase 3 (6.12, 3.43e8, 1030) elsewhere; shock in phase
    3 at x = 0.25 with the Rankine-Hugoniot state for p_shock."""
    g, pi, D = _eos([AIR_SI, CAVITY_WATER_SI, WATER_SI])
    rho = np.array([1.0, 1000.0, 1030.0])
    dx = 1.0 / n
    box = ((0, 1), (0, 1))
    a1 = cell_average_2d(lambda X, Y: _tanh_disc(X, Y, 0.5, 0.5, 0.10, dx), n, n, box)
    a12 = cell_average_2d(lambda X, Y: _tanh_disc(X, Y, 0.5, 0.5, 0.15, dx), n, n, box)
    a1 = np.clip(a1, 0.0, 1.0)
    a2 = np.clip(a12 - a1, 0.0, 1.0)
    a3 = np.clip(1.0 - a1 - a2, 0.0, 1.0)
    xc = (np.arange(n) + 0.5) * dx
    if strip:
        s = np.broadcast_to(xc >= 0.85, (n, n))
        a1 = np.where(s, 0.0, a1)
        a2 = np.where(s, 1.0, a2)
        a3 = np.where(s, 0.0, a3)
    alpha = np.stack([a1, a2, a3])
    r3, u3, S = rh_post_shock(g[2], pi[2], rho[2], 1e5, p_shock)
    post = np.broadcast_to(xc < 0.25, (n, n))
    m = np.stack([rho[0] * a1, rho[1] * a2, np.where(post, r3, rho[2]) * a3])
    u = np.zeros((2, n, n))
    u[0] = np.where(post, u3, 0.0)
    P = np.where(post, p_shock, 1e5)
    U = conserved(alpha, m, u, P, g, pi, D)
    return Workload("shock_interface_n3_%d" % n, 2, (n, n), (dx, dx),
                    ((BC_OUTFLOW,) * 2,) * 2, g, pi, D, default_pmin(pi, 1e5),
                    np.zeros(3), _to4d(U, 2), t_end=0.75 / S,
                    opts=opts or Options(flux=FLUX_HLL, cfl=0.2,
                                         precision=PREC_MIXED))


def batched_draw(seed=0, count=256):
    """The batched parameter sweep: per instance (n, N, r, P_s) drawn with
    numpy's default_rng(seed) in this order."""
    rng = np.random.default_rng(seed)
    n = rng.integers(64, 513, count)
    N = rng.integers(2, 4, count)
    r = rng.uniform(0.05, 0.2, count)
    Ps = rng.uniform(1e8, 2e9, count)
    return n, N, r, Ps


def batched_instance(n, N, r, Ps, opts=None):
    """One shock-bubble instance of the batched sweep: [0,1]^2, n x n, outflow;
    gas bubble r at the centre in water (SI); for N = 3 a (4.4, 6e8, 1000)
    shell of thickness r/2 around it; shock at x_s = 0.5 - 1.5 r - 0.05."""
    n, N = int(n), int(N)
    mats = [AIR_SI, WATER_SI] + ([CAVITY_WATER_SI] if N == 3 else [])
    g, pi, D = _eos(mats)
    rho = np.array([1.0, 1000.0, 1000.0][:N])
    dx = 1.0 / n
    box = ((0, 1), (0, 1))
    a1 = np.clip(cell_average_2d(lambda X, Y: _tanh_disc(X, Y, 0.5, 0.5, r, dx),
                                 n, n, box), 0.0, 1.0)
    if N == 3:
        a13 = np.clip(cell_average_2d(
            lambda X, Y: _tanh_disc(X, Y, 0.5, 0.5, 1.5 * r, dx), n, n, box), 0.0, 1.0)
        a3 = np.clip(a13 - a1, 0.0, 1.0)
        a2 = np.clip(1.0 - a1 - a3, 0.0, 1.0)
        alpha = np.stack([a1, a2, a3])
    else:
        alpha = np.stack([a1, 1.0 - a1])
    xs = 0.5 - 1.5 * r - 0.05
    r2, u2, S = rh_post_shock(g[1], pi[1], rho[1], 1e5, Ps)
    xc = (np.arange(n) + 0.5) * dx
    post = np.broadcast_to(xc < xs, (n, n))
    m = np.stack([rho[p] * alpha[p] if p != 1 else np.where(post, r2, rho[1]) * alpha[1]
                  for p in range(N)])
    u = np.zeros((2, n, n))
    u[0] = np.where(post, u2, 0.0)
    P = np.where(post, Ps, 1e5)
    U = conserved(alpha, m, u, P, g, pi, D)
    return Workload("batched_n%d_N%d" % (n, N), 2, (n, n), (dx, dx),
                    ((BC_OUTFLOW,) * 2,) * 2, g, pi, D, default_pmin(pi, 1e5),
                    np.zeros(N), _to4d(U, 2), t_end=(1.0 - xs) / S,
                    opts=opts or Options(flux=FLUX_HLL, cfl=0.2,
                                         precision=PREC_MIXED))


def batched(seed=0, count=256, opts=None, select=None):
    n, N, r, Ps = batched_draw(seed, count)
    idx = range(count) if select is None else select
    return [batched_instance(n[i], N[i], r[i], Ps[i], opts) for i in idx]


GELATIN_SI = (6.72, 3.70e8, 0.0)          # 10 % gelatin ("tissue")


def shock_vessel_bubble_3d(nx=400, ny=200, nz=200, opts=None):
    """The shock-vessel-bubble problem (Sec. "Shock-vessel-bubble
    interaction"): a quarter of the domain, [-50, 50] x [0, 50] x [0, 50] um,
    with symmetry planes at y = 0 and z = 0 and outflow elsewhere.  Phase 1
    air bubble r = 10 um at the origin, inside a water vessel (phase 2, the
    cylinder of radius 13 um about the z axis), in gelatin (phase 3); a
    40 MPa shock in the gelatin at x > 20 um moving left (u = -24.2 m/s,
    rho_3 = 1046).  The sharp initial interfaces of the paper are smoothed
    over one cell (alpha = (1 + tanh(psi / dx)) / 2 at the cell centres) so
    that the state is a smooth function of position at the grid scale."""
    g, pi, D = _eos([AIR_SI, WATER_SI, GELATIN_SI])
    L = 50e-6
    dx, dy, dz = 2 * L / nx, L / ny, L / nz
    x = -L + (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    z = (np.arange(nz) + 0.5) * dz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    w = min(dx, dy, dz)
    a1 = 0.5 * (1.0 + np.tanh((10e-6 - np.sqrt(X ** 2 + Y ** 2 + Z ** 2)) / w))
    out = 0.5 * (1.0 + np.tanh((np.sqrt(X ** 2 + Y ** 2) - 13e-6) / w))
    a3 = (1.0 - a1) * out
    a2 = np.clip(1.0 - a1 - a3, 0.0, 1.0)
    alpha = np.stack([a1, a2, a3])
    post = X > 20e-6
    rho3 = np.where(post, 1046.0, 1030.0)
    m = np.stack([1.204 * a1, 1000.0 * a2, rho3 * a3])
    # the shock lies in the gelatin: velocity and pressure follow phase 3
    u = np.zeros((3,) + X.shape)
    u[0] = np.where(post, -24.2, 0.0) * a3
    P = np.where(post, 101325.0 + (4.0e7 - 101325.0) * a3, 101325.0)
    U = conserved(alpha, m, u, P, g, pi, D)
    bc = ((BC_OUTFLOW, BC_OUTFLOW), (BC_SYMMETRY, BC_OUTFLOW), (BC_SYMMETRY, BC_OUTFLOW))
    return Workload("shock_vessel_bubble_%dx%dx%d" % (nx, ny, nz), 3, (nx, ny, nz),
                    (dx, dy, dz), bc, g, pi, D, default_pmin(pi, 101325.0),
                    np.zeros(3), U, 0.0,
                    opts or Options(flux=FLUX_HLL, cfl=0.2))


# ---------------------------------------------------------------------------
# the paper's verification problems (Sec. 4.1)
# ---------------------------------------------------------------------------

def paper_two_phase_advection(n=100, opts=None):
    """Sec. 4.1.1: [-0.5,0.5]^2 periodic, air circle r = 0.2 in water,
    non-dimensional materials, u = (1,1), P0 = 4.819e-5, T0 = 300, dt = 1e-3;
    C^T_p from the thermal-equilibrium rule of that section."""
    rho = np.array([1.204e-3, 1.0])
    g = np.array([1.4, 6.12])
    pi = np.array([0.0, 0.1631])
    D = np.zeros(2)
    P0, T0 = 4.819e-5, 300.0
    A = 1.0 / (g - 1.0)
    B = g * pi / (g - 1.0)
    cT = (A * P0 + B - pi) / (rho * T0)
    dx = 1.0 / n
    a1 = np.clip(cell_average_2d(lambda X, Y: _tanh_disc(X, Y, 0.0, 0.0, 0.2, dx),
                                 n, n, ((-0.5, 0.5), (-0.5, 0.5))), 0.0, 1.0)
    alpha = np.stack([a1, 1.0 - a1])
    m = rho[:, None, None] * alpha
    U = conserved(alpha, m, np.ones((2, n, n)), P0, g, pi, D)
    return Workload("paper_two_phase_%d" % n, 2, (n, n), (dx, dx),
                    ((BC_PERIODIC,) * 2,) * 2, g, pi, D, default_pmin(pi, P0), cT,
                    _to4d(U, 2), t_end=1.0, opts=opts or Options(), dt_fixed=1e-3)


FIVE_PHASE_TABLE = (
    # rho, gamma, Pinf, D  (Table 1)
    (1.204e-3, 1.4, 0.0, 0.0),
    (1.0, 6.12, 0.163, 0.0),
    (0.8, 2.35, 0.476, -5.55e-4),
    (0.1e-3, 1.6, 0.0, 0.0),
    (1.0e-3, 3.0, 0.0, 0.0),
)


def paper_five_phase(n=100, opts=None, nphase=5):
    """Sec. 4.1.2 / Table 1: background phase 1, disc of phase 2 at the
    centre (r 0.2), discs of phase 3 at (0, +-0.5) and of phase 4 at
    (+-0.5, 0) (r 0.15), phase 5 absent; u = (1,1), P0 = 4.819e-5."""
    tab = np.array(FIVE_PHASE_TABLE[:nphase])
    rho, g, pi, D = tab[:, 0], tab[:, 1], tab[:, 2], tab[:, 3]
    P0 = 4.819e-5
    dx = 1.0 / n
    box = ((-0.5, 0.5), (-0.5, 0.5))

    def disc_sum(centres, r):
        # periodic images so the discs on the boundary are whole
        def f(X, Y):
            s = np.zeros_like(X)
            for (cx, cy) in centres:
                for ox in (-1.0, 0.0, 1.0):
                    for oy in (-1.0, 0.0, 1.0):
                        s = s + _tanh_disc(X, Y, cx + ox, cy + oy, r, dx)
            return np.clip(s, 0.0, 1.0)
        return cell_average_2d(f, n, n, box)

    a2 = disc_sum([(0.0, 0.0)], 0.2)
    a3 = disc_sum([(0.0, 0.5)], 0.15)
    a4 = disc_sum([(0.5, 0.0)], 0.15)
    a1 = np.clip(1.0 - a2 - a3 - a4, 0.0, 1.0)
    alist = [a1, a2, a3, a4] + [np.zeros_like(a1)] * (nphase - 4)
    alpha = np.stack(alist[:nphase])
    m = rho[:, None, None] * alpha
    U = conserved(alpha, m, np.ones((2, n, n)), P0, g, pi, D)
    return Workload("paper_five_phase_%d" % n, 2, (n, n), (dx, dx),
                    ((BC_PERIODIC,) * 2,) * 2, g, pi, D, default_pmin(pi, P0),
                    np.zeros(nphase), _to4d(U, 2), t_end=1.0,
                    opts=opts or Options(), dt_fixed=1e-3)


def paper_four_phase_miscible(n=100, opts=None):
    """Sec. 4.1.3: alpha_1 = 0.8 in the disc r = 0.2, alpha_2 = 0.8 outside,
    alpha_3 = 0.2 everywhere, alpha_4 = 0; Table 1 materials."""
    tab = np.array(FIVE_PHASE_TABLE[:4])
    rho, g, pi, D = tab[:, 0], tab[:, 1], tab[:, 2], tab[:, 3]
    P0 = 4.819e-5
    dx = 1.0 / n
    h = np.clip(cell_average_2d(lambda X, Y: _tanh_disc(X, Y, 0.0, 0.0, 0.2, dx),
                                n, n, ((-0.5, 0.5), (-0.5, 0.5))), 0.0, 1.0)
    a1 = 0.8 * h
    a3 = np.full_like(h, 0.2)
    a2 = 0.8 - a1
    a4 = np.zeros_like(h)
    alpha = np.stack([a1, a2, a3, a4])
    m = rho[:, None, None] * alpha
    U = conserved(alpha, m, np.ones((2, n, n)), P0, g, pi, D)
    return Workload("paper_four_phase_%d" % n, 2, (n, n), (dx, dx),
                    ((BC_PERIODIC,) * 2,) * 2, g, pi, D, default_pmin(pi, P0),
                    np.zeros(4), _to4d(U, 2), t_end=1.0,
                    opts=opts or Options(recon=RECON_WENO_CL), dt_fixed=1e-3)


CAVITY_AIR = (1.4, 0.0, 0.0)              # Sec. 4.2.1, nondimensional
CAVITY_WATER = (4.4, 6000.0, 0.0)


def cavity_collapse(nx=1600, ny=800, opts=None, t_end=0.02):
    """Sec. 4.2.1 (Eq. (32)): shock-induced collapse of an air cavity in
    water on [0, 10] x [-2.5, 2.5], outflow: air (phase 1, gamma 1.4,
    rho 1e-3) inside the circle of radius 1 about (4.375, 0), water (phase 2,
    gamma 4.4, Pinf 6000, rho 1, P = 1) elsewhere, and the post-shock water
    state (rho 1.325, u 68.52, P = 1.915e4) left of x_S = 1.  The sharp
    regions of Eq. (32) enter as cell averages (4 x 4 Gauss points per cell,
    so interface cells hold the area fraction).  HLL, CFL 0.2 (Sec. 4.2)."""
    g, pi, D = _eos([CAVITY_AIR, CAVITY_WATER])
    box = ((0.0, 10.0), (-2.5, 2.5))
    dx, dy = 10.0 / nx, 5.0 / ny
    a1 = cell_average_2d(lambda X, Y: (np.hypot(X - 4.375, Y) <= 1.0).astype(np.float64),
                         nx, ny, box)
    post = cell_average_2d(lambda X, Y: (X < 1.0).astype(np.float64), nx, ny, box)
    a1 = np.clip(a1, 0.0, 1.0)
    alpha = np.stack([a1, 1.0 - a1])
    rho2 = 1.0 + post * (1.325 - 1.0)
    m = np.stack([1.0e-3 * alpha[0], rho2 * alpha[1]])
    u = np.zeros((2, ny, nx))
    u[0] = post * 68.52
    P = 1.0 + post * (1.915e4 - 1.0)
    U = conserved(alpha, m, u, P, g, pi, D)
    return Workload("cavity_%dx%d" % (nx, ny), 2, (nx, ny), (dx, dy),
                    ((BC_OUTFLOW,) * 2,) * 2, g, pi, D, default_pmin(pi, 1.0),
                    np.zeros(2), _to4d(U, 2), t_end=t_end,
                    opts=opts or Options(flux=FLUX_HLL, cfl=0.2))


def air_helium_shock_tube(dx=0.01, opts=None):
    """Sec. 4.1.5 (Eq. (31)): [0,2], helium (phase 1, gamma 1.6) and air
    (phase 2, gamma 1.4); left (0,1]: pure air, P = 1; right: pure helium,
    P = 0.1; rho_1 = 0.125, rho_2 = 1; CFL 0.4; outflow."""
    n = int(round(2.0 / dx))
    g = np.array([1.6, 1.4])
    pi = np.zeros(2)
    D = np.zeros(2)
    xc = (np.arange(n) + 0.5) * dx
    left = xc <= 1.0
    a1 = np.where(left, 0.0, 1.0)
    alpha = np.stack([a1, 1.0 - a1])
    m = np.stack([0.125 * alpha[0], 1.0 * alpha[1]])
    P = np.where(left, 1.0, 0.1)
    U = conserved(alpha, m, np.zeros((1, n)), P, g, pi, D)
    return Workload("air_helium_%d" % n, 1, (n,), (dx,),
                    ((BC_OUTFLOW, BC_OUTFLOW),), g, pi, D, default_pmin(pi, 0.1),
                    np.zeros(2), _to4d(U, 1), t_end=0.4,
                    opts=opts or Options(cfl=0.4))


# ---------------------------------------------------------------------------
# random admissible states for parity tests
# ---------------------------------------------------------------------------

def pf_bubble(shape, nphase=2, width=1.0, bc=BC_PERIODIC, u=(1.0, 0.5, 0.25),
              r=0.25, opts=None):
    """A Phase-Field test state: gas bubble (radius r of the unit box, tanh
    profile `width` cells wide) in water (SI); for N = 3 a shell of the third
    liquid (thickness r/2) around it; uniform velocity and P = 1e5.  1D: a
    slab [0.5 - r, 0.5 + r]; 3D: a ball about the box centre.  Cell averages
    by Gauss quadrature."""
    shape = tuple(shape)
    ndim = len(shape)
    N = nphase
    mats = [AIR_SI, WATER_SI, CAVITY_WATER_SI][:N]
    g, pi, D = _eos(mats)
    rho = np.array([1.0, 1000.0, 1030.0])[:N]
    if ndim == 1:
        n = shape[0]
        dx = 1.0 / n
        w = width * dx
        a1 = np.clip(cell_average_1d(lambda x: _tanh_slab(x, 0.5 - r, 0.5 + r, w),
                                     n, 0.0, 1.0), 0.0, 1.0)
        if N == 3:
            a13 = np.clip(cell_average_1d(
                lambda x: _tanh_slab(x, 0.5 - 1.5 * r, 0.5 + 1.5 * r, w), n, 0.0, 1.0), 0.0, 1.0)
        dxs = (dx,)
        vel = np.full((1, n), float(u[0]))
    elif ndim == 3:
        nx, ny, nz = shape
        dx = 1.0 / nx
        w = width * dx
        box = ((0, 1), (0, ny / nx), (0, nz / nx))
        c = (0.5, 0.5 * ny / nx, 0.5 * nz / nx)
        a1 = np.clip(cell_average_3d(lambda X, Y, Z: _tanh_ball(X, Y, Z, c, r, w),
                                     nx, ny, nz, box), 0.0, 1.0)
        if N == 3:
            a13 = np.clip(cell_average_3d(
                lambda X, Y, Z: _tanh_ball(X, Y, Z, c, 1.5 * r, w), nx, ny, nz, box), 0.0, 1.0)
        dxs = (dx, dx, dx)
        vel = np.stack([np.full((nz, ny, nx), float(u[k])) for k in range(3)])
    else:
        nx, ny = shape
        dx = 1.0 / nx
        w = width * dx
        box = ((0, 1), (0, ny / nx))
        yc = 0.5 * ny / nx
        a1 = np.clip(cell_average_2d(lambda X, Y: _tanh_disc(X, Y, 0.5, yc, r, w),
                                     nx, ny, box), 0.0, 1.0)
        if N == 3:
            a13 = np.clip(cell_average_2d(
                lambda X, Y: _tanh_disc(X, Y, 0.5, yc, 1.5 * r, w), nx, ny, box), 0.0, 1.0)
        dxs = (dx, dx)
        vel = np.stack([np.full((ny, nx), float(u[0])), np.full((ny, nx), float(u[1]))])
    if N == 3:
        a3 = np.clip(a13 - a1, 0.0, 1.0)
        alpha = np.stack([a1, 1.0 - a1 - a3, a3])
        alpha[1] = np.clip(alpha[1], 0.0, 1.0)
    else:
        alpha = np.stack([a1, 1.0 - a1])
    m = np.stack([rho[p] * alpha[p] for p in range(N)])
    U = conserved(alpha, m, vel, 1e5, g, pi, D)
    o = opts or Options(flux=FLUX_HLL, cfl=0.2, phase_field=1)
    return Workload("pf_bubble_%s_N%d" % ("x".join(map(str, shape)), N), ndim, shape,
                    dxs, ((bc, bc),) * ndim, g, pi, D, default_pmin(pi, 1e5),
                    np.zeros(N), _to4d(U, ndim), t_end=0.0, opts=o)


def random_state(shape, nphase=2, seed=0, ndim=None, bc=BC_PERIODIC,
                 si=True, absent=(), opts=None, rough=0.5, lowp=0.02):
    """Admissible but rough states: sharp material jumps, mixed cells, random
    velocities and pressures, some cells close to the minimum pressure, and
    the phases listed in `absent` identically zero.  Seeded."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape)
    ndim = ndim or len(shape)
    N = nphase
    if si:
        pal = [AIR_SI, WATER_SI, CAVITY_WATER_SI, (1.6, 0.0, 0.0),
               (2.35, 4.76e7, 0.0), (4.4, 6.0e8, 0.0), (1.4, 0.0, 0.0), (6.12, 3.43e8, 0.0)]
        rho_ref = np.array([1.2, 1000.0, 1030.0, 0.17, 800.0, 1000.0, 1.0, 1000.0])
        p_ref = 1e5
        u_ref = 50.0
    else:
        pal = [(1.4, 0.0, 0.0), (6.12, 0.1631, 0.0), (2.35, 0.476, -5.55e-4),
               (1.6, 0.0, 0.0), (3.0, 0.0, 0.0), (1.5, 0.0, 0.0), (1.01, 0.02, 3.0),
               (1.4, 0.0, 0.0)]
        rho_ref = np.array([1.204e-3, 1.0, 0.8, 1e-4, 1e-3, 2.0, 1.0, 1.0])
        p_ref = 1.0
        u_ref = 1.0
    g, pi, D = _eos(pal[:N])
    rho_ref = rho_ref[:N]
    # smooth blobs plus a fraction of random (rough) cells
    coords = np.meshgrid(*[np.linspace(0, 1, s, endpoint=False) for s in shape],
                         indexing="ij")
    w = rng.uniform(0.2, 1.0, size=(N,) + shape)
    for p in range(N):
        ph = rng.uniform(0, 2 * np.pi, size=len(shape))
        k = rng.integers(1, 4, size=len(shape))
        s = np.ones(shape)
        for j, c in enumerate(coords):
            s = s * np.sin(2 * np.pi * k[j] * c + ph[j])
        w[p] = np.where(s > rng.uniform(-0.3, 0.3), w[p] + 2.0, w[p])
    rough_mask = rng.random(shape) < rough
    pure = rng.integers(0, N, size=shape)
    wr = np.where(rng.random((N,) + shape) < 0.5, 0.0, rng.random((N,) + shape))
    for p in range(N):
        wr[p] = np.where(pure == p, wr[p] + 1.0, wr[p])
    w = np.where(rough_mask[None], wr, w)
    sharp = rng.random(shape) < 0.5
    for p in range(N):
        w[p] = np.where(sharp & (w[p] < w.max(axis=0)), 0.0, w[p])
    for p in absent:
        w[p] = 0.0
    present = [p for p in range(N) if p not in absent]
    empty = w.sum(axis=0) == 0.0
    w[present[0]] = np.where(empty, 1.0, w[present[0]])
    alpha = w / w.sum(axis=0, keepdims=True)
    rho_p = rho_ref.reshape((N,) + (1,) * len(shape)) * \
        rng.uniform(0.5, 2.0, size=(N,) + shape)
    m = rho_p * alpha
    u = u_ref * rng.uniform(-1, 1, size=(ndim,) + shape)
    P = p_ref * rng.uniform(0.5, 2.0, size=shape)
    pmin = default_pmin(pi, p_ref)
    # a few cells close to the smallest admissible pressure of their mixture
    low = rng.random(shape) < lowp
    pfloor = np.max(np.where(alpha > 0, pmin.reshape((N,) + (1,) * len(shape)), -np.inf),
                    axis=0)
    P = np.where(low, pfloor + 1e-3 * (p_ref + np.abs(pfloor)), P)
    U = conserved(alpha, m, u, P, g, pi, D)
    bcs = tuple((bc, bc) for _ in range(ndim))
    return Workload("random_%s_N%d_s%d" % ("x".join(map(str, shape)), N, seed), ndim,
                    tuple(reversed(shape)) if ndim > 1 else shape,
                    tuple(1.0 / s for s in reversed(shape)) if ndim > 1 else (1.0 / shape[0],),
                    bcs, g, pi, D, pmin, np.zeros(N), _to4d(U, ndim),
                    opts=opts or Options())
