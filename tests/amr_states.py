"""Shared builders of smooth two-level states for the coupling tests: the
coarse grid and its refined blocks (with their ring of 3 ghost cells) as
cell averages of the same analytic fields."""
import numpy as np

from paper_2608_00746_amd import inputs as I

MATS = [(1.5, 0.0, 0.0), (1.01, 0.02, 3.0)]      # Sec. 4.1.4 materials
RHO = np.array([2.0, 1.0])


def alpha1(X, Y):
    return 0.2 * (3.0 + np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y))


def state(box, nx, ny, N=2, flow=True):
    """Cell averages on box = ((x0, x1), (y0, y1)) with nx x ny cells."""
    a1 = I.cell_average_2d(alpha1, nx, ny, box)
    if N == 2:
        alpha = np.stack([a1, 1.0 - a1])
    else:
        a3 = I.cell_average_2d(lambda X, Y: 0.1 * (1.0 + np.cos(2 * np.pi * X)), nx, ny, box)
        alpha = np.stack([a1, 1.0 - a1 - a3, a3])
    rho = np.array([2.0, 1.0, 1.5])[:N]
    m = rho[:, None, None] * alpha
    if flow:
        u = np.stack([1.0 + 0.2 * I.cell_average_2d(lambda X, Y: np.sin(2 * np.pi * Y), nx, ny, box),
                      0.5 + 0.2 * I.cell_average_2d(lambda X, Y: np.cos(2 * np.pi * X), nx, ny, box)])
    else:
        u = np.stack([np.ones((ny, nx)), 0.5 * np.ones((ny, nx))])
    mats = (MATS + [(2.0, 0.1, 0.0)])[:N]
    g = np.array([m_[0] for m_ in mats])
    pi = np.array([m_[1] for m_ in mats])
    D = np.array([m_[2] for m_ in mats])
    U = I.conserved(alpha, m, u, np.ones((ny, nx)), g, pi, D)
    return U, g, pi, D


def two_level(nc, lo, W, H, N=2, flow=True, opts=None):
    """Workloads (coarse, fine block) on the periodic unit square: coarse
    nc x nc, block [lo, lo + (W, H)) refined by 2 with its ring."""
    h = 1.0 / nc
    Uc, g, pi, D = state(((0, 1), (0, 1)), nc, nc, N, flow)
    x0, y0 = (lo[0] - 1.5) * h, (lo[1] - 1.5) * h
    box = ((x0, x0 + (W + 3) * h), (y0, y0 + (H + 3) * h))
    Uf, *_ = state(box, 2 * W + 6, 2 * H + 6, N, flow)
    pmin = I.default_pmin(pi, 1.0)
    opts = opts or I.Options(flux=I.FLUX_HLL, cfl=0.4)
    wc = I.Workload("coarse", 2, (nc, nc), (h, h), ((0, 0), (0, 0)), g, pi, D, pmin,
                    np.zeros(N), I._to4d(Uc, 2), opts=opts)
    wf = I.Workload("fine", 2, (2 * W + 6, 2 * H + 6), (h / 2, h / 2), ((1, 1), (1, 1)), g, pi,
                    D, pmin, np.zeros(N), I._to4d(Uf, 2), opts=opts)
    return wc, wf
