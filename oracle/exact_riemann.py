"""Exact solution of the one-dimensional Riemann problem between two
stiffened gases (one pure material on each side of the initial jump).

TEST INFRASTRUCTURE ONLY: an independent mathematical reference for the
oracle's interface fluxes and for the air-helium shock tube of Sec. 4.1.5
(Eq. (31)).  It shares nothing with oracle/mpo.c or with the HIP library.

Each material obeys P = (gamma - 1) rho e - gamma Pinf (Eq. (26) with D = 0),
so with Pbar = P + Pinf the Euler equations of one material are those of an
ideal gas in (rho, u, Pbar): the wave curves below are the ideal-gas ones
written in Pbar, with the left and right materials each keeping their own
(gamma, Pinf).  The pressure P* and velocity u* of the star region solve
f_L(P*) + f_R(P*) + u_R - u_L = 0, where f_K is the shock curve
(Rankine-Hugoniot) for P* > P_K and the rarefaction curve (isentrope,
Riemann invariant) otherwise.  Newton iteration on that scalar equation,
then the self-similar solution is sampled at x / t.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Side:
    rho: float
    u: float
    P: float
    gamma: float
    pinf: float = 0.0

    @property
    def pbar(self) -> float:
        return self.P + self.pinf

    @property
    def c(self) -> float:
        return math.sqrt(self.gamma * self.pbar / self.rho)


def _f_and_df(p: float, s: Side):
    """Velocity jump across the K-wave as a function of the star pressure p
    (the wave curve through the state s) and its derivative."""
    g, pb = s.gamma, s.pbar
    ps = p + s.pinf                      # star pressure in the shifted variable
    if ps > pb:                          # shock: Rankine-Hugoniot
        A = 2.0 / ((g + 1.0) * s.rho)
        B = (g - 1.0) / (g + 1.0) * pb
        q = math.sqrt(A / (ps + B))
        f = (ps - pb) * q
        df = q * (1.0 - 0.5 * (ps - pb) / (ps + B))
    else:                                # rarefaction: isentrope
        e = (g - 1.0) / (2.0 * g)
        r = (ps / pb) ** e
        f = 2.0 * s.c / (g - 1.0) * (r - 1.0)
        df = (1.0 / (s.rho * s.c)) * (ps / pb) ** (-(g + 1.0) / (2.0 * g)) \
            if ps > 0.0 else math.inf
    return f, df


def star_state(L: Side, R: Side, tol: float = 1e-15, maxit: int = 200):
    """(P*, u*) of the Riemann problem (L | R).  Raises if the data create a
    vacuum (the pressure-positivity condition fails)."""
    du = R.u - L.u
    # vacuum check: the two rarefaction curves at the lowest admissible star
    # pressure (Pbar of both sides >= 0 there)
    pmin = max(-L.pinf, -R.pinf)
    fl0, _ = _f_and_df(pmin, L)
    fr0, _ = _f_and_df(pmin, R)
    if fl0 + fr0 + du >= 0.0:
        raise ValueError("the Riemann problem generates a vacuum")
    # start from the two-rarefaction approximation in Pbar when both Pinf
    # agree, else from the arithmetic mean; then safeguarded Newton
    p = 0.5 * (L.P + R.P)
    p = max(p, pmin + 1e-12 * (abs(L.P) + abs(R.P) + L.pinf + R.pinf + 1.0))
    lo, hi = pmin, None
    for _ in range(maxit):
        fl, dfl = _f_and_df(p, L)
        fr, dfr = _f_and_df(p, R)
        F = fl + fr + du
        if F > 0.0:
            hi = p
        else:
            lo = p
        pn = p - F / (dfl + dfr)
        if not (lo < pn and (hi is None or pn < hi)):
            pn = 0.5 * (lo + hi) if hi is not None else 2.0 * p - lo
        if abs(pn - p) <= tol * max(abs(pn) + max(L.pinf, R.pinf), 1e-300):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, L)
    fr, _ = _f_and_df(p, R)
    u = 0.5 * (L.u + R.u) + 0.5 * (fr - fl)
    return p, u


def _side_solution(s: Side, ps: float, us: float, xi, sign: int):
    """rho, u, P at similarity coordinates xi on the side of the contact of
    state s; sign = -1 for the left wave, +1 for the right wave."""
    g, pinf = s.gamma, s.pinf
    pb, pbs = s.pbar, ps + pinf
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    P = np.empty_like(xi)
    if pbs > pb:  # shock
        ratio = pbs / pb
        gm = (g - 1.0) / (g + 1.0)
        rhos = s.rho * (ratio + gm) / (gm * ratio + 1.0)
        S = s.u + sign * s.c * math.sqrt((g + 1.0) / (2.0 * g) * ratio + (g - 1.0) / (2.0 * g))
        outside = (xi < S) if sign < 0 else (xi > S)
        rho[:] = np.where(outside, s.rho, rhos)
        u[:] = np.where(outside, s.u, us)
        P[:] = np.where(outside, s.P, ps)
        return rho, u, P
    # rarefaction: head, tail, and the isentropic fan between them
    rhos = s.rho * (pbs / pb) ** (1.0 / g)
    cs = s.c * (pbs / pb) ** ((g - 1.0) / (2.0 * g))
    head = s.u + sign * s.c
    tail = us + sign * cs
    if sign < 0:
        outside = xi < head
        star = xi > tail
    else:
        outside = xi > head
        star = xi < tail
    # inside the fan: u - sign c = u_K - sign 2 c_K/(g-1) ... written with the
    # characteristic xi = u + sign c and the Riemann invariant of the side
    fac = 2.0 / (g + 1.0)
    cf = fac * (s.c - sign * (g - 1.0) / 2.0 * (s.u - xi))
    cf = np.maximum(cf, 0.0)
    uf = fac * (-sign * s.c + (g - 1.0) / 2.0 * s.u + xi)
    rhof = s.rho * (cf / s.c) ** (2.0 / (g - 1.0))
    pbf = pb * (cf / s.c) ** (2.0 * g / (g - 1.0))
    rho[:] = np.where(outside, s.rho, np.where(star, rhos, rhof))
    u[:] = np.where(outside, s.u, np.where(star, us, uf))
    P[:] = np.where(outside, s.P, np.where(star, ps, pbf - pinf))
    return rho, u, P


def sample(L: Side, R: Side, xi):
    """Exact (rho, u, P, side) at similarity coordinates xi = (x - x0) / t;
    side is 0 where the material is the left one, 1 where it is the right
    one (the contact moves with u*)."""
    ps, us = star_state(L, R)
    xi = np.asarray(xi, dtype=np.float64)
    rl, ul, pl = _side_solution(L, ps, us, xi, -1)
    rr, ur, pr = _side_solution(R, ps, us, xi, +1)
    right = xi > us
    return (np.where(right, rr, rl), np.where(right, ur, ul),
            np.where(right, pr, pl), right.astype(np.int64))


def wave_speeds(L: Side, R: Side):
    """(slowest, fastest) signal speed of the exact solution: the left
    shock or rarefaction head, and the right one."""
    ps, us = star_state(L, R)
    out = []
    for s, sign in ((L, -1), (R, +1)):
        pbs = ps + s.pinf
        if pbs > s.pbar:
            g = s.gamma
            ratio = pbs / s.pbar
            out.append(s.u + sign * s.c * math.sqrt((g + 1.0) / (2.0 * g) * ratio
                                                    + (g - 1.0) / (2.0 * g)))
        else:
            out.append(s.u + sign * s.c)
    return out[0], out[1]


def conserved(rho, u, P, gamma, pinf):
    """Single-material conserved variables (rho, rho u, rho E)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    pinf = np.asarray(pinf, dtype=np.float64)
    rhoe = (P + gamma * pinf) / (gamma - 1.0)
    return rho, rho * u, rhoe + 0.5 * rho * u * u


def fan_average(L: Side, R: Side, sl: float, sr: float, npts: int = 200001):
    """Average over xi in [sl, sr] of the exact conserved solution
    (rho, rho u, rho E, alpha_L, rho alpha_L): by the integral form of the conservation
    laws over [sl t, sr t] x [0, t] it equals
    (sr U_R - sl U_L - (F_R - F_L)) / (sr - sl) whenever sl and sr bound all
    waves.  Composite Simpson on a fine uniform grid of xi, with the exact
    wave positions inserted as break points so that every jump is resolved."""
    ps, us = star_state(L, R)
    breaks = [sl, sr, us]
    for s, sign in ((L, -1), (R, +1)):
        pbs = ps + s.pinf
        if pbs > s.pbar:
            g = s.gamma
            ratio = pbs / s.pbar
            breaks.append(s.u + sign * s.c * math.sqrt((g + 1.0) / (2.0 * g) * ratio
                                                       + (g - 1.0) / (2.0 * g)))
        else:
            cs = s.c * (pbs / s.pbar) ** ((s.gamma - 1.0) / (2.0 * s.gamma))
            breaks += [s.u + sign * s.c, us + sign * cs]
    pts = sorted({b for b in breaks if sl <= b <= sr})
    tot = np.zeros(5)
    per = max(2, (npts // max(len(pts) - 1, 1)) // 2 * 2)
    for a, b in zip(pts[:-1], pts[1:]):
        if b <= a:
            continue
        # open interval: nudge the end points inside the segment so that the
        # sampled state is the one of the segment, not of its neighbour
        x = np.linspace(a, b, per + 1)
        eps = (b - a) * 1e-12
        x[0] += eps
        x[-1] -= eps
        rho, u, P, side = sample(L, R, x)
        g = np.where(side == 1, R.gamma, L.gamma)
        pi = np.where(side == 1, R.pinf, L.pinf)
        r, m, E = conserved(rho, u, P, g, pi)
        aL = (side == 0).astype(np.float64)
        wts = np.ones(per + 1)
        wts[1:-1:2] = 4.0
        wts[2:-1:2] = 2.0
        h = (b - a) / per
        for k, f in enumerate((r, m, E, aL, r * aL)):
            tot[k] += h / 3.0 * np.dot(wts, f)
    return tot / (sr - sl)


def cell_averages(L: Side, R: Side, x0: float, t: float, edges, sub: int = 64):
    """Cell averages of the exact (rho, u, P, alpha_R) at time t over the
    cells with the given edges (midpoint rule on `sub` points per cell;
    alpha_R = 1 where the right material is)."""
    edges = np.asarray(edges, dtype=np.float64)
    n = edges.size - 1
    fr = (np.arange(sub) + 0.5) / sub
    x = edges[:-1, None] + (edges[1:] - edges[:-1])[:, None] * fr[None, :]
    rho, u, P, side = sample(L, R, (x - x0) / t)
    return (rho.mean(axis=1), u.mean(axis=1), P.mean(axis=1),
            side.astype(np.float64).mean(axis=1))
