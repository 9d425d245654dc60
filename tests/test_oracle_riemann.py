"""Pins of the oracle's interface fluxes where the waves meet: the star region
of HLLC, the HLL fan state and the Davis wave speeds (Sec. 4.1 HLLC, Sec. 4.2
HLL; the solvers are only cited by the paper, their reading is Davis speeds,
Toro's contact speed and star states, and the three-branch HLL formula).

Independent references:
* an exact Riemann solver for two stiffened gases (oracle/exact_riemann.py),
  itself pinned to the textbook star states of Toro's Table 4.2 and to the
  Rankine-Hugoniot conditions and Riemann invariants it must satisfy;
* the integral form of the conservation laws over the wave fan: for any
  speeds S_L <= (slowest wave) and S_R >= (fastest wave), the average of the
  exact solution over [S_L t, S_R t] is
  (S_R U_R - S_L U_L - (F_R - F_L)) / (S_R - S_L), and the HLL flux is
  F_L + S_L (that average - U_L);
* Galilean invariance: the flux of a problem seen from a frame moving with
  speed V is the boosted flux, so the contact of HLLC can be put on either
  side of the face and both star states read off the flux.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import exact_riemann as ER

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# the exact solver
# ---------------------------------------------------------------------------

def test_exact_solver_textbook_star_states():
    d = json.load(open(os.path.join(GOLD, "toro_star_states.json")))
    g = d["gamma"]
    for case in d["cases"]:
        L = ER.Side(*case["left"], g)
        R = ER.Side(*case["right"], g)
        p, u = ER.star_state(L, R)
        # the table prints 6 significant digits (5 for u* = 0)
        assert abs(p - case["p_star"]) <= 6e-6 * abs(case["p_star"]) + 6e-6, (case, p)
        assert abs(u - case["u_star"]) <= 6e-6 * abs(case["u_star"]) + 6e-6, (case, u)


def _rand_side(rng, mat):
    g, pinf, rho0, p0 = mat
    return ER.Side(rho0 * rng.uniform(0.5, 2.0), rng.uniform(-1, 1) * math.sqrt(g * (p0 + pinf) / rho0),
                   p0 * 10 ** rng.uniform(-1, 1), g, pinf)


MATS = [(1.4, 0.0, 1.0, 1e5), (6.12, 3.43e8, 1000.0, 1e5), (1.6, 0.0, 0.125, 1e5),
        (4.4, 6e8, 1000.0, 1e6)]


@pytest.mark.parametrize("seed", range(6))
def test_exact_solver_jump_conditions(seed):
    """Across each computed shock the mass, momentum and energy fluxes in
    the shock frame agree (Rankine-Hugoniot); across each rarefaction the
    entropy P + Pinf over rho^gamma and the Riemann invariant
    u -+ 2c/(gamma - 1) are those of the undisturbed side."""
    rng = np.random.default_rng(seed)
    for _ in range(20):
        L = _rand_side(rng, MATS[rng.integers(len(MATS))])
        R = _rand_side(rng, MATS[rng.integers(len(MATS))])
        try:
            ps, us = ER.star_state(L, R)
        except ValueError:
            continue
        for s, sign in ((L, -1), (R, +1)):
            # the star state of this side: sample just on its side of the contact
            smin, smax = ER.wave_speeds(L, R)
            xi = us + sign * 1e-9 * (abs(us) + abs(smax - smin))
            rho_s, u_s, P_s, side = ER.sample(L, R, np.array([xi]))
            rho_s, u_s, P_s = float(rho_s[0]), float(u_s[0]), float(P_s[0])
            assert abs(u_s - us) <= 1e-12 * (abs(us) + s.c)
            assert abs(P_s - ps) <= 1e-12 * (abs(ps) + s.pinf)
            if ps + s.pinf > s.pbar:
                S = smin if sign < 0 else smax
                def fluxes(rho, u, P):
                    _, m, E = ER.conserved(rho, u, P, s.gamma, s.pinf)
                    return np.array([rho * (u - S), m * (u - S) + P, E * (u - S) + P * u])
                fa, fb = fluxes(s.rho, s.u, s.P), fluxes(rho_s, u_s, P_s)
                scale = np.abs(fa).max() + abs(S) * (s.rho * (abs(S) + s.c) * (s.c + abs(S)))
                assert np.abs(fa - fb).max() <= 1e-10 * scale, (fa, fb)
            else:
                g = s.gamma
                ent0 = s.pbar / s.rho ** g
                ent1 = (P_s + s.pinf) / rho_s ** g
                assert abs(ent1 - ent0) <= 1e-10 * ent0
                cs = math.sqrt(g * (P_s + s.pinf) / rho_s)
                inv0 = s.u - sign * 2 * s.c / (g - 1)
                inv1 = u_s - sign * 2 * cs / (g - 1)
                assert abs(inv1 - inv0) <= 1e-10 * (abs(s.u) + s.c)


def test_exact_solver_fan_average_matches_integral_form():
    """The numerical fan average equals the integral-form expression (checks
    the sampling of every wave, not only the star state)."""
    L = ER.Side(1.0, 0.0, 1.0, 1.4)
    R = ER.Side(0.125, 0.0, 0.1, 1.6)
    smin, smax = ER.wave_speeds(L, R)
    sl, sr = smin - 0.3, smax + 0.2
    avg = ER.fan_average(L, R, sl, sr)
    UL = np.array(ER.conserved(L.rho, L.u, L.P, L.gamma, L.pinf))
    UR = np.array(ER.conserved(R.rho, R.u, R.P, R.gamma, R.pinf))
    FL = np.array([UL[1], UL[1] * L.u + L.P, L.u * (UL[2] + L.P)])
    FR = np.array([UR[1], UR[1] * R.u + R.P, R.u * (UR[2] + R.P)])
    ref = (sr * UR - sl * UL - (FR - FL)) / (sr - sl)
    assert np.allclose(avg[:3], ref, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------------------
# oracle fluxes between two pure materials
# ---------------------------------------------------------------------------

def _pair_problem(oracle, L, R, flux):
    """Two phases, phase 1 = the left material, phase 2 = the right one."""
    return oracle.Problem(1, (8,), (1.0,), ((0, 0),), [L.gamma, R.gamma], [L.pinf, R.pinf],
                          [0.0, 0.0], [-L.pinf, -R.pinf], flux=flux)


def _face(s, first, V=0.0):
    """(U, V) vectors of a pure-material face state seen from a frame moving
    with speed V: phase 1 if first, else phase 2."""
    u = s.u - V
    rho, m, E = ER.conserved(s.rho, u, s.P, s.gamma, s.pinf)
    a = (1.0, 0.0) if first else (0.0, 1.0)
    mp = (rho * a[0], rho * a[1])
    U = np.array([mp[0], mp[1], m, E, a[0], a[1]])
    Vv = np.array([mp[0], mp[1], u, s.P, a[0], a[1]])
    return U, Vv


def _phys(U, Vv):
    u, P = Vv[2], Vv[3]
    return np.array([U[0] * u, U[1] * u, U[2] * u + P, u * (U[3] + P), U[4] * u, U[5] * u])


def _davis(L, R, V=0.0):
    """Davis' estimates (the reading of the cited solvers): the smaller of
    u - c and the larger of u + c over the two face states."""
    return min(L.u - V - L.c, R.u - V - R.c), max(L.u - V + L.c, R.u - V + R.c)


def _cases(rng, n):
    out = []
    while len(out) < n:
        iL, iR = rng.integers(len(MATS)), rng.integers(len(MATS))
        L, R = _rand_side(rng, MATS[iL]), _rand_side(rng, MATS[iR])
        try:
            ER.star_state(L, R)
        except ValueError:
            continue
        out.append((L, R))
    return out


@pytest.mark.parametrize("seed", range(4))
def test_hll_flux_is_the_exact_fan_average(oracle, seed):
    """HLL: F = F_L + S_L (Ubar - U_L) with Ubar the average of the exact
    solution over the Davis fan, for every component that is conserved
    (phase masses, momentum, energy), whenever the Davis speeds bound the
    exact waves.  Cases where the right material is the faster one make
    the min / max of the Davis speeds matter."""
    rng = np.random.default_rng(100 + seed)
    checked = 0
    for L, R in _cases(rng, 40):
        sl, sr = _davis(L, R)
        smin, smax = ER.wave_speeds(L, R)
        if not (sl < 0.0 < sr) or not (sl <= smin and sr >= smax):
            continue
        pb = _pair_problem(oracle, L, R, oracle.FLUX_HLL)
        UL, VL = _face(L, True)
        UR, VR = _face(R, False)
        F, uh = pb.flux(UL, VL, UR, VR)
        avg = ER.fan_average(L, R, sl, sr)
        # the materials' masses: density times the indicator of each material
        Ubar = np.array([avg[4], avg[0] - avg[4], avg[1], avg[2]])
        FL = _phys(UL, VL)
        ref = FL[:4] + sl * (Ubar - UL[:4])
        scale = np.abs(FL[:4]).max() + np.abs(_phys(UR, VR)[:4]).max() + \
            abs(sl) * np.abs(np.concatenate([UL[:4], UR[:4]])).max()
        assert np.abs(F[:4] - ref).max() <= 2e-8 * scale, (F[:4], ref)
        checked += 1
    assert checked >= 5


def _boost(U, V):
    """Conserved vector seen from a frame moving with -V relative to the one
    it was written in (undoes a boost by V)."""
    rho = U[0] + U[1]
    out = U.copy()
    out[3] = U[3] + U[2] * V + 0.5 * rho * V * V
    out[2] = U[2] + rho * V
    return out


@pytest.mark.parametrize("seed", range(4))
def test_hllc_star_states_conserve_and_match_at_the_contact(oracle, seed):
    """HLLC: boosting the problem moves its contact S* across the face, so
    the flux yields the left star state (S* > 0 in the frame) and the right
    one (S* < 0) by the jump condition across S_K; back in the rest frame
    the two star states must
    * move with the contact (u*_L = u*_R = S*) and carry one pressure
      (p*_K = F*_K[momentum] - U*_K[momentum] S* equal on both sides),
    * satisfy the integral form over the fan,
      (S* - S_L) U*_L + (S_R - S*) U*_R = S_R U_R - S_L U_L - (F_R - F_L),
      for every component (masses, momentum, energy, volume fractions),
    * scale masses and volume fractions by one factor per side."""
    rng = np.random.default_rng(200 + seed)
    checked = 0
    for L, R in _cases(rng, 12):
        pb = _pair_problem(oracle, L, R, oracle.FLUX_HLLC)
        sl, sr = _davis(L, R)

        def flux_in_frame(V):
            UL, VL = _face(L, True, V)
            UR, VR = _face(R, False, V)
            return pb.flux(UL, VL, UR, VR)[0]

        # the frame in which the contact does not move: the mass flux through
        # the face, rho*_K (S* - V), changes sign there; bisection on V
        lo, hi = sl, sr
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            F = flux_in_frame(mid)
            if F[0] + F[1] > 0.0:
                lo = mid
            else:
                hi = mid
        ss = 0.5 * (lo + hi)
        U0L, V0L = _face(L, True)
        U0R, V0R = _face(R, False)
        star = {}
        for side, V in (("L", 0.5 * (sl + ss)), ("R", 0.5 * (ss + sr))):
            K = _face(L, True, V) if side == "L" else _face(R, False, V)
            S_rest = sl if side == "L" else sr
            Fm = flux_in_frame(V)
            Us = K[0] + (Fm - _phys(*K)) / (S_rest - V)   # jump across S_K in the frame
            Us = _boost(Us, V)                            # rest frame
            K0 = (U0L, V0L) if side == "L" else (U0R, V0R)
            Fs = _phys(*K0) + S_rest * (Us - K0[0])       # jump across S_K at rest
            star[side] = (Us, Fs)
        UsL, FsL = star["L"]
        UsR, FsR = star["R"]
        rhoL, rhoR = UsL[0] + UsL[1], UsR[0] + UsR[1]
        vscale = abs(sl) + abs(sr)
        assert abs(UsL[2] / rhoL - ss) <= 1e-8 * vscale, (UsL[2] / rhoL, ss)
        assert abs(UsR[2] / rhoR - ss) <= 1e-8 * vscale, (UsR[2] / rhoR, ss)
        pL, pR = FsL[2] - UsL[2] * ss, FsR[2] - UsR[2] * ss
        pscale = abs(L.P) + abs(R.P) + L.pinf + R.pinf + L.rho * L.c ** 2 + R.rho * R.c ** 2
        assert abs(pL - pR) <= 1e-8 * pscale, (pL, pR)
        lhs = (ss - sl) * UsL + (sr - ss) * UsR
        rhs = sr * U0R - sl * U0L - (_phys(U0R, V0R) - _phys(U0L, V0L))
        terms = np.abs(np.stack([sr * U0R, sl * U0L, _phys(U0R, V0R), _phys(U0L, V0L)]))
        scale = terms.max(axis=0)
        assert np.all(np.abs(lhs - rhs) <= 1e-8 * scale + 1e-300), (lhs, rhs)
        # one factor per side for the masses and volume fractions
        chiL = UsL[0] / U0L[0]
        chiR = UsR[1] / U0R[1]
        assert abs(UsL[4] / U0L[4] - chiL) <= 1e-9 * chiL
        assert abs(UsR[5] / U0R[5] - chiR) <= 1e-9 * chiR
        assert abs(UsL[1]) <= 1e-9 * rhoL and abs(UsR[0]) <= 1e-9 * rhoR
        checked += 1
    assert checked >= 10
