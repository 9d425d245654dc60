"""Pins of the oracle's WENO building blocks against exact mathematics.

Nothing here retypes the oracle's formulas: candidates and ideal weights are
checked against exact point values of polynomials, the smoothness indicators
against their integral definition evaluated in exact rationals, and the WENO-W
weights against the epsilon -> 0 limit of WENO-JS (a different formula) and
the affine invariance stated in Sec. 3.3.
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_values.json")))


def _poly_cell_avgs(coeffs, centres, h=Fr(1)):
    """Exact cell averages of sum_k c_k x^k over [x-h/2, x+h/2]."""
    out = []
    for xc in centres:
        a, b = xc - h / 2, xc + h / 2
        s = sum(c * (b ** (k + 1) - a ** (k + 1)) / (k + 1) for k, c in enumerate(coeffs))
        out.append(s / h)
    return out


def _peval(coeffs, x):
    return sum(c * x ** k for k, c in enumerate(coeffs))


@pytest.mark.parametrize("seed", range(20))
def test_candidates_exact_on_quadratics(oracle, seed):
    rng = np.random.default_rng(seed)
    co = [Fr(int(v)) / 7 for v in rng.integers(-50, 50, 3)]
    q = _poly_cell_avgs(co, [Fr(j) for j in range(-2, 3)])
    cl, cr = oracle.weno5_candidates([float(v) for v in q])
    exact_l, exact_r = float(_peval(co, Fr(1, 2))), float(_peval(co, Fr(-1, 2)))
    scale = 1 + max(abs(float(v)) for v in q)
    assert np.allclose(cl, exact_l, rtol=0, atol=1e-14 * scale)
    assert np.allclose(cr, exact_r, rtol=0, atol=1e-14 * scale)


@pytest.mark.parametrize("seed", range(20))
def test_ideal_weights_exact_on_quartics(oracle, seed):
    rng = np.random.default_rng(100 + seed)
    co = [Fr(int(v)) / 11 for v in rng.integers(-50, 50, 5)]
    q = _poly_cell_avgs(co, [Fr(j) for j in range(-2, 3)])
    cl, cr = oracle.weno5_candidates([float(v) for v in q])
    dl, dr = oracle.weno5_ideal()
    scale = 1 + max(abs(float(v)) for v in q)
    assert abs(float(np.dot(dl, cl)) - float(_peval(co, Fr(1, 2)))) < 1e-13 * scale
    assert abs(float(np.dot(dr, cr)) - float(_peval(co, Fr(-1, 2)))) < 1e-13 * scale
    assert abs(sum(dl) - 1) < 1e-15 and abs(sum(dr) - 1) < 1e-15


def _quad_from_avgs(centres, avgs):
    # average over [x-1/2, x+1/2] of a + b x + c x^2 = a + b x + c (x^2 + 1/12)
    M = [[Fr(1), Fr(x), Fr(x) ** 2 + Fr(1, 12)] for x in centres]
    A = [row[:] + [v] for row, v in zip(M, avgs)]
    n = 3
    for i in range(n):
        piv = next(r for r in range(i, n) if A[r][i] != 0)
        A[i], A[piv] = A[piv], A[i]
        for r in range(n):
            if r != i and A[r][i] != 0:
                f = A[r][i] / A[i][i]
                A[r] = [x - f * y for x, y in zip(A[r], A[i])]
    return [A[i][3] / A[i][i] for i in range(n)]


def _beta_exact(avgs5, s):
    centres = [Fr(j) for j in range(s - 2, s + 1)]   # s = 0, 1, 2
    a, b, c = _quad_from_avgs(centres, avgs5[s:s + 3])
    # p' = b + 2 c x, p'' = 2c ; integrate over [-1/2, 1/2]
    int_p1sq = b * b + Fr(4) * c * c / 12          # integral of (b + 2cx)^2
    int_p2sq = 4 * c * c
    return int_p1sq + int_p2sq


@pytest.mark.parametrize("seed", range(30))
def test_beta_matches_integral_definition(oracle, seed):
    rng = np.random.default_rng(200 + seed)
    q = [Fr(int(v), 8) for v in rng.integers(-40, 40, 5)]
    b = oracle.weno5_beta([float(v) for v in q])
    for s in range(3):
        ex = float(_beta_exact(q, s))
        assert abs(b[s] - ex) <= 1e-13 * max(1.0, abs(ex)), (s, b[s], ex)


def _js_limit(beta, d, eps):
    a = [Fr(dk) / (Fr(bk) + eps) ** 2 for bk, dk in zip(beta, d)]
    s = sum(a)
    return [float(x / s) for x in a]


@pytest.mark.parametrize("seed", range(40))
def test_wenow_is_js_limit(oracle, seed):
    """Eq. (15) equals the epsilon -> 0 limit of the WENO-JS weights (with
    exponent 2), including indicator sets with exact zeros."""
    rng = np.random.default_rng(300 + seed)
    beta = [float(v) for v in rng.integers(0, 5, 3) * rng.random(3)]
    if seed % 4 == 0:
        beta[rng.integers(0, 3)] = 0.0
    if seed % 8 == 1:
        beta = [0.0, 0.0, float(rng.random())]
    if seed == 2:
        beta = [0.0, 0.0, 0.0]
    dl, dr = oracle.weno5_ideal()
    for d in (dl, dr):
        w = oracle.wenow_weights(beta, d)
        ref = _js_limit([Fr(b) for b in beta], [Fr(x) for x in d], Fr(1, 10 ** 60))
        assert np.allclose(w, ref, rtol=0, atol=1e-14), (beta, w, ref)
        assert abs(w.sum() - 1.0) < 1e-15 and (w >= 0).all()


@pytest.mark.parametrize("a", [1.204e-3, 1e-9, 3.7, 1e6])
def test_wenow_affine_invariance(oracle, a):
    """Sec. 3.3: with g = a f + b the weights are unchanged, so
    g^L = a f^L + b whatever a is (the property WENO-JS lacks)."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        f = rng.random(5)
        f[rng.integers(0, 5):] += 1.0           # a jump somewhere
        b = rng.normal()
        fl, fr = oracle.weno5w(f)
        gl, gr = oracle.weno5w(a * f + b)
        sc = abs(a) * 2 + abs(b)
        assert abs(gl - (a * fl + b)) < 1e-14 * sc
        assert abs(gr - (a * fr + b)) < 1e-14 * sc


def test_wenojs_loses_affine_invariance(oracle):
    """Sec. 3.2: for g = rho_1 alpha with rho_1 = 1.204e-3 WENO-JS sees
    eps/rho_1^2 = 0.6898, not eps, and keeps a non-smooth stencil."""
    g = GOLD["wenojs_eps_over_rho1_sq"]
    assert abs(g["eps"] / g["rho1"] ** 2 - g["value"]) < 5e-5
    f = np.array([0.0, 0.0, 0.0, 1.0, 1.0])      # an interface in alpha
    beta_f = oracle.weno5_beta(f)
    beta_g = oracle.weno5_beta(g["rho1"] * f)
    dl, _ = oracle.weno5_ideal()
    w_f = oracle.wenojs_weights(beta_f, dl, g["eps"])
    w_g = oracle.wenojs_weights(beta_g, dl, g["eps"])
    # JS with the scaled function gives substantial weight to the stencils
    # crossing the jump, unlike the unscaled one
    assert w_f[0] > 0.99 and w_g[0] < 0.9
    # WENO-W gives the same weights for both
    assert np.array_equal(oracle.wenow_weights(beta_f, dl),
                          oracle.wenow_weights(beta_g, dl))


def test_gl_interior_from_quartic(oracle):
    """Eq. (22) quartic: its averages over cells i-1, i, i+1 and its end values
    determine it; the interior Gauss-Lobatto nodes +-sqrt(5)/10 carry weights
    5/12 (the end weights are 1/12, Sec. 4.2), so f^C of Eq. (6) inverted is
    the mean of the quartic at those nodes.  Checked in exact rationals."""
    rng = np.random.default_rng(11)
    g = GOLD["gauss_lobatto_end_weight"]
    w1 = Fr(g["value_num"], g["value_den"])
    for _ in range(20):
        co = [Fr(int(v), 9) for v in rng.integers(-30, 30, 5)]
        ub = _poly_cell_avgs(co, [Fr(-1), Fr(0), Fr(1)])
        uL, uR = _peval(co, Fr(1, 2)), _peval(co, Fr(-1, 2))
        # the paper's B coefficients (Eq. (22), dx = 1) recover the quartic
        B0 = ((ub[2] + 298 * ub[1] + ub[0]) - 54 * (uL + uR)) / 192
        B1 = -((ub[2] - ub[0]) + 10 * (uR - uL)) / 8
        B2 = -((ub[2] + 58 * ub[1] + ub[0]) - 30 * (uL + uR)) / 8
        B3 = ((ub[2] - ub[0]) + 2 * (uR - uL)) / 2
        B4 = Fr(5, 12) * ((ub[2] + 10 * ub[1] + ub[0]) - 6 * (uL + uR))
        assert [B0, B1, B2, B3, B4] == co
        # p(a) + p(-a) with a^2 = 1/20 is rational
        a2 = Fr(1, 20)
        mean_int = co[0] + co[2] * a2 + co[4] * a2 * a2
        quad = w1 * uR + w1 * uL + (1 - 2 * w1) * mean_int
        assert quad == ub[1]                      # Eq. (6) holds exactly
        fc = oracle.gl_interior(float(ub[1]), float(uL), float(uR))
        assert abs(fc - float(mean_int)) < 1e-13 * (1 + abs(float(mean_int)))
