"""Pins of the input generators: the Rankine-Hugoniot seeding against the
post-shock states printed in the paper, and the batched parameter draw."""
import json
import os

import numpy as np

from paper_2608_00746_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_values.json")))


def test_cavity_post_shock_state():
    """Sec. 4.2.1, Eq. (32): (rho, u) = (1.325, 68.52) behind a Mach 1.72
    shock in water with P = 1.915e4."""
    g = GOLD["cavity_post_shock"]
    rho1, u1, S = I.rh_post_shock(g["gamma"], g["pinf"], g["rho0"], g["p0"], g["p1"])
    c0 = np.sqrt(g["gamma"] * (g["p0"] + g["pinf"]) / g["rho0"])
    assert abs(rho1 - g["rho1"]) < 5e-4 * g["rho1"]
    assert abs(u1 - g["u1"]) < 5e-4 * g["u1"]
    assert abs(S / c0 - g["mach"]) < 5e-3


def test_vessel_post_shock_state():
    """Sec. 4.2.2, Eq. (33): gelatin behind a 40 MPa shock moving to -x,
    (rho, u) = (1046.0, -24.2) as printed (to the printed digits)."""
    g = GOLD["vessel_post_shock"]
    rho1, u1, S = I.rh_post_shock(g["gamma"], g["pinf"], g["rho0"], g["p0"], g["p1"],
                                  direction=-1)
    assert abs(rho1 - g["rho1"]) < 5e-4 * g["rho1"]
    assert abs(u1 - g["u1"]) < 0.05
    assert S < 0


def test_batched_draw():
    n, N, r, Ps = I.batched_draw(0)
    assert len(n) == 256 and n.min() >= 64 and n.max() <= 512
    assert set(np.unique(N)) <= {2, 3}
    assert (r >= 0.05).all() and (r <= 0.2).all() and (Ps >= 1e8).all() and (Ps <= 2e9).all()
    assert int((n.astype(np.int64) ** 2).sum()) == 27238496


def test_conserved_states_admissible():
    for w in (I.advection_1d(50), I.shock_bubble_2d(64, 32), I.shock_interface_n3(32),
              I.paper_five_phase(20), I.batched_instance(70, 3, 0.1, 1e9)):
        U = w.U.reshape(w.nU, -1)
        a = U[-w.N:]
        assert np.abs(a.sum(0) - 1).max() < 1e-15
        assert (a >= 0).all() and (a <= 1).all() and (U[:w.N] >= 0).all()
