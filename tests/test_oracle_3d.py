"""The oracle in 3D (the z sweep of the shock-vessel-bubble problem,
Sec. "Shock-vessel-bubble interaction"), pinned by two exact reductions:

* a 3D grid with one periodic cell along z is the 2D problem: the z
  stencil is constant, its fluxes cancel exactly, and L(U) of every 2D
  component equals the 2D L(U) bit for bit (the z momentum's L is zero);
* permuting the axes of a state on a cubic grid permutes L(U): an index or
  stride slip in one direction breaks it (to round-off: the directions are
  summed in another order).
"""
import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I
from conftest import oracle_problem


def as_3d(w):
    """w (2D) on a grid with one periodic cell along z and zero z momentum."""
    N = w.N
    U2 = w.U                                   # (nU2, ny, nx)
    U3 = np.zeros((w.nU + 1, 1) + U2.shape[1:])
    U3[:N + 2, 0] = U2[:N + 2]                 # masses, x and y momenta
    U3[N + 3:, 0] = U2[N + 2:]                 # energy, volume fractions
    w3 = w.copy()
    w3.ndim = 3
    w3.n = tuple(w.n) + (1,)
    w3.dx = tuple(w.dx) + (w.dx[0],)
    w3.bc = tuple(w.bc) + ((I.BC_PERIODIC, I.BC_PERIODIC),)
    w3.U = U3
    return w3


@pytest.mark.parametrize("N,seed", [(1, 1), (2, 2), (3, 3)])
@pytest.mark.parametrize("flux", [I.FLUX_HLLC, I.FLUX_HLL])
def test_3d_with_one_z_cell_is_2d(oracle, N, seed, flux):
    w = I.random_state((14, 11), nphase=N, seed=seed, lowp=0.0)
    w.bc = ((I.BC_PERIODIC, I.BC_PERIODIC), (I.BC_OUTFLOW, I.BC_SYMMETRY))
    w.opts.flux = flux
    w3 = as_3d(w)
    L2 = oracle_problem(oracle, w).rhs(w.U.reshape(-1)).reshape(w.nU, -1)
    L3 = oracle_problem(oracle, w3).rhs(w3.U.reshape(-1)).reshape(w3.nU, -1)
    keep = [c for c in range(w3.nU) if c != N + 2]
    assert np.array_equal(L3[keep], L2)
    assert np.all(L3[N + 2] == 0.0)


def test_3d_axis_permutation(oracle):
    """A state on an 8 x 8 x 8 cube with outflow ends, rotated so that
    (x, y, z) -> (y, z, x): L(U) rotates with it to round-off."""
    w = I.shock_vessel_bubble_3d(8, 8, 8)
    w.dx = (w.dx[1],) * 3
    w.bc = ((I.BC_OUTFLOW, I.BC_OUTFLOW),) * 3
    N = w.N
    L = oracle_problem(oracle, w).rhs(w.U.reshape(-1)).reshape(w.U.shape)
    # U[c, z, y, x] -> V[c, x, z, y]: new (x', y', z') = (y, z, x)
    V = np.transpose(w.U, (0, 3, 1, 2)).copy()
    mom = V[N:N + 3].copy()
    V[N + 0], V[N + 1], V[N + 2] = mom[1], mom[2], mom[0]
    wr = w.copy()
    wr.U = V
    Lr = oracle_problem(oracle, wr).rhs(V.reshape(-1)).reshape(V.shape)
    Lb = np.transpose(Lr, (0, 2, 3, 1)).copy()        # back to [c, z, y, x]
    mb = Lb[N:N + 3].copy()
    Lb[N + 0], Lb[N + 1], Lb[N + 2] = mb[2], mb[0], mb[1]
    sc = np.abs(L).reshape(w.nU, -1).max(axis=1)
    err = np.abs(Lb - L).reshape(w.nU, -1).max(axis=1) / np.where(sc > 0, sc, 1)
    print("axis permutation rel err", np.array2string(err, precision=2))
    assert np.isfinite(L).all() and (sc > 0).all()
    assert (err <= 1e-12).all(), err
