"""The oracle's Phase-Field step in 3D (the shock-vessel-bubble problem runs
it, Sec. 4.2.2), pinned by the two exact reductions that pin its 3D
hyperbolic step:

* a 3D grid with one periodic cell along z is the 2D problem: the z
  Laplacian of phi and the z faces of Eq. (4) vanish, so [div J_p], the
  face gradients of x and y, L^PF and the step equal the 2D ones (to
  rounding: the multiplier integrals carry another cell volume), and the z
  gradients and the z momentum's L^PF are zero;
* permuting the axes of a state on a grid with equal spacings permutes
  [div J_p], the face gradients (direction with the axes) and L^PF (the
  momentum components with the axes): an index or stride slip in one
  direction breaks it (to round-off, amplified for the gradients by the
  conditioning of Eq. (4): the directions are summed in another order, and
  Eq. (4) is solved in another cell order).
"""
import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I
from conftest import oracle_problem
from test_oracle_3d import as_3d


def _parts(pb, U, eta, dt):
    divj, info = pb.pf_divj(U, eta)
    G, res = pb.pf_gradients(U, divj)
    K = pb.pf_k(U)
    L = pb.pf_rhs(U, G, K)
    U1, _ = pb.pf_step(U, dt, eta)
    return divj, G, L, U1


@pytest.mark.parametrize("N", [2, 3])
def test_pf_3d_with_one_z_cell_is_2d(oracle, N):
    w = I.pf_bubble((20, 16), N, width=1.5)
    w.bc = ((I.BC_PERIODIC, I.BC_PERIODIC), (I.BC_OUTFLOW, I.BC_OUTFLOW))
    w3 = as_3d(w)
    eta, dt = w.dx[0], 2e-4
    d2, G2, L2, U2 = _parts(oracle_problem(oracle, w), w.U.reshape(-1), eta, dt)
    d3, G3, L3, U3 = _parts(oracle_problem(oracle, w3), w3.U.reshape(-1), eta, dt)
    # the integrals of Eq. (28) carry the cell volume dx dy dz instead of
    # dx dy: the multipliers agree to rounding
    assert np.abs(d3 - d2).max() <= 1e-12 * np.abs(d2).max()
    # Eq. (4) is the same linear system with a right side that differs by
    # rounding; its conditioning (k from 1e-6 to 1/4) amplifies that, so
    # the gradients, and L^PF through them, are held to the Phase-Field bar
    # of the GPU parity, 1e-9 of their maximum
    gs = np.abs(G2).max()
    assert np.abs(G3[:2] - G2).max() <= 1e-9 * gs
    assert np.all(G3[2] == 0.0)
    L3 = L3.reshape(w3.nU, -1)
    U3 = U3.reshape(w3.nU, -1)
    keep = [c for c in range(w3.nU) if c != N + 2]
    Ls = np.abs(L2.reshape(w.nU, -1)).max(axis=1, keepdims=True)
    assert (np.abs(L3[keep] - L2.reshape(w.nU, -1)) <= 1e-9 * np.maximum(Ls, 1e-300)).all()
    assert np.all(L3[N + 2] == 0.0)
    Us = np.abs(U2.reshape(w.nU, -1)).max(axis=1, keepdims=True)
    assert (np.abs(U3[keep] - U2.reshape(w.nU, -1)) <= 1e-13 * Us).all()


def _rotate(A, N, mom_axis0):
    """[c, z, y, x] -> [c, x, z, y] (new (x', y', z') = (y, z, x)); the
    momentum components, from index mom_axis0 on, follow."""
    V = np.transpose(A, (0, 3, 1, 2)).copy()
    m = V[mom_axis0:mom_axis0 + 3].copy()
    V[mom_axis0 + 0], V[mom_axis0 + 1], V[mom_axis0 + 2] = m[1], m[2], m[0]
    return V


def test_pf_3d_axis_permutation(oracle):
    N = 3
    w = I.pf_bubble((12, 10, 8), N, width=1.5)
    w.bc = ((I.BC_OUTFLOW, I.BC_OUTFLOW), (I.BC_PERIODIC, I.BC_PERIODIC),
            (I.BC_OUTFLOW, I.BC_OUTFLOW))
    # an off-centre ball, so that no mirror symmetry hides a slip
    U = w.U.copy()
    U = np.roll(U, (1, 2, 3), axis=(1, 2, 3))
    w.U = U
    eta = w.dx[0]
    pb = oracle_problem(oracle, w)
    divj, _ = pb.pf_divj(U.reshape(-1), eta)
    G, _ = pb.pf_gradients(U.reshape(-1), divj)
    K = pb.pf_k(U.reshape(-1))
    L = pb.pf_rhs(U.reshape(-1), G, K).reshape(U.shape)

    V = _rotate(U, N, N)
    wr = w.copy()
    wr.U = V
    wr.n = (w.n[1], w.n[2], w.n[0])
    wr.bc = (w.bc[1], w.bc[2], w.bc[0])
    pr = oracle_problem(oracle, wr)
    dr, _ = pr.pf_divj(V.reshape(-1), eta)
    Gr, _ = pr.pf_gradients(V.reshape(-1), dr)
    Kr = pr.pf_k(V.reshape(-1))
    Lr = pr.pf_rhs(V.reshape(-1), Gr, Kr).reshape(V.shape)

    sh = U.shape[1:]
    shr = V.shape[1:]
    back = lambda a: np.transpose(a.reshape(shr), (1, 2, 0))     # [x, z, y] -> [z, y, x]
    db = np.stack([back(dr[p]) for p in range(N)])
    assert np.abs(db - divj.reshape((N,) + sh)).max() <= 1e-12 * np.abs(divj).max()
    # gradient directions: new x' = old y, y' = old z, z' = old x
    Gb = np.stack([np.stack([back(Gr[(d + 2) % 3, p]) for p in range(N)]) for d in range(3)])
    gs = np.abs(G).max()
    assert np.abs(Gb - G.reshape((3, N) + sh)).max() <= 1e-9 * gs
    Lb = np.transpose(Lr, (0, 2, 3, 1)).copy()
    mb = Lb[N:N + 3].copy()
    Lb[N + 0], Lb[N + 1], Lb[N + 2] = mb[2], mb[0], mb[1]
    sc = np.abs(L).reshape(w.nU, -1).max(axis=1)
    err = np.abs(Lb - L).reshape(w.nU, -1).max(axis=1) / np.where(sc > 0, sc, 1)
    print("PF axis permutation rel err", np.array2string(err, precision=2))
    assert np.isfinite(L).all() and (sc[:N] > 0).all()
    assert (err <= 1e-9).all(), err
