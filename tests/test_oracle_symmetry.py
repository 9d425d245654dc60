"""Symmetry planes in the oracle, pinned by a mirrored periodic domain.

At a symmetry plane the ghost cells are the mirror images of the interior
cells with the normal momentum negated (the shock-vessel-bubble problem of
Sec. "Shock-vessel-bubble interaction" computes a quarter of the domain
between two such planes).  A periodic line of 2n cells whose second half
is the mirror image of the first (normal momentum negated) is symmetric
about both ends of the first half, so every stencil of the first half holds
exactly the values the half line with symmetry planes at both ends builds
from its ghosts: L(U) of the half must equal the first half of L(U) of the
periodic line bit for bit.  A sign slip in the flip, an off-by-one mirror or
a ghost taken from the wrong end breaks the equality.
"""
import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I
from conftest import oracle_problem


def mirrored_pair(w, d):
    """(half workload with symmetry planes along d, periodic full workload)."""
    N = w.N
    ax = w.U.ndim - 1 - d
    flip = np.flip(w.U, axis=ax).copy()
    flip[N + d] *= -1.0
    full = w.copy()
    full.U = np.concatenate([w.U, flip], axis=ax)
    n = list(w.n)
    n[d] *= 2
    full.n = tuple(n)
    bc = [tuple(b) for b in w.bc]
    bc[d] = (I.BC_PERIODIC, I.BC_PERIODIC)
    full.bc = tuple(bc)
    half = w.copy()
    bc = [tuple(b) for b in w.bc]
    bc[d] = (I.BC_SYMMETRY, I.BC_SYMMETRY)
    half.bc = tuple(bc)
    return half, full


CASES = [
    (lambda: I.random_state((24,), nphase=2, seed=3, lowp=0.0), 0),
    (lambda: I.random_state((19,), nphase=3, seed=4, lowp=0.0), 0),
    (lambda: I.random_state((12, 10), nphase=2, seed=5, lowp=0.0), 0),
    (lambda: I.random_state((12, 10), nphase=3, seed=6, lowp=0.0), 1),
    (lambda: I.random_state((3,), nphase=2, seed=7, lowp=0.0), 0),
]


@pytest.mark.parametrize("make,d", CASES)
@pytest.mark.parametrize("flux", [I.FLUX_HLLC, I.FLUX_HLL])
def test_symmetry_equals_mirrored_periodic(oracle, make, d, flux):
    w = make()
    w.opts.flux = flux
    half, full = mirrored_pair(w, d)
    Lh = oracle_problem(oracle, half).rhs(half.U.reshape(-1)).reshape(half.U.shape)
    Lf = oracle_problem(oracle, full).rhs(full.U.reshape(-1)).reshape(full.U.shape)
    ax = w.U.ndim - 1 - d
    first = np.take(Lf, np.arange(w.n[d]), axis=ax)
    assert np.isfinite(Lh).all()
    assert np.array_equal(Lh, first)


def test_symmetry_plane_carries_no_mass(oracle):
    """A state at rest next to the plane with a pressure jump: the mass of
    every phase is conserved exactly up to summation order (no flux through
    the plane), while an outflow end lets the wave out."""
    w = I.random_state((32,), nphase=2, seed=9, lowp=0.0)
    w.bc = ((I.BC_SYMMETRY, I.BC_SYMMETRY),)
    pb = oracle_problem(oracle, w)
    L = pb.rhs(w.U.reshape(-1)).reshape(w.nU, -1)
    scale = np.abs(L[:2]).max()
    for p in range(2):
        assert abs(L[p].sum()) <= 1e-13 * scale * w.n[0]
    with pytest.raises(Exception):
        bad = w.copy()
        bad.bc = ((I.BC_PERIODIC, I.BC_SYMMETRY),)
        oracle_problem(oracle, bad).rhs(bad.U.reshape(-1))
