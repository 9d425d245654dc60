"""Two-level coupling of uniform grids (block-structured refinement by 2,
Sec. 3.4.2), written plainly on top of the oracle's operators.

TEST INFRASTRUCTURE ONLY: the reference the GPU coupling is checked
against.  Only the tests may import it.

Definition (one SSP-RK3 step of a coarse grid C and fine blocks F, all
with the same dt):
* a block covers the coarse cells [lo, lo + W) (x) [lo_y, lo_y + H); its
  grid is the block refined by 2 plus a ring of 3 ghost cells;
* before each RK stage the ring takes, cell by cell, the coarse parent's
  average of the stage state (piecewise-constant prolongation);
* each level's stage is the oracle's L(U) of that level (the ring is part of
  the fine grid, so the stencils of fine cells next to the block edge reach
  into it);
* at each coarse face of the block boundary the coarse flux (from the coarse
  cells' reconstructions) and the fine fluxes of its two sub-faces (from the
  fine cells') give the correction of the outside coarse cell's L: the fine
  minus the coarse flux over the coarse width, and for alpha_p the source
  alpha_p (1 + K_p) on the face-velocity difference; it is summed over the
  stages with the RK3 weights 1/6, 1/6, 2/3;
* after the step the coarse cells under a block take the mean of their
  children, the outside cells add dt times the summed correction, and the
  rings take the new coarse values (so that they hold admissible data
  between steps).
"""
from __future__ import annotations

import numpy as np

HALO = 3
WEIGHTS = (1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0)


class Block:
    def __init__(self, lo, W, H=1):
        self.lo = tuple(lo)
        self.W, self.H = W, H


def _grid(U, pb):
    """(nU, ny, nx) view of a state vector (1D: ny = 1)."""
    nx = pb.shape[0]
    ny = pb.shape[1] if pb.ndim > 1 else 1
    return U.reshape(pb.nU, ny, nx)


def prolong(pbc, pbf, Uc, Uf, blk):
    """Ring cells of the fine grid <- their coarse parents' values."""
    C, F = _grid(Uc, pbc), _grid(Uf, pbf).copy()
    nfy, nfx = F.shape[1], F.shape[2]
    for fy in range(nfy):
        for fx in range(nfx):
            inx = HALO <= fx < nfx - HALO
            iny = pbf.ndim == 1 or HALO <= fy < nfy - HALO
            if inx and iny:
                continue
            cx = blk.lo[0] + (fx - HALO) // 2
            cy = 0 if pbf.ndim == 1 else blk.lo[1] + (fy - HALO) // 2
            F[:, fy, fx] = C[:, cy, cx]
    return F.reshape(-1)


def faces(pbc, blk):
    """Coarse faces of the block boundary: (dir, minus cell, plus cell,
    outside-is-minus, [fine minus cells of the sub-faces])."""
    out = []
    W, H, (lx, *rest) = blk.W, blk.H, blk.lo
    ly = rest[0] if pbc.ndim > 1 else 0
    one = pbc.ndim == 1
    for J in range(H):
        for left in (True, False):
            xm = lx - 1 if left else lx + W - 1
            fxm = HALO - 1 if left else HALO + 2 * W - 1
            sub = [(fxm, 0)] if one else [(fxm, HALO + 2 * J + k) for k in (0, 1)]
            out.append((0, (xm, ly + J), (xm + 1, ly + J), left, sub))
    if not one:
        for I in range(W):
            for bot in (True, False):
                ym = ly - 1 if bot else ly + H - 1
                fym = HALO - 1 if bot else HALO + 2 * H - 1
                sub = [(HALO + 2 * I + k, fym) for k in (0, 1)]
                out.append((1, (lx + I, ym), (lx + I, ym + 1), bot, sub))
    return out


def face_flux(pb, G, d, cm):
    """Numerical flux (and u-hat) at the face between cell cm and its plus
    neighbour along d, from the two cells' reconstructions."""
    x, y = cm
    cells = []
    for j in range(-2, 4):
        cx, cy = (x + j, y) if d == 0 else (x, y + j)
        cells.append(G[:, cy, cx])
    S = np.array(cells)
    UL, _, VL, _, _ = pb.reconstruct_cell(S[0:5], d)      # minus cell: its plus face
    _, UR, _, VR, _ = pb.reconstruct_cell(S[1:6], d)      # plus cell: its minus face
    return pb.flux(UL, VL, UR, VR, d)


def stage_correction(pbc, pbf, Uc, Uf, blk, alpha_source=0):
    """Correction of the outside coarse cells' L at one stage state:
    {(x, y): dL}."""
    N, nd = pbc.N, pbc.ndim
    Gc, Gf = _grid(Uc, pbc), _grid(Uf, pbf)
    out = {}
    for d, cm, cp, out_minus, sub in faces(pbc, blk):
        Fc, uc = face_flux(pbc, Gc, d, cm)
        fl = [face_flux(pbf, Gf, d, s) for s in sub]
        Ff = sum(f[0] for f in fl) / len(fl)
        uf = sum(f[1] for f in fl) / len(fl)
        sg = -1.0 if out_minus else 1.0
        rd = 1.0 / pbc.dx[d]
        dL = sg * (Ff - Fc) * rd
        du = sg * (uf - uc) * rd
        o = cm if out_minus else cp
        ub = Gc[:, o[1], o[0]]
        a = ub[N + nd + 1:]
        S = a.sum()
        for p in range(N):
            ap = a[p] / S if (alpha_source and S > 0.0) else (0.0 if alpha_source else a[p])
            dL[N + nd + 1 + p] -= ap * pbc.one_plus_K(ub, p) * du
        out[o] = out.get(o, 0.0) + dL
    return out


def restrict(pbc, pbf, Uc, Uf, blk):
    C, F = _grid(Uc, pbc).copy(), _grid(Uf, pbf)
    lx = blk.lo[0]
    ly = blk.lo[1] if pbc.ndim > 1 else 0
    for J in range(blk.H):
        for I in range(blk.W):
            fx = HALO + 2 * I
            if pbc.ndim == 1:
                C[:, 0, lx + I] = 0.5 * (F[:, 0, fx] + F[:, 0, fx + 1])
            else:
                fy = HALO + 2 * J
                C[:, ly + J, lx + I] = 0.25 * ((F[:, fy, fx] + F[:, fy, fx + 1]) +
                                              (F[:, fy + 1, fx] + F[:, fy + 1, fx + 1]))
    return C.reshape(-1)


def composite_step(pbc, pbfs, Uc, Ufs, blocks, dt, alpha_source=0):
    """One SSP-RK3 step of the coarse grid and its blocks (lists pbfs, Ufs,
    blocks)."""
    def rk(U, L, s, Un):
        if s == 0:
            return U + dt * L
        if s == 1:
            return 0.75 * Un + 0.25 * (U + dt * L)
        return Un / 3.0 + 2.0 / 3.0 * (U + dt * L)

    Ucs, Ufs_s = Uc.copy(), [u.copy() for u in Ufs]
    corr = [dict() for _ in blocks]
    for s in range(3):
        Ufs_s = [prolong(pbc, pbf, Ucs, Uf, b) for pbf, Uf, b in zip(pbfs, Ufs_s, blocks)]
        if s == 0:
            Ufs = [u.copy() for u in Ufs_s]          # the step-start fine states, ring filled
        for k, (pbf, Uf, b) in enumerate(zip(pbfs, Ufs_s, blocks)):
            for o, dL in stage_correction(pbc, pbf, Ucs, Uf, b, alpha_source).items():
                corr[k][o] = corr[k].get(o, 0.0) + WEIGHTS[s] * dL
        Lc = pbc.rhs(Ucs)
        Lfs = [pbf.rhs(u) for pbf, u in zip(pbfs, Ufs_s)]
        Ucs = rk(Ucs, Lc, s, Uc)
        Ufs_s = [rk(u, L, s, un) for u, L, un in zip(Ufs_s, Lfs, Ufs)]
    for pbf, Uf, b in zip(pbfs, Ufs_s, blocks):
        Ucs = restrict(pbc, pbf, Ucs, Uf, b)
    G = _grid(Ucs, pbc).copy()
    for cmap in corr:
        for (x, y), dL in cmap.items():
            G[:, y, x] += dt * dL
    Uc_new = G.reshape(-1)
    # the rings take the new coarse values between steps
    Ufs_s = [prolong(pbc, pbf, Uc_new, Uf, b) for pbf, Uf, b in zip(pbfs, Ufs_s, blocks)]
    return Uc_new, Ufs_s


def composite_totals(pbc, pbfs, Uc, Ufs, blocks):
    """Sum of U times the cell volume over the coarse cells outside the
    blocks and the fine cells inside them (ring excluded)."""
    C = _grid(Uc, pbc)
    mask = np.ones(C.shape[1:], dtype=bool)
    tot = np.zeros(pbc.nU)
    for pbf, Uf, b in zip(pbfs, Ufs, blocks):
        lx = b.lo[0]
        ly = b.lo[1] if pbc.ndim > 1 else 0
        mask[ly:ly + b.H, lx:lx + b.W] = False
        F = _grid(Uf, pbf)
        inner = F[:, (HALO if pbf.ndim > 1 else 0):F.shape[1] - (HALO if pbf.ndim > 1 else 0),
                  HALO:F.shape[2] - HALO]
        tot += inner.reshape(pbc.nU, -1).sum(axis=1) * float(np.prod(pbf.dx))
    tot += C[:, mask].sum(axis=1) * float(np.prod(pbc.dx))
    return tot
