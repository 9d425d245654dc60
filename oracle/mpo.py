"""ctypes wrapper of the FP64 CPU oracle (oracle/mpo.c).

TEST INFRASTRUCTURE ONLY: the slow, plain reference the HIP path is checked
against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It imports nothing from the product
package and the product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpo.so")
MAXP = 8
# floor of the coefficient k = phi (1 - phi) of Eq. (4) (reading): with it
# the equation joins all cells and is solvable for every right side of zero
# total, and its condition number stays bounded; it changes k only where
# phi < 1e-6 or 1 - phi < 1e-6
PF_KFLOOR = 1e-6
# the Phase-Field step's own CFL bound (reading): |G_d| dt / dx_d <= 1/12, the
# sufficient bound of the Gauss-Lobatto argument (end weight 1/12).  The
# solve's gradient is clipped there; that happens only in nearly pure cells,
# where Eq. (4) would carry volume between separate interfaces through a
# medium of conductivity ~ PF_KFLOOR and the capped flux is negligible.
PF_CFL = 1.0 / 12.0

BC_PERIODIC, BC_OUTFLOW, BC_SYMMETRY = 0, 1, 2
RECON_WENO_C, RECON_WENO_CL, RECON_WENO_JS, RECON_WENO_W = 0, 1, 2, 3
SRC_CELL, SRC_NORMALIZED = 0, 1
FLUX_HLLC, FLUX_HLL = 0, 1
MODEL_ALLAIRE, MODEL_KAPILA = 0, 1


def build(verbose: bool = False) -> str:
    """Compile libmpo.so with gcc (plain C99, OpenMP, no FP contraction)."""
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", LIB_PATH,
           os.path.join(HERE, "mpo.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB_PATH


class _Problem(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3),
        ("bc", (C.c_int * 2) * 3), ("nphase", C.c_int),
        ("gamma", C.c_double * MAXP), ("pinf", C.c_double * MAXP),
        ("D", C.c_double * MAXP), ("pmin", C.c_double * MAXP),
        ("cT", C.c_double * MAXP), ("recon", C.c_int), ("flux", C.c_int),
        ("model", C.c_int), ("energy_limiter", C.c_int), ("cfl", C.c_double),
        ("t_end", C.c_double), ("alpha_source", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(_Problem)
        L.mpo_rhs.argtypes = [pp, dp, dp]
        L.mpo_step.argtypes = [pp, dp, C.c_double]
        L.mpo_dt.argtypes = [pp, dp, C.c_double]
        L.mpo_dt.restype = C.c_double
        L.mpo_diag.argtypes = [pp, dp, dp]
        L.mpo_weno5_beta.argtypes = [dp, dp]
        L.mpo_weno5_candidates.argtypes = [dp, dp, dp]
        L.mpo_weno5_ideal.argtypes = [dp, dp]
        L.mpo_weno5_increments.argtypes = [dp, dp, dp]
        L.mpo_wenow_weights.argtypes = [dp, dp, dp]
        L.mpo_wenojs_weights.argtypes = [dp, dp, C.c_double, dp]
        L.mpo_weno5w.argtypes = [dp, dp, dp]
        L.mpo_pressure.argtypes = [pp, dp, C.c_int, dp]
        L.mpo_pressure.restype = C.c_double
        L.mpo_sound_speed.argtypes = [pp, dp, dp, C.c_double]
        L.mpo_sound_speed.restype = C.c_double
        L.mpo_psi.argtypes = [pp, dp]
        L.mpo_psi.restype = C.c_double
        L.mpo_temperature.argtypes = [pp, dp, C.c_int]
        L.mpo_temperature.restype = C.c_double
        L.mpo_reconstruct_cell.argtypes = [pp, dp, C.c_int, dp, dp, dp, dp, dp]
        L.mpo_flux.argtypes = [pp, C.c_int, dp, dp, dp, dp, dp, dp]
        L.mpo_gl_interior.argtypes = [C.c_double] * 3
        L.mpo_gl_interior.restype = C.c_double
        L.mpo_pf_gprime.argtypes = [C.c_double]
        L.mpo_pf_gprime.restype = C.c_double
        L.mpo_pf_divj.argtypes = [pp, dp, C.c_double, dp, dp]
        L.mpo_pf_flux.argtypes = [pp, C.c_int, dp, dp, dp, dp, dp]
        L.mpo_pf_rhs.argtypes = [pp, dp, dp, dp, dp]
        L.mpo_pf_rk3.argtypes = [pp, dp, dp, dp, C.c_double]
        L.mpo_one_plus_K.argtypes = [pp, dp, C.c_int]
        L.mpo_one_plus_K.restype = C.c_double
        L.mpo_num_threads.restype = C.c_int
        L.mpo_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


class Problem:
    """Grid, boundary conditions, per-phase EOS and scheme switches."""

    def __init__(self, ndim, n, dx, bc, gamma, pinf, D=None, pmin=None,
                 cT=None, recon=RECON_WENO_C, flux=FLUX_HLLC,
                 model=MODEL_ALLAIRE, energy_limiter=1, cfl=0.5, t_end=0.0,
                 alpha_source=SRC_CELL):
        N = len(gamma)
        assert 1 <= N <= MAXP
        p = _Problem()
        p.ndim = ndim
        nn = list(n) + [1] * (3 - len(n))
        dd = list(dx) + [1.0] * (3 - len(dx))
        for k in range(3):
            p.n[k] = int(nn[k])
            p.dx[k] = float(dd[k])
        bcl = list(bc) + [(0, 0)] * (3 - len(bc))
        for k in range(3):
            p.bc[k][0] = int(bcl[k][0])
            p.bc[k][1] = int(bcl[k][1])
        p.nphase = N
        z = [0.0] * N
        for name, vals in (("gamma", gamma), ("pinf", pinf), ("D", D or z),
                           ("pmin", pmin if pmin is not None else z),
                           ("cT", cT if cT is not None else z)):
            arr = getattr(p, name)
            for k in range(N):
                arr[k] = float(vals[k])
        p.recon, p.flux, p.model = int(recon), int(flux), int(model)
        p.energy_limiter = int(energy_limiter)
        p.cfl = float(cfl)
        p.t_end = float(t_end)
        p.alpha_source = int(alpha_source)
        self._p = p
        self.ndim, self.N = ndim, N
        self.dx = tuple(float(dd[k]) for k in range(ndim))
        self.bc = tuple((int(bcl[k][0]), int(bcl[k][1])) for k in range(ndim))
        self.nU = 2 * N + ndim + 1
        self.shape = tuple(int(nn[k]) for k in range(ndim))

    @property
    def ncells(self):
        return int(np.prod(self.shape))

    def ref(self):
        return C.byref(self._p)

    # ---- whole-grid operators ------------------------------------------
    def rhs(self, U):
        U = _arr(U, self.nU * self.ncells)
        L = np.empty_like(U)
        st = lib().mpo_rhs(self.ref(), _ptr(U), _ptr(L))
        if st != 0:
            raise RuntimeError(f"mpo_rhs status {st}")
        return L

    def step(self, U, dt):
        U = _arr(U, self.nU * self.ncells).copy()
        st = lib().mpo_step(self.ref(), _ptr(U), float(dt))
        if st != 0:
            raise RuntimeError(f"mpo_step status {st}")
        return U

    def dt(self, U, t=0.0):
        U = _arr(U, self.nU * self.ncells)
        return lib().mpo_dt(self.ref(), _ptr(U), float(t))

    def diag(self, U):
        U = _arr(U, self.nU * self.ncells)
        out = np.zeros(self.nU + 6)
        lib().mpo_diag(self.ref(), _ptr(U), _ptr(out))
        return out

    # ---- Phase-Field step ----------------------------------------------
    def pf_divj(self, U, eta):
        """[div J_p] of Eq. (28) on the volume fractions of U: (N, ncells)
        and info = (M, number of present phases, B_1..B_N)."""
        U = _arr(U, self.nU * self.ncells)
        out = np.zeros(self.N * self.ncells)
        info = np.zeros(2 + MAXP)
        st = lib().mpo_pf_divj(self.ref(), _ptr(U), float(eta), _ptr(out), _ptr(info))
        if st != 0:
            raise RuntimeError(f"mpo_pf_divj status {st}")
        return out.reshape(self.N, self.ncells), {
            "M": info[0], "present": int(info[1]), "B": info[2:2 + self.N].copy()}

    def _faces(self):
        """Upper-face pairs (i, j) per direction: j is the neighbour of cell i
        at x_{i+1/2}; an outflow end has no face (zero flux)."""
        shape = self.shape[::-1]            # (ny, nx) / (nx,)
        idx = np.arange(self.ncells).reshape(shape)
        out = []
        for d in range(self.ndim):
            ax = self.ndim - 1 - d
            j = np.roll(idx, -1, axis=ax)
            i = idx
            if self.bc[d][1] != BC_PERIODIC:
                sl = [slice(None)] * self.ndim
                sl[ax] = slice(0, shape[ax] - 1)
                i, j = i[tuple(sl)], j[tuple(sl)]
            out.append((i.reshape(-1), j.reshape(-1)))
        return out

    def q_operator(self, phi):
        """The matrix of the discrete left side of Eq. (4):
        (A Q)_i = sum_d [k_{i+1/2}(Q_{i+1} - Q_i) - k_{i-1/2}(Q_i - Q_{i-1})]/dx_d^2
        with k = max(phi (1 - phi), PF_KFLOOR) and the face k the mean of its two cells
        (reading: second order, as the other discrete operators of
        Eq. (28))."""
        import scipy.sparse as sp
        k = np.maximum(phi * (1.0 - phi), PF_KFLOOR)
        rows, cols, vals = [], [], []
        for d, (i, j) in enumerate(self._faces()):
            c = 0.5 * (k[i] + k[j]) / self.dx[d] ** 2
            rows += [i, i, j, j]
            cols += [i, j, j, i]
            vals += [-c, c, -c, c]
        n = self.ncells
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                     np.concatenate(cols))), shape=(n, n))

    def pf_gradients(self, U, divj):
        """Solve Eq. (4) for each phase by a sparse direct solve (the
        definition: the solution of the discrete system) and return the face
        gradients G (ndim, N, ncells): dQ_p/dx_d at the upper face of each
        cell (0 at an outflow end), plus the relative residuals.  Q is fixed
        up to a constant (the floored k joins all cells); one cell is held at
        0.  A phase with [div J_p] = 0 everywhere has Q_p = 0."""
        import scipy.sparse.csgraph as cg
        import scipy.sparse.linalg as sla
        U = _arr(U, self.nU * self.ncells).reshape(self.nU, self.ncells)
        faces = self._faces()
        G = np.zeros((self.ndim, self.N, self.ncells))
        res = np.zeros(self.N)
        for p in range(self.N):
            phi = U[self.N + self.ndim + 1 + p]
            r = np.asarray(divj[p], dtype=np.float64)
            Q = np.zeros(self.ncells)
            if np.any(r != 0.0):
                A = self.q_operator(phi)
                off = A.copy()
                off.setdiag(0.0)
                off.eliminate_zeros()
                ncomp, lab = cg.connected_components(off != 0, directed=False)
                deg = np.asarray((off != 0).sum(axis=1)).ravel()
                keep = np.ones(self.ncells, dtype=bool)
                keep[deg == 0] = False
                for c in range(ncomp):
                    cells = np.nonzero((lab == c) & keep)[0]
                    if cells.size:
                        keep[cells[0]] = False
                ix = np.nonzero(keep)[0]
                if ix.size:
                    # sparse LU, then iterative refinement with the same
                    # factors (the coefficient spans many decades)
                    Ar = A[ix][:, ix].tocsc()
                    lu = sla.splu(Ar)
                    x = lu.solve(r[ix])
                    for _ in range(4):
                        x = x + lu.solve(r[ix] - Ar @ x)
                    Q[ix] = x
                nr = np.linalg.norm(r)
                res[p] = np.linalg.norm(A @ Q - r) / nr
            for d, (i, j) in enumerate(faces):
                G[d, p, i] = (Q[j] - Q[i]) / self.dx[d]
        return G, res

    def pf_k(self, U):
        """k_p = max(phi_p (1 - phi_p), PF_KFLOOR) of Eq. (4), (N, ncells)."""
        a = _arr(U, self.nU * self.ncells).reshape(self.nU, -1)[self.N + self.ndim + 1:]
        return np.ascontiguousarray(np.maximum(a * (1.0 - a), PF_KFLOOR))

    def pf_rhs(self, U, G, K):
        U = _arr(U, self.nU * self.ncells)
        G = _arr(G, self.ndim * self.N * self.ncells)
        K = _arr(K, self.N * self.ncells)
        L = np.empty_like(U)
        st = lib().mpo_pf_rhs(self.ref(), _ptr(U), _ptr(G), _ptr(K), _ptr(L))
        if st != 0:
            raise RuntimeError(f"mpo_pf_rhs status {st}")
        return L

    def pf_rk3(self, U, G, K, dt):
        U = _arr(U, self.nU * self.ncells).copy()
        G = _arr(G, self.ndim * self.N * self.ncells)
        K = _arr(K, self.N * self.ncells)
        st = lib().mpo_pf_rk3(self.ref(), _ptr(U), _ptr(G), _ptr(K), float(dt))
        if st != 0:
            raise RuntimeError(f"mpo_pf_rk3 status {st}")
        return U

    def pf_clip(self, G, dt):
        """Gradients clipped to the Phase-Field CFL bound PF_CFL dx_d / dt."""
        G = np.array(G, dtype=np.float64, copy=True)
        for d in range(self.ndim):
            g = PF_CFL * self.dx[d] / dt
            G[d] = np.minimum(np.maximum(G[d], -g), g)
        return G

    def pf_step(self, U, dt, eta):
        """The Phase-Field step of Sec. 2.2.1: phi_p = alpha_p of U (the
        hyperbolic result), [div J_p] by Eq. (28), Q_p by Eq. (4), the face
        gradients clipped to the PF CFL bound, then SSP-RK3 of Eq. (5) with
        the gradients frozen over the step."""
        divj, info = self.pf_divj(U, eta)
        G, res = self.pf_gradients(U, divj)
        G = self.pf_clip(G, dt)
        K = self.pf_k(U)
        return self.pf_rk3(U, G, K, dt), {"divj": divj, "G": G, "K": K, "residual": res,
                                          **info}

    def step_pf(self, U, dt, eta):
        """One full time step with the Phase-Field mechanism: the hyperbolic
        SSP-RK3 step, then the Phase-Field step, both with dt."""
        return self.pf_step(self.step(U, dt), dt, eta)

    def pf_flux(self, VL, VR, G, kf=None, dir=0):
        F = np.zeros(self.nU)
        kf = np.full(self.N, np.inf) if kf is None else kf
        lib().mpo_pf_flux(self.ref(), int(dir), _ptr(_arr(VL, self.nU)),
                          _ptr(_arr(VR, self.nU)), _ptr(_arr(G, self.N)),
                          _ptr(_arr(kf, self.N)), _ptr(F))
        return F

    # ---- pointwise building blocks -------------------------------------
    def pressure(self, Ucell):
        U = _arr(Ucell, self.nU)
        u = np.zeros(3)
        P = lib().mpo_pressure(self.ref(), _ptr(U), 1, _ptr(u))
        return P, u[: self.ndim].copy()

    def temperature(self, Ucell):
        U = _arr(Ucell, self.nU)
        return lib().mpo_temperature(self.ref(), _ptr(U), 1)

    def sound_speed(self, alpha, m, P):
        a = _arr(alpha, self.N)
        mm = _arr(m, self.N)
        return lib().mpo_sound_speed(self.ref(), _ptr(a), _ptr(mm), float(P))

    def one_plus_K(self, Ucell, p):
        return lib().mpo_one_plus_K(self.ref(), _ptr(_arr(Ucell, self.nU)), int(p))

    def psi(self, Ucell):
        U = _arr(Ucell, self.nU)
        return lib().mpo_psi(self.ref(), _ptr(U))

    def reconstruct_cell(self, Ustencil, dir=0):
        """Ustencil: (5, nU) conserved states of cells i-2..i+2."""
        Us = _arr(Ustencil, 5 * self.nU)
        UL, UR, VL, VR = (np.zeros(self.nU) for _ in range(4))
        info = np.zeros(3)
        lib().mpo_reconstruct_cell(self.ref(), _ptr(Us), int(dir), _ptr(UL),
                                   _ptr(UR), _ptr(VL), _ptr(VR), _ptr(info))
        return UL, UR, VL, VR, info

    def flux(self, UL, VL, UR, VR, dir=0):
        F = np.zeros(self.nU)
        uh = np.zeros(1)
        lib().mpo_flux(self.ref(), int(dir), _ptr(_arr(UL, self.nU)),
                       _ptr(_arr(VL, self.nU)), _ptr(_arr(UR, self.nU)),
                       _ptr(_arr(VR, self.nU)), _ptr(F), _ptr(uh))
        return F, float(uh[0])


def weno5_beta(q):
    q = _arr(q, 5)
    b = np.zeros(3)
    lib().mpo_weno5_beta(_ptr(q), _ptr(b))
    return b


def weno5_candidates(q):
    q = _arr(q, 5)
    cl, cr = np.zeros(3), np.zeros(3)
    lib().mpo_weno5_candidates(_ptr(q), _ptr(cl), _ptr(cr))
    return cl, cr


def weno5_increments(q):
    q = _arr(q, 5)
    dl, dr = np.zeros(3), np.zeros(3)
    lib().mpo_weno5_increments(_ptr(q), _ptr(dl), _ptr(dr))
    return dl, dr


def weno5_ideal():
    dl, dr = np.zeros(3), np.zeros(3)
    lib().mpo_weno5_ideal(_ptr(dl), _ptr(dr))
    return dl, dr


def wenow_weights(beta, d):
    w = np.zeros(3)
    lib().mpo_wenow_weights(_ptr(_arr(beta, 3)), _ptr(_arr(d, 3)), _ptr(w))
    return w


def wenojs_weights(beta, d, eps):
    w = np.zeros(3)
    lib().mpo_wenojs_weights(_ptr(_arr(beta, 3)), _ptr(_arr(d, 3)), float(eps),
                             _ptr(w))
    return w


def weno5w(q):
    ql, qr = np.zeros(1), np.zeros(1)
    lib().mpo_weno5w(_ptr(_arr(q, 5)), _ptr(ql), _ptr(qr))
    return float(ql[0]), float(qr[0])


def gl_interior(fbar, fL, fR):
    return lib().mpo_gl_interior(float(fbar), float(fL), float(fR))


def pf_gprime(phi):
    return lib().mpo_pf_gprime(float(phi))


def num_threads():
    return lib().mpo_num_threads()


def set_num_threads(n):
    lib().mpo_set_num_threads(int(n))


def interface_thickness(alpha, shape, dx, alpha_min=0.05, alpha_max=0.95):
    """Interface thickness N_I of Eq. (30): the volume where
    alpha_min <= alpha <= alpha_max, over dx times the integral of
    |grad alpha|.  Integrals are sums over cells times the cell volume; the
    gradient is the second-order central difference in the interior and the
    one-sided difference at the ends of each direction.  alpha: cell values
    in the state layout ([z][y][x], x fastest); dx: the cell size of each
    direction (x first); Eq. (30) divides by the cell size, taken as the
    smallest one."""
    a = np.asarray(alpha, dtype=np.float64).reshape(tuple(shape)[::-1])
    vol = float(np.prod(dx))
    inside = ((a >= alpha_min) & (a <= alpha_max)).sum() * vol
    g2 = np.zeros_like(a)
    for d in range(len(shape)):
        ax = a.ndim - 1 - d
        if a.shape[ax] > 1:
            g2 += np.gradient(a, dx[d], axis=ax) ** 2
    grad = np.sqrt(g2).sum() * vol
    return inside / (min(dx) * grad) if grad > 0.0 else 0.0
