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

BC_PERIODIC, BC_OUTFLOW = 0, 1
RECON_WENO_C, RECON_WENO_CL = 0, 1
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
        ("t_end", C.c_double),
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
                 model=MODEL_ALLAIRE, energy_limiter=1, cfl=0.5, t_end=0.0):
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
        self._p = p
        self.ndim, self.N = ndim, N
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


def num_threads():
    return lib().mpo_num_threads()


def set_num_threads(n):
    lib().mpo_set_num_threads(int(n))
