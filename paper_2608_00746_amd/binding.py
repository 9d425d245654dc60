"""Thin ctypes binding of libmpweno.so (include/mp_weno.h).

Argument marshalling only: every step of the scheme runs in the HIP kernels
of the library.  PyTorch provides device memory and the stream.  The binding
raises if the library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpweno.so")
MAXP = 8
DIAG_LEN = 40

OK, ERR_ARG, ERR_HIP, ERR_OOM, ERR_INADMISSIBLE, ERR_NONFINITE, ERR_SOLVER, \
    ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
WHERE_DEVICE, WHERE_HOST = 0, 1


class MpWenoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mp_weno status {status}: {msg}")
        self.status = status


class Instance(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double * 3),
        ("bc", (C.c_int32 * 2) * 3), ("nphase", C.c_int32),
        ("gamma", C.c_double * MAXP), ("pinf", C.c_double * MAXP),
        ("D", C.c_double * MAXP), ("pmin", C.c_double * MAXP),
        ("cT", C.c_double * MAXP), ("t_end", C.c_double),
        ("U", C.c_void_p),
    ]


class Link(C.Structure):
    _fields_ = [("fine", C.c_int32), ("coarse", C.c_int32), ("lo", C.c_int32 * 3)]


class Opts(C.Structure):
    _fields_ = [
        ("recon", C.c_int32), ("flux", C.c_int32), ("model", C.c_int32),
        ("precision", C.c_int32), ("energy_limiter", C.c_int32),
        ("phase_field", C.c_int32), ("cfl", C.c_double),
        ("eta_over_dx", C.c_double), ("cg_rtol", C.c_double),
        ("cg_maxit", C.c_int32), ("check_bounds", C.c_int32),
        ("use_graph", C.c_int32), ("alpha_source", C.c_int32),
    ]


_lib = None


def lib():
    """Load the built library (build it with paper_2608_00746_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.mp_weno_abi_version.restype = C.c_int32
        L.mp_weno_max_phases.restype = C.c_int32
        L.mp_weno_init.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(Instance),
                                   C.POINTER(Opts), vp]
        L.mp_weno_init.restype = C.c_int
        L.mp_weno_rhs.argtypes = [vp, C.POINTER(vp), C.POINTER(vp)]
        L.mp_weno_rhs.restype = C.c_int
        L.mp_weno_pf_fields.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                        C.POINTER(vp)]
        L.mp_weno_pf_fields.restype = C.c_int
        L.mp_weno_autotune.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32)]
        L.mp_weno_autotune.restype = C.c_int
        L.mp_weno_advance.argtypes = [vp, C.c_int32]
        L.mp_weno_advance.restype = C.c_int
        L.mp_weno_dt.argtypes = [vp, vp, C.c_int32]
        L.mp_weno_dt.restype = C.c_int
        L.mp_weno_step.argtypes = [vp, vp]
        L.mp_weno_step.restype = C.c_int
        L.mp_weno_diag.argtypes = [vp, vp, C.c_int32]
        L.mp_weno_diag.restype = C.c_int
        L.mp_weno_set_time.argtypes = [vp, C.POINTER(C.c_double)]
        L.mp_weno_set_time.restype = C.c_int
        L.mp_weno_destroy.argtypes = [vp]
        L.mp_weno_destroy.restype = C.c_int
        L.mp_weno_strerror.argtypes = [C.c_int]
        L.mp_weno_strerror.restype = C.c_char_p
        L.mp_weno_last_error.argtypes = [vp]
        L.mp_weno_last_error.restype = C.c_char_p
        L.mp_weno_profile.argtypes = [vp, C.c_int32]
        L.mp_weno_profile.restype = C.c_int
        L.mp_weno_timing.argtypes = [vp, C.c_int32, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int64)]
        L.mp_weno_timing.restype = C.c_int
        L.mp_weno_amr_link.argtypes = [vp, C.c_int32, C.POINTER(Link)]
        L.mp_weno_amr_link.restype = C.c_int
        L.mp_weno_rhs_noalloc.argtypes = [C.POINTER(Instance), C.POINTER(Opts), vp, vp, vp]
        L.mp_weno_rhs_noalloc.restype = C.c_int
        L.mp_weno_rhs_noalloc_scratch_bytes.restype = C.c_size_t
        _lib = L
    return _lib


EXPORTED = ["mp_weno_abi_version", "mp_weno_max_phases", "mp_weno_init",
            "mp_weno_rhs", "mp_weno_pf_fields", "mp_weno_autotune", "mp_weno_dt",
            "mp_weno_step", "mp_weno_advance", "mp_weno_diag",
            "mp_weno_set_time", "mp_weno_destroy", "mp_weno_strerror",
            "mp_weno_last_error", "mp_weno_profile", "mp_weno_timing",
            "mp_weno_rhs_noalloc", "mp_weno_rhs_noalloc_scratch_bytes", "mp_weno_amr_link"]


def make_instance(w, U_ptr):
    """Fill the C instance struct from an inputs.Workload and a device pointer."""
    s = Instance()
    s.ndim = w.ndim
    nn = list(w.n) + [1] * (3 - len(w.n))
    dd = list(w.dx) + [1.0] * (3 - len(w.dx))
    for k in range(3):
        s.n[k] = int(nn[k])
        s.dx[k] = float(dd[k])
    bcl = list(w.bc) + [(0, 0)] * (3 - len(w.bc))
    for k in range(3):
        s.bc[k][0], s.bc[k][1] = int(bcl[k][0]), int(bcl[k][1])
    s.nphase = w.N
    for name, vals in (("gamma", w.gamma), ("pinf", w.pinf), ("D", w.D),
                       ("pmin", w.pmin), ("cT", w.cT)):
        arr = getattr(s, name)
        for p in range(w.N):
            arr[p] = float(vals[p])
    s.t_end = float(w.t_end)
    s.U = C.c_void_p(int(U_ptr))
    return s


def make_opts(o, check_bounds=False, use_graph=False):
    x = Opts()
    x.recon, x.flux, x.model = int(o.recon), int(o.flux), int(o.model)
    x.precision, x.energy_limiter = int(o.precision), int(o.energy_limiter)
    x.phase_field = int(o.phase_field)
    x.cfl = float(o.cfl)
    x.eta_over_dx = float(o.eta_over_dx)
    x.cg_rtol, x.cg_maxit = float(o.cg_rtol), int(o.cg_maxit)
    x.check_bounds, x.use_graph = int(check_bounds), int(use_graph)
    x.alpha_source = int(getattr(o, "alpha_source", 0))
    return x


def rhs_noalloc(w, U, out, stream=None, opts=None):
    """mp_weno_rhs_noalloc for one inputs.Workload: L(U) of the device state
    U (torch float64 tensor) into out (same shape), on `stream` (a torch
    stream; default: the current one).  Returns the status code."""
    import torch
    st = stream or torch.cuda.current_stream(U.device)
    inst = make_instance(w, U.data_ptr())
    o = make_opts(opts or w.opts)
    return lib().mp_weno_rhs_noalloc(C.byref(inst), C.byref(o), C.c_void_p(U.data_ptr()),
                                     C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream))


class Solver:
    """Instances advanced together by one context.

    workloads: list of inputs.Workload (same Options for all); their states
    are copied to the GPU once and stay resident (self.U[i], torch float64).
    """

    def __init__(self, workloads, opts=None, device="cuda:0", stream=None,
                 check_bounds=False, use_graph=False):
        import torch
        if not isinstance(workloads, (list, tuple)):
            workloads = [workloads]
        self.torch = torch
        self.w = list(workloads)
        self.opts = opts or self.w[0].opts
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.U = [torch.from_numpy(np.ascontiguousarray(w.U)).to(self.device)
                  for w in self.w]
        self._inst = (Instance * len(self.w))(
            *[make_instance(w, u.data_ptr()) for w, u in zip(self.w, self.U)])
        self._opts = make_opts(self.opts, check_bounds, use_graph)
        self.ctx = C.c_void_p()
        st = lib().mp_weno_init(C.byref(self.ctx), len(self.w), self._inst,
                                C.byref(self._opts), C.c_void_p(self.stream.cuda_stream))
        self._check(st)
        torch.cuda.synchronize(self.device)

    def _enter(self):
        """Order the context stream after work queued on torch's stream."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _leave(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def _check(self, st):
        if st != OK:
            msg = lib().mp_weno_strerror(st).decode()
            if self.ctx:
                extra = lib().mp_weno_last_error(self.ctx).decode()
                if extra:
                    msg += ": " + extra
            raise MpWenoError(st, msg)

    def rhs(self, U_in=None):
        """L(U) per instance (list of torch tensors)."""
        torch = self.torch
        outs = [torch.empty_like(u) for u in self.U]
        n = len(self.U)
        ins = (C.c_void_p * n)(*[C.c_void_p((U_in[i] if U_in else self.U[i]).data_ptr())
                                 for i in range(n)])
        ptrs = (C.c_void_p * n)(*[C.c_void_p(o.data_ptr()) for o in outs])
        self._enter()
        self._check(lib().mp_weno_rhs(self.ctx, ins, ptrs))
        self._leave()
        return outs

    def pf_fields(self, U_in=None, divj=True, grad=True, dudt=True):
        """Phase-Field fields per instance from the volume fractions of U_in
        (default: the instances' states): dict of lists of torch tensors
        'divj' (N, cells), 'grad' (d, N, cells), 'dudt' (U layout)."""
        torch = self.torch
        n = len(self.U)
        out = {}
        arrs = {}
        for key, on, shape in (("divj", divj, lambda w: (w.N, w.ncells)),
                               ("grad", grad, lambda w: (w.ndim, w.N, w.ncells)),
                               ("dudt", dudt, None)):
            if on:
                out[key] = [torch.empty(shape(w), dtype=torch.float64, device=self.device)
                            if shape else torch.empty_like(u) for w, u in zip(self.w, self.U)]
                arrs[key] = (C.c_void_p * n)(*[C.c_void_p(t.data_ptr()) for t in out[key]])
            else:
                arrs[key] = None
        ins = (C.c_void_p * n)(*[C.c_void_p((U_in[i] if U_in else self.U[i]).data_ptr())
                                 for i in range(n)])
        self._enter()
        self._check(lib().mp_weno_pf_fields(self.ctx, ins, arrs["divj"], arrs["grad"],
                                            arrs["dudt"]))
        self._leave()
        return out

    def autotune(self, reps=8):
        """Pick the fastest sweep tile shapes and tile order per group; returns
        per instance (x strip, y tile width, y tile height, XCD order)."""
        out = (C.c_int32 * (4 * len(self.U)))()
        self._enter()
        self._check(lib().mp_weno_autotune(self.ctx, int(reps), out))
        self._leave()
        return np.array(list(out), dtype=np.int64).reshape(len(self.U), 4)

    def amr_link(self, links):
        """Couple instances: links = [(fine, coarse, (lo_x[, lo_y])), ...]
        (mp_weno_amr_link); [] removes the coupling."""
        arr = (Link * max(len(links), 1))()
        for k, (f, c, lo) in enumerate(links):
            arr[k].fine, arr[k].coarse = int(f), int(c)
            for d, v in enumerate(lo):
                arr[k].lo[d] = int(v)
        self._check(lib().mp_weno_amr_link(self.ctx, len(links), arr))

    def dt(self):
        out = np.zeros(len(self.U))
        self._check(lib().mp_weno_dt(self.ctx, out.ctypes.data_as(C.c_void_p), WHERE_HOST))
        return out

    def step(self, dt=None):
        """One SSP-RK3 step; dt: None (CFL on device) or a float / sequence."""
        if dt is None:
            self._enter()
            self._check(lib().mp_weno_step(self.ctx, None))
            self._leave()
            return
        torch = self.torch
        d = torch.as_tensor(np.broadcast_to(np.asarray(dt, dtype=np.float64),
                                            (len(self.U),)).copy(), device=self.device)
        self._dt_keep = d
        self._enter()
        self._check(lib().mp_weno_step(self.ctx, C.c_void_p(d.data_ptr())))
        self._leave()

    def advance(self, nsteps):
        """nsteps SSP-RK3 steps with the device CFL step (runs of 16 steps
        replay one captured graph when use_graph is on)."""
        self._enter()
        self._check(lib().mp_weno_advance(self.ctx, int(nsteps)))
        self._leave()

    def diag(self):
        out = np.zeros(len(self.U) * DIAG_LEN)
        self._check(lib().mp_weno_diag(self.ctx, out.ctypes.data_as(C.c_void_p), WHERE_HOST))
        return out.reshape(len(self.U), DIAG_LEN)

    def set_time(self, t):
        arr = (C.c_double * len(self.U))(*np.broadcast_to(np.asarray(t, float),
                                                           (len(self.U),)))
        self._check(lib().mp_weno_set_time(self.ctx, arr))

    def profile(self, which):
        """Record events around stage kernels: 0 off, 1 x, 2 y, 3 stage."""
        self._check(lib().mp_weno_profile(self.ctx, int(which)))

    def timing(self, reset=False):
        """(total ms, launches) of the stage kernel since the last reset."""
        ms = C.c_double()
        n = C.c_int64()
        self._check(lib().mp_weno_timing(self.ctx, int(reset), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def host(self, i=0):
        self.torch.cuda.synchronize(self.device)
        return self.U[i].cpu().numpy()

    def interface_thickness(self, diag=None):
        """N_I of Eq. (30) for alpha_1 per instance, from the diagnostics'
        two integrals (slots 32 and 33)."""
        d = self.diag() if diag is None else diag
        out = np.zeros(len(self.U))
        for i, w in enumerate(self.w):
            den = min(w.dx) * d[i, 33]
            out[i] = d[i, 32] / den if den > 0.0 else 0.0
        return out

    def checkpoint(self, path=None):
        """The state that decides every later step: the instances' U and
        times (and, for the record, their step counts).  A context holds no
        other state the hyperbolic step reads; with the Phase-Field step the
        solve of Eq. (4) starts from the previous step's Q, which a
        checkpoint does not hold (a resumed run then matches to the solver
        tolerance, not bitwise).  path: also written there as .npz."""
        d = self.diag()
        ck = {"t": d[:, 26].copy(), "steps": d[:, 27].copy()}
        for i in range(len(self.U)):
            ck["U%d" % i] = self.host(i).copy()
        if path is not None:
            np.savez(path, **ck)
        return ck

    def restore(self, ck):
        """Load a checkpoint (dict or .npz path) into this context: the
        states are copied into the device buffers in place and the times
        set.  The step count is the context's own."""
        if not isinstance(ck, dict):
            with np.load(ck, allow_pickle=False) as f:
                ck = {k: f[k] for k in f.files}
        if len(ck["t"]) != len(self.U):
            raise ValueError("checkpoint of %d instances for %d" % (len(ck["t"]), len(self.U)))
        self.torch.cuda.synchronize(self.device)
        for i, u in enumerate(self.U):
            src = np.ascontiguousarray(ck["U%d" % i], dtype=np.float64)
            if src.size != u.numel():
                raise ValueError("instance %d: %d values for %d" % (i, src.size, u.numel()))
            u.copy_(self.torch.from_numpy(src.reshape(u.shape)))
        self.torch.cuda.synchronize(self.device)
        self.set_time(ck["t"])

    def close(self):
        if self.ctx:
            lib().mp_weno_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
