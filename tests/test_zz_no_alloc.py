"""The allocation-free L(U) entry point (mp_weno_rhs_noalloc) against the
context entry point mp_weno_rhs on the same instance: identical results, on
two calls in a row (the second on a smaller input, so the shared scratch
holds the first call's larger accumulator), in 1D, 2D and 3D, and sizes
beyond the scratch are rejected on the host."""
import numpy as np
import pytest

from paper_2608_00746_amd import inputs as I

pytestmark = pytest.mark.gpu


def _pair(w):
    import torch
    from paper_2608_00746_amd.binding import Solver, rhs_noalloc
    s = Solver([w])
    ref = s.rhs()[0]
    U = s.U[0]
    out = torch.full_like(U, float("nan"))
    st = rhs_noalloc(w, U, out, stream=s.stream)
    assert st == 0, st
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    s.close()
    return a, b


@pytest.mark.parametrize("prec", [I.PREC_FP64, I.PREC_MIXED], ids=["fp64", "mixed"])
def test_noalloc_rhs_matches_context_rhs_twice(prec):
    seq = [
        I.random_state((130, 90), nphase=2, seed=21, opts=I.Options(flux=1, precision=prec)),
        I.random_state((37, 20), nphase=3, seed=22, bc=1, opts=I.Options(precision=prec)),
        I.random_state((300,), nphase=2, seed=23, opts=I.Options(precision=prec)),
        I.random_state((24, 18, 14), nphase=3, seed=24, opts=I.Options(flux=1, precision=prec)),
        I.random_state((11, 9, 7), nphase=2, seed=25, opts=I.Options(precision=prec)),
    ]
    for w in seq:
        a, b = _pair(w)
        print(w.name, "max |diff|", np.abs(a - b).max())
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), w.name


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import torch
    from paper_2608_00746_amd.binding import lib, make_instance, make_opts, MpWenoError
    cap = lib().mp_weno_rhs_noalloc_scratch_bytes()
    w = I.random_state((8, 8), nphase=2, seed=1)
    inst = make_instance(w, 1 << 20)               # never dereferenced: rejected first
    n = int(np.sqrt(cap / (8 * w.nU))) + 16        # n^2 cells need more than the scratch
    inst.n[0] = n
    inst.n[1] = n
    import ctypes as C
    st = lib().mp_weno_rhs_noalloc(C.byref(inst), C.byref(make_opts(w.opts)),
                                   C.c_void_p(1 << 20), C.c_void_p(1 << 20), None)
    assert st == -7   # MP_ERR_UNSUPPORTED, decided on the host
