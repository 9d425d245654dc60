import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: longer CPU-only oracle checks")


@pytest.fixture(scope="session")
def oracle():
    """The FP64 CPU oracle; built from source on first use."""
    from oracle import mpo
    if not os.path.exists(mpo.LIB_PATH):
        mpo.build()
    return mpo


def oracle_problem(mpo, w, **over):
    """Oracle Problem for an inputs.Workload (plain field copy)."""
    o = w.opts
    kw = dict(recon=o.recon, flux=o.flux, model=o.model,
              energy_limiter=o.energy_limiter, cfl=o.cfl, t_end=w.t_end,
              alpha_source=o.alpha_source)
    kw.update(over)
    return mpo.Problem(w.ndim, w.n, w.dx, w.bc, list(w.gamma), list(w.pinf),
                       list(w.D), list(w.pmin), list(w.cT), **kw)
