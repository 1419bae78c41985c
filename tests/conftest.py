import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build(force=True)
    return oracle


_ETA_CACHE = {}


def eta_for(wl, K=None):
    """eta columns of a workload from the oracle's quadrature (cached per session)."""
    from oracle.eta import Bath, eta_columns
    K = wl.K if K is None else K
    key = (wl.bath, wl.beta, wl.dt, K)
    if key not in _ETA_CACHE:
        b = wl.bath
        _ETA_CACHE[key] = eta_columns(Bath(b.ohmic_alpha, b.ohmic_wc, b.peaks), wl.beta, wl.dt, K)
    return _ETA_CACHE[key].copy()


@pytest.fixture(scope="session")
def eta_cache():
    return eta_for
