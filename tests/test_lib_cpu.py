"""CPU tests of the HIP library's C ABI: it loads, exports every function its
header declares, its host tables agree with independent references, and it
rejects invalid input before touching a device."""
import ctypes
import os

import numpy as np
import pytest
from scipy.linalg import expm

from paper_2506_03127_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def Q():
    from paper_2506_03127_amd import quapi
    if not os.path.exists(quapi.LIB_PATH):
        from paper_2506_03127_amd import _build
        _build.build()
    return quapi


def test_library_exports_every_declared_function(Q):
    names = Q.header_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(Q.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_propagator_matches_expm(Q):
    for M, seed in [(2, 1), (3, 2), (4, 3), (6, 4)]:
        H = W.random_hermitian(M, 0.7, seed)
        U = Q.quapi_propagator(H, 0.3)
        assert np.abs(U - expm(-0.3j * H)).max() < 1e-13
    assert np.abs(Q.quapi_propagator(W.tls_hamiltonian(0.5, 1.0), 0.2)
                  - expm(-0.2j * W.tls_hamiltonian(0.5, 1.0))).max() < 1e-14


def test_propagator_rejects_non_hermitian(Q):
    H = np.array([[0.0, 1.0], [0.5, 0.0]], dtype=complex)
    with pytest.raises(Q.QuapiError) as e:
        Q.quapi_propagator(H, 0.1)
    assert e.value.code == Q.QUAPI_EINVAL


@pytest.mark.parametrize("wl", [W.spin_boson_ohmic(), W.structured_bath()], ids=lambda w: w.name)
def test_eta_generator_matches_oracle_quadrature(Q, eta_cache, wl):
    """The library's Gauss-Legendre panels against the oracle's adaptive quadrature."""
    b = wl.bath
    peaks = [x for pk in b.peaks for x in pk]
    mine = Q.quapi_eta(b.ohmic_alpha, b.ohmic_wc, peaks, wl.beta, wl.dt, wl.K)
    ref = eta_cache(wl)
    assert np.abs(mine - ref).max() < 1e-12


def test_eta_rejects_bad_arguments(Q):
    with pytest.raises(Q.QuapiError):
        Q.quapi_eta(0.1, 5.0, [], -1.0, 0.2, 4)
    with pytest.raises(Q.QuapiError):
        Q.quapi_eta(0.1, 5.0, [1.0, -0.05, 0.1], 5.0, 0.2, 4)
    with pytest.raises(Q.QuapiError):
        Q.quapi_eta(0.1, 5.0, [], 5.0, 0.2, 0)


def _create_code(Q, **over):
    wl = W.spin_boson_ohmic()
    args = dict(H=wl.H, q=wl.q, dt=wl.dt, dk_max=wl.K, eta=np.zeros((3, wl.K + 1)), rho0=wl.rho0,
                mask=None, theta=0.0, mode=Q.QUAPI_POST)
    args.update(over)
    try:
        ctx = Q.quapi_create(**args)
    except Q.QuapiError as e:
        return e.code
    Q.quapi_destroy(ctx)
    return 0


def test_create_rejects_invalid_input_without_device(Q):
    assert _create_code(Q, H=np.array([[0, 1], [2, 0]], dtype=complex)) == Q.QUAPI_EINVAL
    assert _create_code(Q, dt=-0.1) == Q.QUAPI_EINVAL
    assert _create_code(Q, theta=-1.0) == Q.QUAPI_EINVAL
    assert _create_code(Q, mask=[0, 2, 3]) == Q.QUAPI_EINVAL          # lag 1 missing
    assert _create_code(Q, mask=[1, 2]) == Q.QUAPI_EINVAL             # lag 0 missing
    assert _create_code(Q, mask=[0, 1, 1]) == Q.QUAPI_EINVAL          # not strictly sorted
    assert _create_code(Q, mask=[0, 1, 8]) == Q.QUAPI_EINVAL          # lag beyond dk_max - 1
    assert _create_code(Q, mode=7) == Q.QUAPI_EINVAL
    assert _create_code(Q, merge=5) == Q.QUAPI_EINVAL                 # no such store
    eta_nan = np.zeros((3, 9), dtype=complex)
    eta_nan[0, 3] = np.nan
    assert _create_code(Q, eta=eta_nan) == Q.QUAPI_EINVAL
    # valid but outside this build: merge positions that are not 0..L-1 with more
    # other points than one 64-bit word holds (38 two-bit points), a key over 62
    # bits (32 two-bit merge positions), M = 5, and M = 4 on a store other than the
    # hash table or with a history over 128 bits (33 four-bit points)
    assert _create_code(Q, dk_max=40, eta=np.zeros((3, 41)), mask=[0, 1, 3]) == Q.QUAPI_EUNSUPPORTED
    mask64 = list(range(31)) + [40, 63]
    assert _create_code(Q, dk_max=64, eta=np.zeros((3, 65)), mask=mask64) == Q.QUAPI_EUNSUPPORTED
    H5 = W.random_hermitian(5, 0.5, 1)
    assert _create_code(Q, H=H5, q=[1, 0.5, 0, -0.5, -1], rho0=W.ground_projector(5)) == Q.QUAPI_EUNSUPPORTED
    H4 = W.random_hermitian(4, 0.5, 1)
    four = dict(H=H4, q=[1, 0.5, -0.5, -1], rho0=W.ground_projector(4))
    for merge in (Q.QUAPI_MERGE_DIRECT, Q.QUAPI_MERGE_BUCKETED):
        assert _create_code(Q, merge=merge, **four) == Q.QUAPI_EUNSUPPORTED
    assert _create_code(Q, dk_max=33, eta=np.zeros((3, 34)), **four) == Q.QUAPI_EUNSUPPORTED


def _create_batch_code(Q, n_inst=2, **over):
    wl = W.structured_bath(K=8, n_exact=4)
    args = dict(H=wl.H, q=wl.q, dt=wl.dt, dk_max=wl.K, etas=np.zeros((n_inst, 3, wl.K + 1)), rho0=wl.rho0,
                mask=wl.mask, theta=0.0, mode=Q.QUAPI_PRE)
    args.update(over)
    try:
        ctx = Q.quapi_create_batch(**args)
    except Q.QuapiError as e:
        return e.code
    Q.quapi_destroy(ctx)
    return 0


def test_create_batch_rejects_invalid_input_without_device(Q):
    assert _create_batch_code(Q, n_inst=0) == Q.QUAPI_EINVAL
    assert _create_batch_code(Q, n_inst=1025) == Q.QUAPI_EINVAL
    etas = np.zeros((3, 3, 9), dtype=complex)
    etas[2, 1, 4] = np.inf                              # the last instance's table
    assert _create_batch_code(Q, n_inst=3, etas=etas) == Q.QUAPI_EINVAL
    assert _create_batch_code(Q, mask=[0, 1, 3]) == Q.QUAPI_EUNSUPPORTED   # hash-table merge
    for merge in (Q.QUAPI_MERGE_HASH, Q.QUAPI_MERGE_PARTITION):
        assert _create_batch_code(Q, merge=merge) == Q.QUAPI_EUNSUPPORTED
    assert _create_batch_code(Q, mode=9) == Q.QUAPI_EINVAL
    Hb = np.stack([W.tls_hamiltonian(0.5, 1.0), np.array([[0, 1], [2, 0]], dtype=complex)])
    assert _create_batch_code(Q, H_batch=Hb) == Q.QUAPI_EINVAL          # second H not Hermitian


def test_mlp_create_rejects_invalid_sizes_without_device(Q):
    import ctypes
    h = ctypes.c_void_p()
    for args in [(0, 256, 4, 4, 64), (6, 0, 4, 4, 64), (6, 256, 0, 4, 64), (6, 256, 4, 0, 64), (6, 256, 4, 4, 0),
                 (6, 5000, 4, 4, 64), (6, 256, 65, 4, 64), (6, 256, 4, 4, (1 << 22) + 1)]:
        rc = Q.lib().quapi_mlp_create(*args, ctypes.c_ulonglong(1), None, ctypes.byref(h))
        assert rc == Q.QUAPI_EINVAL, args
        assert not h.value


def test_strerror_names_every_code(Q):
    names = {Q.strerror(c) for c in (0, -1, -2, -3, -4, -5)}
    assert len(names) == 6 and "unknown error" not in names


def test_calls_on_no_context_are_rejected_without_device(Q):
    """Every stepping and reading call checks its context before any device
    work: a null context is EINVAL."""
    L = Q.lib()
    assert L.quapi_step(None, 1) == Q.QUAPI_EINVAL
    assert L.quapi_step_graph(None, 1) == Q.QUAPI_EINVAL
    assert L.quapi_sync(None) == Q.QUAPI_EINVAL
    assert L.quapi_reset(None) == Q.QUAPI_EINVAL
    assert L.quapi_set_chunk_run(None, 1) == Q.QUAPI_EINVAL
