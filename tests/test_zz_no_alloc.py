"""quapi_run_static, the entry point that allocates nothing: its rho(t), for
two calls in a row (the second smaller), equal those of a context on the
direct-mapped store (the entry point it is a variant of), and a run that does
not fit its static array is refused before any device work."""
import numpy as np
import pytest

from paper_2506_03127_amd import workloads as W

pytestmark = pytest.mark.gpu

RHO_TOL = 1e-12


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_03127_amd import quapi
    quapi.lib()
    return quapi


def _static_rho(Q, wl, eta, n, mask, theta, mode, stream):
    import torch
    out = torch.full(((n + 1) * 4 * 2,), float("nan"), dtype=torch.float64, device="cuda")
    Q.quapi_run_static(wl.H, wl.q, wl.dt, wl.K, eta, wl.rho0, n, out.data_ptr(), mask=mask, theta=theta,
                       mode=mode, stream=stream.cuda_stream)
    stream.synchronize()
    r = out.cpu().numpy()
    return (r[0::2] + 1j * r[1::2]).reshape(n + 1, 2, 2)


def test_static_entry_point_equals_the_direct_store(Q, eta_cache):
    import torch
    s = torch.cuda.Stream()
    cases = [
        # exact iQUAPI (every lag on the mask, post-merging), 4^8 slots
        (W.spin_boson_ohmic(mode="post"), None, 0.0, Q.QUAPI_POST, 100),
        # then a smaller one: the structured bath with lags 0..6 exact (4^6 slots)
        (W.structured_bath(K=12), (0, 1, 2, 3, 4, 5, 6), 1e-7, Q.QUAPI_PRE, 60),
    ]
    for wl, mask, theta, mode, n in cases:
        eta = eta_cache(wl)
        print(f"[no-alloc] K={wl.K} mask={mask} mode={mode} n={n}", flush=True)
        got = _static_rho(Q, wl, eta, n, mask, theta, mode, s)
        ref = Q.Propagator(wl.H, wl.q, wl.dt, wl.K, eta, wl.rho0, mask=mask, theta=theta, mode=mode,
                           merge=Q.QUAPI_MERGE_DIRECT)
        ref.step(n)
        want = ref.rho_history()
        err = np.abs(got - want).max()
        print(f"[no-alloc] max |rho_static - rho_context| = {err:.3e}", flush=True)
        assert np.isfinite(got).all() and err <= RHO_TOL


def test_static_entry_point_refuses_what_does_not_fit(Q, eta_cache):
    import torch
    wl = W.structured_bath()                  # lags 0..11 exact: 4^11 slots, beyond the array
    eta = eta_cache(wl)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(Q.QuapiError) as e:
        Q.quapi_run_static(wl.H, wl.q, wl.dt, wl.K, eta, wl.rho0, 1, out.data_ptr(), mask=wl.mask,
                           theta=wl.theta)
    assert e.value.code == Q.QUAPI_EUNSUPPORTED
    # 4^10 slots fit, but not with 2000000 steps of counters (96 MB of them)
    wl2 = W.structured_bath(K=14)
    eta2 = eta_cache(wl2)
    with pytest.raises(Q.QuapiError) as e2:
        Q.quapi_run_static(wl2.H, wl2.q, wl2.dt, 14, eta2, wl2.rho0, 2000000, out.data_ptr(),
                           mask=tuple(range(11)), theta=1e-7)
    assert e2.value.code == Q.QUAPI_ENOMEM
