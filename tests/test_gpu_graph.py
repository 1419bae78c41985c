"""quapi_step_graph: the launches of quapi_step recorded once into a HIP graph
and replayed.  Every replay must equal eager stepping bit for bit (rho(t),
counters, stored groups), also with eager steps, synchronisations and other
replays between them, on the direct-mapped and the bucketed store; the batched
form likewise; the hash-table merge refuses.
"""
import numpy as np
import pytest

import oracle
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


def _eta(Q, wl, bath, K):
    return Q.quapi_eta(bath.ohmic_alpha, bath.ohmic_wc, [x for pk in bath.peaks for x in pk], wl.beta, wl.dt, K)


# lags 0..5 exact: merge positions 0..4, the bucketed store; lags 0..7: 0..6, the
# direct-mapped store
@pytest.mark.parametrize("n_exact,store", [(6, "BUCKETED"), (8, "DIRECT")])
def test_graph_replays_equal_eager_steps(Q, n_exact, store):
    wl = W.structured_bath(K=12, n_exact=n_exact, theta=1e-7)
    K, n, extra = 12, 40, 5
    eta = _eta(Q, wl, wl.bath, K)
    mk = lambda: Q.Propagator(wl.H, wl.q, wl.dt, K, eta, wl.rho0, mask=wl.mask, theta=wl.theta)
    ref = mk()
    assert ref.info()["store"] == getattr(Q, f"QUAPI_MERGE_{store}")
    ref.step(n)
    ref_groups = ref.groups()
    ref_stats = ref.stats(1, n)
    ref.step(extra)
    ref_rho = ref.rho_history(0, n + extra + 1)
    g = mk()
    for rep in range(3):
        print(f"[graph] replay {rep}: {n} steps", flush=True)
        g.reset()
        g.step_graph(n)
        g.sync()
        assert np.array_equal(g.rho_history(0, n + 1), ref_rho[:n + 1]), rep
        assert g.stats(1, n) == ref_stats, rep
        h, w = g.groups()
        assert np.array_equal(h, ref_groups[0]) and np.array_equal(w, ref_groups[1]), rep
        g.step(extra)                                    # eager steps after a replay
        assert np.array_equal(g.rho_history(0, n + extra + 1), ref_rho), rep
    # a run recorded at another start, then the first one recorded anew
    g.reset()
    g.step(10)
    g.step_graph(n - 10)
    assert np.array_equal(g.rho_history(0, n + 1), ref_rho[:n + 1])
    g.reset()
    g.step_graph(n)
    assert np.array_equal(g.rho_history(0, n + 1), ref_rho[:n + 1])
    # and the oracle
    o = oracle.Oracle(wl.H, wl.q, wl.dt, K, eta, wl.rho0, mask=wl.mask, theta=wl.theta, mode=oracle.PRE)
    o.step(n)
    assert np.abs(g.rho_history(0, n + 1) - o.rho_history()).max() < RHO_TOL


def test_graph_batched_form(Q):
    wl, baths = W.batched_scan(n_inst=4, seed=6, K=12, n_exact=6, theta=1e-7)
    K, n = 12, 30
    etas = np.stack([_eta(Q, wl, b, K) for b in baths])
    mk = lambda: Q.BatchPropagator(wl.H, wl.q, wl.dt, K, etas, wl.rho0, mask=wl.mask, theta=wl.theta)
    ref = mk()
    ref.step(n)
    ref_rho = ref.rho_all(0, n + 1)
    ref_groups = [ref.groups(j) for j in range(4)]
    g = mk()
    for rep in range(3):
        print(f"[graph] batched replay {rep}: 4 instances, {n} steps", flush=True)
        g.reset()
        g.step_graph(n)
        assert np.array_equal(g.rho_all(0, n + 1), ref_rho), rep
        for j in range(4):
            h, w = g.groups(j)
            assert np.array_equal(h, ref_groups[j][0]) and np.array_equal(w, ref_groups[j][1]), (rep, j)


def test_graph_refused_on_the_hash_table_merge(Q):
    wl = W.structured_bath(K=12, n_exact=6, theta=1e-7)
    K = 12
    eta = _eta(Q, wl, wl.bath, K)
    g = Q.Propagator(wl.H, wl.q, wl.dt, K, eta, wl.rho0, mask=tuple(range(6)) + (8, 10), theta=wl.theta)
    assert g.info()["hash_merge"] == 1
    with pytest.raises(Q.QuapiError) as e:
        g.step_graph(5)
    assert e.value.code == Q.QUAPI_EUNSUPPORTED
    g.step(5)                                            # eager stepping is unaffected
    g.sync()
