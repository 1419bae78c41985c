"""The batched form (quapi_create_batch): several instances -- bath parameter
points -- propagated by one step-kernel launch per time step.

Each instance's groups start at a chunk boundary and reduce in the order a
lone instance has, so every instance must equal, bit for bit, a context made
by quapi_create on its own eta with the same bucket depth (rho(t), counters
and stored groups), and through it the oracle.
"""
import numpy as np
import pytest

import oracle
from golden_runs import GoldenRun, check_fingerprint, check_stats
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


def _etas(Q, wl, baths, K):
    """One eta table per bath from the library's generator (pinned against the
    oracle's quadrature in the CPU tests); both sides of every comparison here
    take the same tables."""
    return np.stack([Q.quapi_eta(b.ohmic_alpha, b.ohmic_wc, [x for pk in b.peaks for x in pk], wl.beta, wl.dt, K)
                     for b in baths])


def _singles_like(Q, monkeypatch, g, wl, etas, K, mode, **kw):
    """Lone contexts with the batch's bucket depth (the batched form caps a
    super-bucket count per instance at 4096 / P)."""
    monkeypatch.setenv("QUAPI_MAX_SUPER", str(4096 // (wl.M * wl.M)))
    return [Q.Propagator(wl.H, wl.q, wl.dt, K, e, wl.rho0, mask=wl.mask, theta=wl.theta, mode=mode,
                         merge=Q.QUAPI_MERGE_BUCKETED, **kw)
            for e in etas]


def _assert_same(Q, g, singles, n, insts=None):
    for j, s in enumerate(singles):
        inst = j if insts is None else insts[j]
        rb, rs = g.rho_history(inst, 0, n + 1), s.rho_history(0, n + 1)
        assert np.array_equal(rb, rs), (inst, np.abs(rb - rs).max())
        assert g.stats(inst, 1, n) == s.stats(1, n), inst
        hb, wb = g.groups(inst)
        hs, ws = s.groups()
        assert np.array_equal(hb, hs) and np.array_equal(wb, ws), inst


@pytest.mark.parametrize("mode", ["pre", "post"])
def test_batch_equals_lone_instances(Q, monkeypatch, mode):
    wl, baths = W.batched_scan(n_inst=5, seed=3, K=12, n_exact=6, theta=1e-7)
    K, n = 12, 60
    etas = _etas(Q, wl, baths, K)
    mq = Q.QUAPI_PRE if mode == "pre" else Q.QUAPI_POST
    print(f"[batch] 5 instances K={K} mode={mode} n={n}", flush=True)
    g = Q.BatchPropagator(wl.H, wl.q, wl.dt, K, etas, wl.rho0, mask=wl.mask, theta=wl.theta, mode=mq)
    assert g.info()["n_instances"] == 5
    singles = _singles_like(Q, monkeypatch, g, wl, etas, K, mq)
    g.step(n)
    for s in singles:
        s.step(n)
    _assert_same(Q, g, singles, n)
    # and the oracle, for two of them
    for j in (0, 3):
        o = oracle.Oracle(wl.H, wl.q, wl.dt, K, etas[j], wl.rho0, mask=wl.mask, theta=wl.theta,
                          mode=oracle.PRE if mode == "pre" else oracle.POST)
        o.step(n)
        assert sum(o.stats(t)["n_amb_rep"] + o.stats(t)["n_amb_theta"] for t in range(1, n + 1)) == 0
        assert np.abs(g.rho_history(j, 0, n + 1) - o.rho_history()).max() < RHO_TOL


def test_batch_uneven_instances(Q, monkeypatch):
    """Instances of very different size: a strongly coupled bath (few groups
    survive theta) beside weakly coupled ones, and chunk-sized instances."""
    wl, _ = W.batched_scan(n_inst=1, K=14, n_exact=9, theta=1e-5)
    K, n = 14, 30
    baths = [W.BathSpec(a, 5.0, ((w0, gam, lam),)) for a, w0, gam, lam in
             [(0.05, 1.0, 0.05, 0.1), (2.0, 1.0, 0.05, 2.0), (0.01, 0.5, 0.1, 0.01), (0.5, 2.0, 0.02, 0.5)]]
    etas = _etas(Q, wl, baths, K)
    print(f"[batch] uneven instances K={K} n={n}", flush=True)
    g = Q.BatchPropagator(wl.H, wl.q, wl.dt, K, etas, wl.rho0, mask=wl.mask, theta=wl.theta)
    singles = _singles_like(Q, monkeypatch, g, wl, etas, K, Q.QUAPI_PRE)
    g.step(n)
    for s in singles:
        s.step(n)
    sizes = [g.stats(j, n, 1)[0]["n_groups"] for j in range(4)]
    print(f"[batch] groups per instance at step {n}: {sizes}", flush=True)
    assert max(sizes) > 4 * min(sizes)
    _assert_same(Q, g, singles, n)


def test_batch_full_size_sampled(Q, monkeypatch):
    """64 instances of the structured bath (dk_max 24, lags 0..11, theta 1e-8)
    as the benchmark runs them, for the whole 1000 steps; three sampled
    instances against lone contexts bit for bit, and instance 37 against the
    stored oracle run of its bath point at every step (rho(t), counters) and
    its group sets up to step 100 and every tenth step after."""
    wl, baths = W.batched_scan(n_inst=64)
    K, n = wl.K, wl.n_steps
    etas = _etas(Q, wl, baths, K)
    gold = GoldenRun("batched_scan_37")
    assert gold.steps == n and gold.ambiguous(n) == 0
    etas[37] = gold.eta                     # the oracle's coefficients for the stored instance
    print(f"[batch] 64 instances K={K} n={n}", flush=True)
    g = Q.BatchPropagator(wl.H, wl.q, wl.dt, K, etas, wl.rho0, mask=wl.mask, theta=wl.theta)
    pick = [0, 37, 63]
    singles = _singles_like(Q, monkeypatch, g, wl, etas[pick], K, Q.QUAPI_PRE)
    t = 0
    for tf in [s for s in range(1, n + 1) if s <= 100 or s % 10 == 0 or s == n]:
        g.step(tf - t)
        t = tf
        check_fingerprint(g.groups(37), gold, tf, RHO_TOL)
    g.sync()
    for s in singles:
        s.step(n)
        s.sync()
    _assert_same(Q, g, singles, n, insts=pick)
    total = sum(g.stats(j, n, 1)[0]["n_groups"] for j in range(64))
    print(f"[batch] groups at step {n}, all instances: {total}", flush=True)
    for j in range(64):
        assert abs(np.trace(g.rho_history(j, n, 1)[0]).real - 1.0) < 1e-2
    err = np.abs(g.rho_history(37, 0, n + 1) - gold.rho).max()
    print(f"[batch] instance 37: max |drho| over {n} steps = {err:.3e}", flush=True)
    assert err < RHO_TOL
    check_stats(g.stats(37, 1, n), gold)


def test_batch_capacity_overflow_and_reset(Q):
    # lags 0..7 exact: 4^7 keys per instance over 4^5 buckets of one group each
    wl, baths = W.batched_scan(n_inst=3, K=12, n_exact=8, theta=0.0)
    K = 12
    etas = _etas(Q, wl, baths, K)
    g = Q.BatchPropagator(wl.H, wl.q, wl.dt, K, etas, wl.rho0, mask=wl.mask, theta=0.0, max_groups=1024)
    g.step(12)
    with pytest.raises(Q.QuapiError) as e:
        g.sync()
    assert e.value.code == Q.QUAPI_ENOMEM
    t = Q.quapi_time(g.ctx)
    for j in range(3):
        o = oracle.Oracle(wl.H, wl.q, wl.dt, K, etas[j], wl.rho0, mask=wl.mask, theta=0.0, mode=oracle.PRE)
        o.step(t)
        assert np.abs(g.rho_history(j, 0, t + 1) - o.rho_history()).max() < RHO_TOL
        # every instance keeps the groups of the last complete step
        assert sum(o.stats(k)["n_amb_rep"] for k in range(1, t + 1)) == 0
        ho, wo = o.groups()
        hg, wg = g.groups(j)
        assert ho.shape == hg.shape, (j, ho.shape, hg.shape)
        io, ig = np.lexsort(ho.T[::-1]), np.lexsort(hg.T[::-1])
        assert np.array_equal(ho[io], hg[ig])
        assert np.abs(wo[io] - wg[ig]).max() < RHO_TOL
    g.reset()
    g.step(3)
    o = oracle.Oracle(wl.H, wl.q, wl.dt, K, etas[1], wl.rho0, mask=wl.mask, theta=0.0, mode=oracle.PRE)
    o.step(3)
    assert np.abs(g.rho_history(1, 0, 4) - o.rho_history()).max() < RHO_TOL


def test_chunk_runs_and_autotune_leave_results_unchanged(Q):
    """Chunk run lengths change which workgroup takes which chunk, not what a
    chunk computes: every run length gives the same bits."""
    wl, baths = W.batched_scan(n_inst=6, seed=5, K=12, n_exact=7, theta=1e-7)
    K, n = 12, 50
    etas = _etas(Q, wl, baths, K)
    g = Q.BatchPropagator(wl.H, wl.q, wl.dt, K, etas, wl.rho0, mask=wl.mask, theta=wl.theta)
    ref = None
    for run in (1, 3, 16):
        g.reset()
        g.set_chunk_run(run)
        g.step(n)
        r = g.rho_all(0, n + 1)
        assert r.shape == (n + 1, 6, 2, 2)
        for j in (0, 5):
            assert np.array_equal(r[:, j], g.rho_history(j, 0, n + 1))
        if ref is None:
            ref = (r, [g.groups(j) for j in range(6)])
        else:
            assert np.array_equal(r, ref[0]), run
            for j in range(6):
                h, w = g.groups(j)
                assert np.array_equal(h, ref[1][j][0]) and np.array_equal(w, ref[1][j][1])
    best = g.autotune(20)
    assert best in (1, 2, 4, 8, 16)
    assert g.t == 0
    g.step(n)
    assert np.array_equal(g.rho_all(0, n + 1), ref[0])


def test_batch_per_instance_hamiltonians(Q, monkeypatch):
    """Instances that differ in the bias eps of H_S as well as in the bath."""
    wl, baths = W.batched_scan(n_inst=4, seed=8, K=12, n_exact=6, theta=1e-7)
    K, n = 12, 50
    etas = _etas(Q, wl, baths, K)
    Hs = np.stack([W.tls_hamiltonian(eps, 1.0) for eps in (0.0, 0.5, 1.0, -0.7)])
    print(f"[batch] 4 instances with their own H_S K={K} n={n}", flush=True)
    g = Q.BatchPropagator(wl.H, wl.q, wl.dt, K, etas, wl.rho0, mask=wl.mask, theta=wl.theta, H_batch=Hs)
    monkeypatch.setenv("QUAPI_MAX_SUPER", "1024")
    singles = [Q.Propagator(Hs[j], wl.q, wl.dt, K, etas[j], wl.rho0, mask=wl.mask, theta=wl.theta,
                            merge=Q.QUAPI_MERGE_BUCKETED)
               for j in range(4)]
    g.step(n)
    for s in singles:
        s.step(n)
    _assert_same(Q, g, singles, n)
    o = oracle.Oracle(Hs[3], wl.q, wl.dt, K, etas[3], wl.rho0, mask=wl.mask, theta=wl.theta, mode=oracle.PRE)
    o.step(n)
    assert np.abs(g.rho_history(3, 0, n + 1) - o.rho_history()).max() < RHO_TOL


def test_batch_of_one_equals_lone_context(Q, monkeypatch):
    """The batched planner and layout with a single instance (one closing list
    entry, the lone step kernel)."""
    wl, baths = W.batched_scan(n_inst=1, seed=4, K=12, n_exact=6, theta=1e-7)
    K, n = 12, 40
    etas = _etas(Q, wl, baths, K)
    g = Q.BatchPropagator(wl.H, wl.q, wl.dt, K, etas, wl.rho0, mask=wl.mask, theta=wl.theta)
    assert g.info()["n_instances"] == 1
    singles = _singles_like(Q, monkeypatch, g, wl, etas, K, Q.QUAPI_PRE)
    g.step(n)
    singles[0].step(n)
    _assert_same(Q, g, singles, n)


def test_batch_three_level(Q, monkeypatch):
    """Three levels (9 pairs, 4-bit points): the seeded random H_S with
    q = (+1, 0, -1), dk_max 16, lags 0..5 exact, at five bath points (peak
    frequency and width varied), against lone contexts and the oracle."""
    wl = W.three_level(K=16, n_exact=6, theta=1e-8)
    K, n = 16, 30
    baths = [W.BathSpec(wl.bath.ohmic_alpha, wl.bath.ohmic_wc, ((w0, gam, 0.1),))
             for w0, gam in [(1.0, 0.05), (0.5, 0.02), (2.0, 0.1), (1.4, 0.05), (0.8, 0.1)]]
    etas = _etas(Q, wl, baths, K)
    print(f"[batch] three-level, 5 instances K={K} n={n}", flush=True)
    g = Q.BatchPropagator(wl.H, wl.q, wl.dt, K, etas, wl.rho0, mask=wl.mask, theta=wl.theta)
    assert g.info()["n_instances"] == 5
    singles = _singles_like(Q, monkeypatch, g, wl, etas, K, Q.QUAPI_PRE)
    g.step(n)
    for s in singles:
        s.step(n)
    _assert_same(Q, g, singles, n)
    for j in (1, 4):
        o = oracle.Oracle(wl.H, wl.q, wl.dt, K, etas[j], wl.rho0, mask=wl.mask, theta=wl.theta, mode=oracle.PRE)
        o.step(n)
        assert sum(o.stats(t)["n_amb_rep"] + o.stats(t)["n_amb_theta"] for t in range(1, n + 1)) == 0
        assert np.abs(g.rho_history(j, 0, n + 1) - o.rho_history()).max() < RHO_TOL
