"""The FP32 precision form (QUAPI_FP32_LOG) against the FP64 oracle.

The form stores each group amplitude as FP32 (ln|w|, arg w) and forms each
child's influence exponent and amplitude in FP32; the merge sums, eta and the
rho(t) sums stay FP64.  It is not bit-exact: each child carries FP32 rounding
(relative ~1e-7, times |ln|w|| for the magnitude), and the filter and
representative decisions that sit within that rounding of their thresholds may
go the other way.  The form therefore compares 12 mantissa bits of |w|^2 by
default (qbits = 40): with the FP64 form's 20 (qbits = 32), values that tie
exactly split across quanta under FP32 rounding and change the representative.
The reference here is the oracle at the same qbits.  The bar is 1e-5 absolute
on every rho(t) element, the target the precision form is built to; the
measured error of each case is printed.
"""
import numpy as np
import pytest

import oracle
from paper_2506_03127_amd import workloads as W

pytestmark = pytest.mark.gpu

FP32_RHO_TOL = 1e-5
FP32_QBITS = 40


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_03127_amd import quapi
    quapi.lib()
    return quapi


@pytest.mark.parametrize("store", ["HASH", "PARTITION"])
@pytest.mark.parametrize("make,mode,K,mask,theta,n", [
    # the plain method: no mask, no filter
    (lambda K: W.spin_boson_ohmic(), "pre", 8, None, 0.0, 100),
    # contiguous masks (the FP64 form runs these on the bucketed store)
    (W.structured_bath, "pre", 12, tuple(range(6)), 1e-7, 60),
    (W.structured_bath, "post", 10, tuple(range(5)), 1e-7, 40),
    # masks that keep distant lags, one- and two-word histories
    (W.structured_bath, "pre", 24, tuple(range(12)) + (15, 19, 23), 1e-8, 16),
    (W.structured_bath, "pre", 40, tuple(range(12)) + (16, 24, 32), 1e-9, 12),
    (W.three_level, "pre", 8, (0, 1, 2, 5, 7), 1e-7, 25),
], ids=["spin-boson-K8", "structured-K12-E6", "structured-K10-post", "K24-tail", "K40-lags-16-24-32",
        "three-level-K8"])
def test_fp32_form_against_oracle(Q, eta_cache, store, make, mode, K, mask, theta, n):
    check_fp32_against_oracle(Q, eta_cache, store, make, mode, K, mask, theta, n)


# two-level masks whose merge positions are 0..L-1 with 6 <= L <= 12: the
# precision form runs them on the direct-mapped store
@pytest.mark.parametrize("make,mode,K,mask,theta,n", [
    (lambda K: W.spin_boson_ohmic(), "pre", 8, None, 0.0, 100),
    (W.structured_bath, "pre", 12, tuple(range(8)), 1e-7, 60),
    (W.structured_bath, "post", 10, tuple(range(6)), 1e-7, 40),
    (W.structured_bath, "pre", 12, tuple(range(9)), 1e-8, 40),
], ids=["spin-boson-K8", "structured-K12-E8", "structured-K10-post-E6", "structured-K12-E9"])
def test_fp32_direct_store_against_oracle(Q, eta_cache, make, mode, K, mask, theta, n):
    check_fp32_against_oracle(Q, eta_cache, "DIRECT", make, mode, K, mask, theta, n)


def check_fp32_against_oracle(Q, eta_cache, store, make, mode, K, mask, theta, n):
    wl = make(K=K)
    eta = eta_cache(wl, K)
    mo = oracle.PRE if mode == "pre" else oracle.POST
    mq = Q.QUAPI_PRE if mode == "pre" else Q.QUAPI_POST
    print(f"[fp32] M={wl.H.shape[0]} K={K} mode={mode} mask={mask} theta={theta} n={n} store={store}", flush=True)
    o = oracle.Oracle(wl.H, wl.q, wl.dt, K, eta, wl.rho0, mask=mask, theta=theta, mode=mo,
                      qbits=FP32_QBITS)
    g = Q.Propagator(wl.H, wl.q, wl.dt, K, eta, wl.rho0, mask=mask, theta=theta, mode=mq,
                     precision=Q.QUAPI_FP32_LOG, merge=getattr(Q, f"QUAPI_MERGE_{store}"))
    info = g.info()
    assert info["precision"] == Q.QUAPI_FP32_LOG and info["hash_merge"] == (0 if store == "DIRECT" else 1)
    assert info["store"] == getattr(Q, f"QUAPI_MERGE_{store}")
    o.step(n)
    g.step(n)
    got = g.rho_history(0, n + 1)
    want = o.rho_history()
    err = np.abs(got - want).max()
    print(f"[fp32] max |drho| = {err:.3e}", flush=True)
    assert err < FP32_RHO_TOL
    # group counts: only decisions within FP32 rounding of a threshold may differ
    gs = g.stats(1, n)
    for t in range(1, n + 1):
        a, b = gs[t - 1]["n_groups"], o.stats(t)["n_groups"]
        assert abs(a - b) <= max(2, 1e-3 * b), (t, a, b)
    # stored amplitudes against the oracle's, matched by history
    ho, wo = o.groups()
    hg, wg = g.groups()
    ref = {bytes(h): w for h, w in zip(ho, wo)}
    common = [(ref[bytes(h)], w) for h, w in zip(hg, wg) if bytes(h) in ref]
    assert len(common) >= 0.999 * len(ho)
    d = np.array([abs(a - b) / max(abs(a), 1e-300) for a, b in common])
    print(f"[fp32] groups {len(hg)} vs {len(ho)}, median rel |dw| = {np.median(d):.2e}", flush=True)
    assert np.median(d) < 1e-5


@pytest.mark.parametrize("store,n", [("DIRECT", 1000), ("PARTITION", 200)])
def test_fp32_form_against_fp64_form(Q, eta_cache, store, n):
    """Both forms on the same GPU, on the structured bath at dk_max = 24 with lags
    0..11 kept (the FP64 form on the direct-mapped store), both comparing 12
    mantissa bits for the representative: the FP32 form on the direct-mapped
    store over the whole 1000-step run, and on the hash-table store (partition
    merge) over 200 steps."""
    wl = W.structured_bath()
    eta = eta_cache(wl, wl.K)
    kw = dict(mask=wl.mask, theta=wl.theta, max_steps=n)
    g64 = Q.Propagator(wl.H, wl.q, wl.dt, wl.K, eta, wl.rho0, qbits=FP32_QBITS, **kw)
    g32 = Q.Propagator(wl.H, wl.q, wl.dt, wl.K, eta, wl.rho0, precision=Q.QUAPI_FP32_LOG,
                       max_groups=4 << 20, merge=getattr(Q, f"QUAPI_MERGE_{store}"), **kw)
    assert g64.info()["store"] == Q.QUAPI_MERGE_DIRECT
    assert g32.info()["store"] == getattr(Q, f"QUAPI_MERGE_{store}")
    g64.step(n)
    g32.step(n)
    r64 = g64.rho_history(0, n + 1)
    r32 = g32.rho_history(0, n + 1)
    err = np.abs(r32 - r64).max()
    print(f"[fp32] {store}, {n} steps, max |drho| FP32 form vs FP64 form = {err:.3e}", flush=True)
    assert err < FP32_RHO_TOL
    s64, s32 = g64.stats(1, n), g32.stats(1, n)
    assert all(abs(a["n_groups"] - b["n_groups"]) <= max(2, 1e-3 * a["n_groups"]) for a, b in zip(s64, s32))


def test_long_memory_fp64_spread_over_qbits_and_the_fp32_form(Q, eta_cache):
    """The long-memory workload (dk_max 40, lags 0..11, 16, 24 and 32 exact,
    theta 1e-9) for 200 steps: its FP64 answer itself depends on how finely the
    representative's |w|^2 is compared (Sec. 3.1.2; reading A10), because a
    flipped representative carries other points in its tail.  This records that
    spread over qbits 32, 40 and 44 and states the FP32 form's difference from
    the FP64 form (both at qbits 40) against it: on this workload the 1e-5 bar of
    the precision form cannot be judged by rho(t), the method's own sensitivity
    being far larger."""
    wl = W.long_memory()
    eta = eta_cache(wl, wl.K)
    n = 200
    kw = dict(mask=wl.mask, theta=wl.theta, max_steps=n, max_groups=48 << 20)
    r64 = {}
    for qb in (32, 40, 44):
        g = Q.Propagator(wl.H, wl.q, wl.dt, wl.K, eta, wl.rho0, qbits=qb, **kw)
        g.step(n)
        r64[qb] = g.rho_history(0, n + 1)
        g.close()
    g = Q.Propagator(wl.H, wl.q, wl.dt, wl.K, eta, wl.rho0, qbits=FP32_QBITS, precision=Q.QUAPI_FP32_LOG, **kw)
    g.step(n)
    r32 = g.rho_history(0, n + 1)
    g.close()
    spread = max(np.abs(r64[a] - r64[b]).max() for a in r64 for b in r64)
    d32 = np.abs(r32 - r64[FP32_QBITS]).max()
    print(f"[fp32] long memory, {n} steps: FP64 spread over qbits 32/40/44 = {spread:.3e}; "
          f"FP32 form vs FP64 form at qbits {FP32_QBITS} = {d32:.3e}; "
          f"|drho(qbits 32 vs 40)| = {np.abs(r64[32] - r64[40]).max():.3e}, "
          f"|drho(44 vs 40)| = {np.abs(r64[44] - r64[40]).max():.3e}", flush=True)
    # the method's own sensitivity to the quantisation is far above the precision
    # form's bar, and the FP32 form's difference is of that order, not above it
    assert spread > 100 * FP32_RHO_TOL
    assert d32 < 3.0 * spread


def test_fp32_direct_store_is_deterministic(Q, eta_cache):
    """The precision form on the direct-mapped store sums rho(t) and the
    counters in a fixed order: two contexts, and one of them after a reset,
    give the same bits."""
    wl = W.structured_bath(K=12, n_exact=8, theta=1e-7)
    eta = eta_cache(wl, 12)
    n = 60
    mk = lambda: Q.Propagator(wl.H, wl.q, wl.dt, 12, eta, wl.rho0, mask=wl.mask, theta=wl.theta,
                              precision=Q.QUAPI_FP32_LOG)
    a, b = mk(), mk()
    assert a.info()["store"] == Q.QUAPI_MERGE_DIRECT
    a.step(n)
    b.step(n)
    ra = a.rho_history(0, n + 1)
    assert np.array_equal(ra, b.rho_history(0, n + 1))
    assert a.stats(1, n) == b.stats(1, n)
    b.reset()
    b.step(n)
    assert np.array_equal(ra, b.rho_history(0, n + 1))
    ha, wa = a.groups()
    hb, wb = b.groups()
    assert np.array_equal(ha, hb) and np.array_equal(wa, wb)
