"""The stored oracle runs and their fingerprints (no GPU): a fingerprint does
not depend on the order of the groups and changes with any history or a
perturbed amplitude; each stored run starts as the oracle computes it now and
keeps the bookkeeping of the method at every stored step."""
import os

import numpy as np
import pytest

import oracle
from golden_runs import GoldenRun, check_fingerprint, fingerprint_of
from paper_2506_03127_amd import workloads as W
from fingerprint import compare


def test_fingerprint_order_and_sensitivity():
    rng = np.random.default_rng(3)
    h = rng.integers(0, 4, (500, 12)).astype(np.uint8)
    h = np.unique(h, axis=0)
    w = rng.normal(size=len(h)) * 1e-3 + 1j * rng.normal(size=len(h)) * 1e-3
    fp = fingerprint_of(h, w)
    perm = rng.permutation(len(h))
    assert compare(fingerprint_of(h[perm], w[perm]), fp, 1e-15) == ""
    h2 = h.copy()
    h2[17, 11] ^= 1
    assert compare(fingerprint_of(h2, w), fp, 1e-12) == "history sets differ"
    w2 = w.copy()
    w2[5] += 1e-9
    assert "differ" in compare(fingerprint_of(h, w2), fp, 1e-12)
    assert "count" in compare(fingerprint_of(h[:-1], w[:-1]), fp, 1e-12)


RUNS = [("structured_bath", lambda: W.structured_bath(), 14),
        ("batched_scan_37", lambda: W.batched_scan(n_inst=64)[0], 14),
        ("long_memory", lambda: W.long_memory(), 10)]


@pytest.mark.parametrize("name,make,n", RUNS, ids=[r[0] for r in RUNS])
def test_stored_run_starts_as_the_oracle(oracle_mod, name, make, n):
    if not GoldenRun.exists(name):
        pytest.skip(f"stored run {name} not present")
    gold = GoldenRun(name)
    wl = make()
    o = oracle.Oracle(wl.H, wl.q, wl.dt, wl.K, gold.eta, wl.rho0, mask=wl.mask, theta=wl.theta,
                      mode=oracle.PRE)
    for t in range(1, n + 1):
        o.step(1)
        check_fingerprint(o.groups(), gold, t, 0.0)
        s = o.stats(t)
        for k in ("n_groups", "n_children", "n_survivors", "n_stored", "n_amb_rep", "n_amb_theta"):
            assert s[k] == gold.stats[t][k], (t, k)
    assert np.array_equal(o.rho_history(), gold.rho[:n + 1])
    # bookkeeping at every stored step
    # (pre-merging stores the survivors and merges them at the next step)
    for t in range(1, gold.steps + 1):
        s = gold.stats[t]
        assert s["n_children"] == wl.M ** 2 * s["n_groups"]
        assert s["n_stored"] == s["n_survivors"] <= s["n_children"]
        if t > 1:
            assert s["n_groups"] <= gold.stats[t - 1]["n_stored"]
    # (the merge is an approximation: with a mask that keeps distant lags exact the
    # representatives of a path and of its mirror need not be mirrors, and Tr rho
    # picks up an imaginary part of ~1e-7; only a loose bound holds)
    tr = np.trace(gold.rho, axis1=1, axis2=2)
    assert np.isfinite(gold.rho).all() and np.abs(tr).max() < 1.01
