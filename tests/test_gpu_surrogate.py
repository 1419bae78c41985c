"""The learned surrogate (paper_2506_03127_amd.surrogate): trained on the
batched propagation with the library's network kernels, validated per cell
of the (w0, gamma) plane on held-out points, and falling back to the method
wherever its held-out error exceeds the tolerance.

The network reaches held-out errors of a few 1e-2 in rho(t) on this machine (the
loss plateaus near 1e-4 with bf16 hidden products), so at the 1e-3 tolerance
every query goes to the method; at a tolerance it does meet, the accepted
cells are answered by the network within it, far faster than the method.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_03127_amd import surrogate as S
    sur = S.Surrogate(solver=S.Solver(n_steps=50))
    pts = sur.box.sample(448, seed=21)
    print("[surrogate] solving 448 points x 50 steps", flush=True)
    rho = sur.solver.solve(pts)
    train, held = slice(0, 384), slice(384, 448)
    print("[surrogate] training", flush=True)
    sur.fit(pts[train], rho[train], steps=2000, batch=4096)
    err = sur.validate(pts[held], rho[held])
    print(f"[surrogate] loss {sur.history['loss'][-1]}, held-out error median {np.median(err):.3e} "
          f"max {err.max():.3e}", flush=True)
    return S, sur, pts[held], rho[held], err


def test_network_learns(trained):
    S, sur, pts, rho, err = trained
    first, last = sur.history["loss"][0][1], sur.history["loss"][-1][1]
    assert last < first / 100
    assert np.median(err) < 0.1


def test_fallback_at_the_strict_tolerance_is_the_method(trained):
    S, sur, pts, rho, err = trained
    sur.tol = 1e-3
    sur.validate(pts, rho)
    q = pts[:16]
    got, used = sur.query(q)
    # cells whose held-out error exceeds 1e-3 send their queries to the method
    for j in range(len(q)):
        cw, cg = sur._cell(q[j:j + 1])
        assert used[j] == bool(sur.accepted[cw[0], cg[0]])
    assert np.array_equal(got[~used], sur.solver.solve(q[~used]))
    # points outside the box always go to the method
    out = q[:2].copy()
    out[:, 0] = 3.0
    _, used_out = sur.query(out)
    assert not used_out.any()


def test_gain_where_the_network_is_accepted(trained):
    S, sur, pts, rho, err = trained
    sur.tol = float(np.nanmax(sur.cell_error)) * 1.01          # a tolerance the network meets everywhere
    sur.validate(pts, rho)
    assert sur.accepted.all()
    q = pts[:64]
    t0 = time.perf_counter()
    got, used = sur.query(q)
    t_net = time.perf_counter() - t0
    assert used.all()
    assert np.abs(got - rho[:64]).max() <= sur.tol
    t0 = time.perf_counter()
    ref = sur.solver.solve(q)
    t_method = time.perf_counter() - t0
    print(f"[surrogate] 64 points x 51 times: network {1e3 * t_net:.1f} ms, method {1e3 * t_method:.1f} ms "
          f"({t_method / t_net:.0f}x), max |drho| {np.abs(got - ref).max():.3e} within tol {sur.tol:.3e}",
          flush=True)
    assert t_method > 10 * t_net
