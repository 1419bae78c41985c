"""Host logic of the surrogate (no GPU): the bath-free baseline, the box and
its validation cells, and the packing of rho(t)."""
import numpy as np
import scipy.linalg as sl

from paper_2506_03127_amd import surrogate as S
from paper_2506_03127_amd import workloads as W


def test_free_evolution_is_the_unitary_propagation():
    pts = np.array([[1.0, 0.05, 0.07, 0.05, e] for e in (0.0, 0.3, 0.75, -0.4)])
    rho0 = np.array([[0.7, 0.2 - 0.1j], [0.2 + 0.1j, 0.3]])
    got = S.free_evolution(pts, 9, 0.2, rho0)
    for j, e in enumerate(pts[:, 4]):
        H = W.tls_hamiltonian(e, 1.0)
        for k in range(9):
            U = sl.expm(-1j * H * 0.2 * k)
            assert np.abs(got[j, k] - U @ rho0 @ U.conj().T).max() < 1e-14
    # trace and hermiticity are kept
    assert np.abs(np.trace(got, axis1=2, axis2=3) - 1.0).max() < 1e-14
    assert np.abs(got - np.conj(np.swapaxes(got, -1, -2))).max() < 1e-15


def test_components_round_trip():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(5, 3, 2, 2)) + 1j * rng.normal(size=(5, 3, 2, 2))
    rho = a @ np.conj(np.swapaxes(a, -1, -2))             # Hermitian
    c = S.rho_components(rho)
    assert c.shape == (5, 3, 4)
    assert np.allclose(c[..., 0], rho[..., 0, 0].real) and np.allclose(c[..., 3], rho[..., 1, 1].real)
    assert np.allclose(c[..., 1] + 1j * c[..., 2], rho[..., 0, 1])


def test_box_and_cells():
    box = S.Box()
    pts = box.sample(2000, seed=1)
    assert box.contains(pts).all()
    lo, hi = box.lo_hi()
    assert (pts.min(axis=0) >= lo).all() and (pts.max(axis=0) <= hi).all()
    out = pts[:3].copy()
    out[0, 0] = hi[0] + 0.1
    out[1, 4] = lo[4] - 0.1
    assert list(box.contains(out)) == [False, False, True]
    sur = S.Surrogate(box=box)
    cw, cg = sur._cell(pts)
    assert cw.min() == 0 and cw.max() == sur.cells[0] - 1 and cg.min() == 0 and cg.max() == sur.cells[1] - 1
    # the corners land in the corner cells
    cw, cg = sur._cell(np.array([lo, hi]))
    assert (cw[0], cg[0]) == (0, 0) and (cw[1], cg[1]) == (sur.cells[0] - 1, sur.cells[1] - 1)
    # features span [-1, 1], time last
    f = sur._features(np.array([lo, hi]), sur.solver.n_steps + 1)
    assert np.allclose(f[0, :, :5], -1) and np.allclose(f[1, :, :5], 1)
    assert f[0, 0, 5] == -1 and f[0, -1, 5] == 1


class _Stub(S.Solver):
    def solve(self, pts, progress=False, n_steps=None):
        n = self.n_steps if n_steps is None else n_steps
        return np.full((len(pts), n + 1, 2, 2), 7.0 + 0j)


def test_untrained_surrogate_sends_everything_to_the_method():
    sur = S.Surrogate(solver=_Stub(n_steps=4))
    got, used = sur.query(sur.box.sample(3, seed=2))
    assert not used.any() and np.all(got == 7.0)
    got, used = sur.query(sur.box.sample(3, seed=2), t_max=2)
    assert not used.any() and got.shape == (3, 3, 2, 2)


def test_time_windows_and_horizons():
    sur = S.Surrogate(solver=_Stub(n_steps=50), windows=5)
    # equal spans of ten steps, the last one closed at step 50
    assert list(sur._window(np.array([0, 9, 10, 39, 40, 49, 50]))) == [0, 0, 1, 3, 4, 4, 4]
    pts = sur.box.sample(400, seed=3)
    cw, cg = sur._cell(pts)
    # accept windows 0 and 1 of cell (0, 0), and every window of cell (1, 1)
    sur.accepted = np.zeros(sur.cells + (sur.windows,), dtype=bool)
    sur.accepted[0, 0, :2] = True
    sur.accepted[1, 1, :] = True
    for t_max, want in ((5, ((0, 0), (1, 1))), (19, ((0, 0), (1, 1))), (20, ((1, 1),)), (50, ((1, 1),))):
        use = sur.answers(pts, t_max)
        expect = np.zeros(len(pts), dtype=bool)
        for a, b in want:
            expect |= (cw == a) & (cg == b)
        assert np.array_equal(use, expect), t_max
    # outside the box: never the network
    out = pts[:1].copy()
    out[0, 1] = 1.0
    assert not sur.answers(out, 5).any()
    try:
        sur.query(pts[:1], t_max=51)
        assert False
    except ValueError:
        pass
