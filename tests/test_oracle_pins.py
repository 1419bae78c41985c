"""Pins of the FP64 path-propagation oracle against closed forms, invariants,
special cases and brute force (Sec. 2 eqs. quapi_red_rho, SysP, inf_fun;
Sec. 2.1 merging and filtering; Sec. 3.1 pre-merging)."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from oracle.brute import brute_rho
from oracle.eta import Bath, eta_columns, g_of_t
from paper_2506_03127_amd import workloads as W

PRE, POST = oracle.PRE, oracle.POST


def ohmic_eta(K, dt=0.25, alpha=0.1, wc=5.0, beta=5.0):
    return eta_columns(Bath(alpha, wc), beta, dt, K)


def structured_eta(K, dt=0.2):
    return eta_columns(Bath(0.05, 5.0, ((1.0, 0.05, 0.1),)), 5.0, dt, K)


# ----------------------------------------------------------------- propagator
def test_propagator_matches_expm_and_is_unitary(oracle_mod):
    for M, seed in [(2, 1), (3, 2), (4, 3)]:
        H = W.random_hermitian(M, 0.8, seed)
        U = oracle.propagator(H, 0.37)
        assert np.abs(U - expm(-0.37j * H)).max() < 1e-14
        assert np.abs(U @ U.conj().T - np.eye(M)).max() < 1e-14


# ----------------------------------------------------------------- Rabi (eta = 0)
@pytest.mark.parametrize("mode", [PRE, POST])
@pytest.mark.parametrize("mask", [None, (0, 1, 2), (0, 1, 3)])
def test_rabi_closed_form_zero_coupling(oracle_mod, mode, mask):
    K, dt, N = 5, 0.25, 30
    eta = np.zeros((3, K + 1), dtype=complex)
    for eps in (0.0, 0.7):
        H = W.tls_hamiltonian(eps, 1.0)
        o = oracle.Oracle(H, [1, -1], dt, K, eta, W.ground_projector(2), mask=mask, mode=mode)
        o.step(N)
        Om = math.hypot(eps, 1.0)
        for t in range(N + 1):
            r = o.rho(t)
            pflip = (1.0 / Om ** 2) * math.sin(Om * t * dt / 2) ** 2
            assert abs(r[1, 1].real - pflip) < 1e-13
            assert abs(r[0, 0].real - (1 - pflip)) < 1e-13
            if eps == 0.0:
                assert abs((r[0, 0] - r[1, 1]).real - math.cos(t * dt)) < 1e-13


def test_zero_coupling_three_level_unitary(oracle_mod):
    """eta = 0, random three-level H: rho(t) = U^t rho0 U^t^dagger."""
    K, dt, N = 3, 0.2, 12
    H = W.random_hermitian(3, 0.5, 11)
    rho0 = np.array([[0.5, 0.2 - 0.1j, 0], [0.2 + 0.1j, 0.3, 0.05], [0, 0.05, 0.2]], dtype=complex)
    o = oracle.Oracle(H, [1, 0, -1], dt, K, np.zeros((3, K + 1)), rho0, mode=PRE)
    o.step(N)
    U = expm(-1j * dt * H)
    r = rho0.copy()
    for t in range(N + 1):
        assert np.abs(o.rho(t) - r).max() < 1e-13
        r = U @ r @ U.conj().T


# ----------------------------------------------------------------- pure dephasing
@pytest.mark.parametrize("q,expo", [((1.0, -1.0), lambda g: -4.0 * g.real),
                                    ((1.0, 0.0), lambda g: -g)])
def test_pure_dephasing_closed_form(oracle_mod, q, expo):
    """Delta = 0: the coherence of |+><+| decays as exp(-(q0-q1)^2 Re g - i(q0^2-q1^2) Im g),
    exact while the memory covers the whole run (t <= K dt)."""
    K, dt, eps, beta = 10, 0.25, 0.6, 5.0
    bath = Bath(0.1, 5.0)
    eta = eta_columns(bath, beta, dt, K)
    rho0 = np.full((2, 2), 0.5, dtype=complex)
    for mode in (PRE, POST):
        o = oracle.Oracle(W.tls_hamiltonian(eps, 0.0), q, dt, K, eta, rho0, mode=mode)
        o.step(K)
        for t in range(1, K + 1):
            g = g_of_t(bath, beta, t * dt)
            want = 0.5 * np.exp(-1j * eps * t * dt) * np.exp(expo(g))
            assert abs(o.rho(t)[0, 1] - want) < 1e-13, (mode, t)


def test_pure_dephasing_beyond_memory(oracle_mod):
    """t > K dt: the exponent is the sum over the retained pairs (lag <= K) of the
    window-typed coefficients, taken directly from the table."""
    K, dt, eps = 4, 0.25, 0.6
    eta = ohmic_eta(K, dt)
    rho0 = np.full((2, 2), 0.5, dtype=complex)
    o = oracle.Oracle(W.tls_hamiltonian(eps, 0.0), [1, -1], dt, K, eta, rho0, mode=POST)
    N = 11
    o.step(N)
    for t in range(K + 1, N + 1):
        s = 2 * eta[1, 0] + (t - 1) * eta[0, 0]
        for d in range(1, K + 1):
            s += 2 * eta[1, d] + max(0, t - 1 - d) * eta[0, d]
        want = 0.5 * np.exp(-1j * eps * t * dt) * np.exp(-4.0 * s.real)
        assert abs(o.rho(t)[0, 1] - want) < 1e-13


# ----------------------------------------------------------------- brute force
@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_post_full_mask_equals_brute_force(oracle_mod, K):
    """iQUAPI with the full mask and no filter is the memory-truncated path sum, at every N."""
    eta = ohmic_eta(K)
    H = W.tls_hamiltonian(0.3, 1.0)
    rho0 = np.array([[0.7, 0.1 + 0.2j], [0.1 - 0.2j, 0.3]])
    o = oracle.Oracle(H, [1, -1], 0.25, K, eta, rho0, mode=POST)
    o.step(7)
    for N in range(8):
        assert np.abs(o.rho(N) - brute_rho(H, [1, -1], 0.25, K, eta, rho0, N)).max() < 5e-15 * 4 ** 0 + 1e-14


def test_three_level_post_full_mask_brute_force(oracle_mod):
    K = 2
    H = W.random_hermitian(3, 0.5, 5)
    eta = structured_eta(K)
    rho0 = W.ground_projector(3)
    o = oracle.Oracle(H, [1, 0, -1], 0.2, K, eta, rho0, mode=POST)
    o.step(4)
    for N in range(5):
        assert np.abs(o.rho(N) - brute_rho(H, [1, 0, -1], 0.2, K, eta, rho0, N)).max() < 1e-14


def test_four_level_post_full_mask_brute_force(oracle_mod):
    """Four levels (16 forward/backward pairs): post-merging on every lag is the
    exact path sum of eq. quapi_red_rho, against brute force."""
    K = 2
    H = W.random_hermitian(4, 0.5, 9)
    q = [1.5, 0.5, -0.5, -1.5]
    eta = structured_eta(K)
    rho0 = W.ground_projector(4)
    o = oracle.Oracle(H, q, 0.2, K, eta, rho0, mode=POST)
    o.step(3)
    for N in range(4):
        assert np.abs(o.rho(N) - brute_rho(H, q, 0.2, K, eta, rho0, N)).max() < 1e-14


def test_pre_equals_brute_force_before_first_merge(oracle_mod):
    """With mask {0..E-1} the pre-merge first merges at step E+1 (when the paths
    hold more than E-1 points); before that every mode is the exact path sum."""
    K, E = 6, 3
    eta = structured_eta(K)
    H = W.tls_hamiltonian(0.5, 1.0)
    o = oracle.Oracle(H, [1, -1], 0.2, K, eta, W.ground_projector(2), mask=tuple(range(E)), mode=PRE)
    o.step(E)
    for N in range(E + 1):
        assert np.abs(o.rho(N) - brute_rho(H, [1, -1], 0.2, K, eta, W.ground_projector(2), N)).max() < 1e-14
    assert o.stats(E)["n_groups"] == 4 ** (E - 1)


def test_pre_with_zeroed_tail_equals_shorter_memory(oracle_mod):
    """eta zero beyond lag E-1: the off-mask points never act again, so pre-merging
    on {0..E-1} is exact and equals the path sum with memory E-1 (Sec. 3.1 footnote)."""
    K, E = 7, 3
    eta = structured_eta(K)
    eta[:, E:] = 0.0
    H = W.tls_hamiltonian(0.5, 1.0)
    rho0 = W.ground_projector(2)
    o = oracle.Oracle(H, [1, -1], 0.2, K, eta, rho0, mask=tuple(range(E)), mode=PRE)
    o.step(7)
    eta_short = eta[:, :E].copy()
    for N in range(8):
        assert np.abs(o.rho(N) - brute_rho(H, [1, -1], 0.2, E - 1, eta_short, rho0, N)).max() < 1e-14


# ----------------------------------------------------------------- invariants
MASKS = [None, (0, 1, 2, 3), (0, 1, 4), (0, 1, 2, 5)]


@pytest.mark.parametrize("mode", [PRE, POST])
@pytest.mark.parametrize("mask", MASKS)
def test_trace_and_hermiticity(oracle_mod, mode, mask):
    """theta = 0: merging sums every member, so Tr rho is preserved (Sec. 2.1).
    rho(t) = rho(t)^dagger holds exactly when no representative has to be chosen
    among members of equal |w| (the swapped path carries the conjugate weight):
    checked for the full mask of the post-merging form, where groups are exact."""
    K = 6
    eta = structured_eta(K)
    o = oracle.Oracle(W.tls_hamiltonian(0.5, 1.0), [1, -1], 0.2, K, eta, W.ground_projector(2),
                      mask=mask, mode=mode)
    N = 25
    o.step(N)
    for t in range(N + 1):
        r = o.rho(t)
        assert abs(np.trace(r) - 1.0) < 1e-13 * (1 + t)
        if mask is None and mode == POST:
            assert np.abs(r - r.conj().T).max() < 1e-13


def test_path_counts_full_memory(oracle_mod):
    """Full mask, no filter: the stored set reaches M^(2K) paths (Sec. 4.2 quotes
    2^28 for M = 2, K = 14); pre-merging expands M^(2(K-1)) groups into M^(2K) children."""
    K = 5
    eta = ohmic_eta(K)
    H = W.tls_hamiltonian(0.0, 1.0)
    post = oracle.Oracle(H, [1, -1], 0.25, K, eta, W.ground_projector(2), mode=POST)
    pre = oracle.Oracle(H, [1, -1], 0.25, K, eta, W.ground_projector(2), mode=PRE)
    post.step(K + 3)
    pre.step(K + 3)
    for t in range(K, K + 4):
        assert post.stats(t)["n_stored"] == 4 ** K
        assert pre.stats(t)["n_children"] == 4 ** K
        assert pre.stats(t)["n_groups"] == 4 ** (K - 1)


def test_group_count_bound_macgic(oracle_mod):
    K, E = 8, 4
    o = oracle.Oracle(W.tls_hamiltonian(0.5, 1.0), [1, -1], 0.2, K, structured_eta(K),
                      W.ground_projector(2), mask=(0, 1, 2, 6), mode=PRE)
    o.step(20)
    for t in range(1, 21):
        assert o.stats(t)["n_groups"] <= 4 ** (E - 1)


def test_pre_mask_shift_equals_post(oracle_mod):
    """Pre-merging on mask m' = {0} u (m+1) merges exactly the sets that
    post-merging on m merges (both group the step's children on the positions
    of m), so the two produce the same rho(t) and the same groups."""
    K = 6
    eta = structured_eta(K)
    H = W.tls_hamiltonian(0.5, 1.0)
    for m in [(0, 1, 2), (0, 1, 3), (0, 1, 2, 4)]:
        mp = (0,) + tuple(x + 1 for x in m)
        post = oracle.Oracle(H, [1, -1], 0.2, K, eta, W.ground_projector(2), mask=m, mode=POST)
        pre = oracle.Oracle(H, [1, -1], 0.2, K, eta, W.ground_projector(2), mask=mp, mode=PRE)
        post.step(15)
        pre.step(15)
        for t in range(16):
            assert np.abs(post.rho(t) - pre.rho(t)).max() < 1e-14
        hp, wp = post.groups()
        hq, wq = pre.groups()
        ip = np.lexsort(hp.T[::-1])
        iq = np.lexsort(hq.T[::-1])
        assert np.array_equal(hp[ip], hq[iq])
        assert np.abs(wp[ip] - wq[iq]).max() < 1e-15


# ----------------------------------------------------------------- merge rule
def test_merge_rule_worked_example(oracle_mod):
    """Three paths agree on positions {0,1}; the representative is the member of
    largest |w| (Sec. 3.1.2) and the group amplitude is the sum of all three
    (Sec. 2.1).  An exact tie in |w| goes to the history that is smaller read
    from the oldest point."""
    hist = np.array([[1, 2, 3, 0],
                     [1, 2, 0, 3],
                     [1, 2, 2, 2],
                     [0, 0, 0, 0]], dtype=np.uint8)
    w = np.array([0.3 + 0.4j, -0.1 + 0.2j, 0.45 + 0.1j, 0.2])
    rep, sums = oracle.merge_demo(hist, w, [0, 1])
    assert list(rep) == [0, 3]                     # |0.3+0.4i| = 0.5 is the largest of group 0
    assert abs(sums[0] - (0.65 + 0.7j)) < 1e-15
    assert abs(sums[1] - 0.2) < 1e-15
    # exact tie: |0.3+0.4i| = |0.5| = |-0.4-0.3i|; oldest points 0, 3, 1 -> member 0 wins
    w2 = np.array([0.3 + 0.4j, 0.5, -0.4 - 0.3j, 0.2])
    hist2 = hist.copy()
    hist2[1] = [1, 2, 1, 3]
    hist2[2] = [1, 2, 3, 1]
    rep2, _ = oracle.merge_demo(hist2, w2, [0, 1])
    assert rep2[0] == 0
    # quantisation: values closer than the kept mantissa bits are a tie
    w3 = np.array([0.5, 0.5 * (1 + 1e-12), 0.1, 0.2])
    hist3 = np.array([[1, 2, 3, 3], [1, 2, 0, 0], [1, 2, 1, 1], [0, 0, 0, 0]], dtype=np.uint8)
    rep3, _ = oracle.merge_demo(hist3, w3, [0, 1], qbits=32)
    assert rep3[0] == 1                            # tie -> smaller history (oldest point 0)
    rep4, _ = oracle.merge_demo(hist3, w3, [0, 1], qbits=0)
    assert rep4[0] == 1                            # exact compare: member 1 is larger anyway
    w5 = np.array([0.5 * (1 + 1e-12), 0.5, 0.1, 0.2])
    rep5, _ = oracle.merge_demo(hist3, w5, [0, 1], qbits=0)
    assert rep5[0] == 0


# ----------------------------------------------------------------- filter
def test_filter_limits_and_dropped_weight(oracle_mod):
    K = 6
    eta = structured_eta(K)
    H = W.tls_hamiltonian(0.5, 1.0)
    args = (H, [1, -1], 0.2, K, eta, W.ground_projector(2))
    o0 = oracle.Oracle(*args, mask=(0, 1, 2, 3), theta=0.0, mode=PRE)
    otiny = oracle.Oracle(*args, mask=(0, 1, 2, 3), theta=1e-300, mode=PRE)
    o0.step(20)
    otiny.step(20)
    for t in range(21):
        assert np.array_equal(o0.rho(t), otiny.rho(t))
    # first step where theta drops something: the dropped |w| equals the sum over
    # the unfiltered run's children below theta
    theta = 2e-3
    ot = oracle.Oracle(*args, mask=(0, 1, 2, 3), theta=theta, mode=PRE)
    ref = oracle.Oracle(*args, mask=(0, 1, 2, 3), theta=0.0, mode=PRE)
    for t in range(1, 21):
        ot.step(1)
        ref.step(1)
        st = ot.stats(t)
        if st["n_survivors"] < st["n_children"]:
            _, wref = ref.stored()
            small = np.abs(wref) < theta
            assert st["n_children"] - st["n_survivors"] == small.sum()
            assert abs(st["dropped_abs"] - np.abs(wref[small]).sum()) < 1e-15 * len(wref)
            survivors = wref[~small]
            assert st["n_survivors"] == len(survivors)
            break
    else:
        pytest.fail("theta never filtered")


def test_norm_loss_shrinks_with_theta(oracle_mod):
    """Loss of normalisation from filtering decreases as theta decreases (Sec. 4.3)."""
    K = 8
    eta = structured_eta(K)
    H = W.tls_hamiltonian(0.5, 1.0)
    losses = []
    for theta in (1e-3, 1e-4, 1e-5):
        o = oracle.Oracle(H, [1, -1], 0.2, K, eta, W.ground_projector(2), mask=(0, 1, 2, 3, 4),
                          theta=theta, mode=PRE)
        o.step(40)
        losses.append(abs(1.0 - np.trace(o.rho(40)).real))
    assert losses[0] > losses[1] > losses[2]


# ----------------------------------------------------------------- decision log
# The oracle counts representative choices (Sec. 3.1.2) and filter decisions
# (Sec. 2.1) that a relative perturbation of 1e-12 of |w|^2 could flip; every
# parity test requires zero of them.  These worked examples pin that log.  At
# qbits = 32 the compared |w|^2 keeps 20 mantissa bits: in [1, 2) the quanta
# are [1 + k 2^-20, 1 + (k+1) 2^-20).
_Q1 = 1.0 + 2.0 ** -20          # a quantum boundary
_MID = 1.0 + 2.0 ** -21         # the middle of the quantum [1, _Q1)


def _amp(v, split=False):
    """An amplitude with |w|^2 = v (to a few ulp): real, or split evenly over re and im."""
    if split:
        a = math.sqrt(v / 2.0)
        return complex(a, a)
    return complex(math.sqrt(v), 0.0)


@pytest.mark.parametrize("vw,vo,split,qbits,eps,want", [
    (1.5, 1.0, False, 32, 1e-12, False),                         # clear winner
    (_Q1 * (1 + 1e-14), _Q1 * (1 - 1e-14), False, 32, 1e-12, True),   # near tie across a boundary
    (_MID * (1 + 1e-14), _MID * (1 - 1e-14), False, 32, 1e-12, False),  # same quantum, far from its edges
    (_Q1 * (1 - 1e-13), _Q1 * (1 - 2e-13), False, 32, 1e-12, True),   # same quantum, eps reaches the edge
    (_MID, _MID, False, 32, 1e-12, False),                       # exact tie: decided by the history
    (_Q1 * (1 + 5e-11), _Q1 * (1 - 5e-11), False, 32, 1e-12, False),  # adjacent quanta, eps too small to cross
    (1.5, 1.0, True, 32, 1e-12, False),                          # |w|^2 takes both components
    (1.5 * (1 + 1e-14), 1.5, False, 0, 1e-12, True),             # unquantised compare: a near tie
    (1.5 * (1 + 1e-14), 1.5, False, 0, 0.0, False),              # no perturbation: a strict winner
])
def test_could_flip_worked_examples(oracle_mod, vw, vo, split, qbits, eps, want):
    assert oracle.could_flip(_amp(vw, split), _amp(vo), qbits=qbits, eps=eps) is want


def test_flag_ambiguous_worked_example(oracle_mod):
    """Three groups merged on position 0: a near tie across a quantum boundary is
    flagged; an exact tie in the middle of a quantum, decided by the history,
    and a lone member are not."""
    hist = np.array([[0, 1], [0, 2], [0, 3],     # group of point 0 = 0
                     [1, 1], [1, 0],             # point 0 = 1: exact tie
                     [2, 0]], dtype=np.uint8)    # point 0 = 2: alone
    w = np.array([_amp(_Q1 * (1 + 1e-14)), _amp(_Q1 * (1 - 1e-14)), _amp(0.25),
                  _amp(1.25 + 2.0 ** -21), _amp(1.25 + 2.0 ** -21), _amp(0.3)])
    rep, amb = oracle.flag_demo(hist, w, [0])
    assert list(rep) == [0, 4, 5]        # the tie goes to the smaller oldest point (member 4)
    assert list(amb) == [True, False, False]
    # moving both members 1e-9 away from the boundary clears the flag (with the
    # winner still within 1e-12 of it, a perturbation could make the two tie)
    w2 = w.copy()
    w2[0] = _amp(_Q1 * (1 + 1e-9))
    w2[1] = _amp(_Q1 * (1 - 1e-9))
    _, amb2 = oracle.flag_demo(hist, w2, [0])
    assert list(amb2) == [False, False, False]


def test_theta_margin_is_counted(oracle_mod):
    """With no coupling the step-1 children are rho0 times K4 = U (x) conj(U)
    (eq. SysP).  A threshold equal to |U00 U10| -- the modulus of the children
    of pairs (0,1) and (1,0) -- puts both within the ambiguity margin; one
    1e-6 above it drops both with no ambiguity (Sec. 2.1, path filtering).
    Here |U00| > |U10|."""
    K, dt = 3, 0.2
    H = W.tls_hamiltonian(0.5, 1.0)
    U = expm(-1j * H * dt)
    th = abs(U[0, 0]) * abs(U[1, 0])
    eta = np.zeros((3, K + 1), dtype=complex)
    o = oracle.Oracle(H, [1, -1], dt, K, eta, W.ground_projector(2), theta=th, mode=PRE)
    o.step(1)
    s = o.stats(1)
    assert s["n_amb_theta"] == 2 and s["theta_margin"] < 1e-12
    o2 = oracle.Oracle(H, [1, -1], dt, K, eta, W.ground_projector(2), theta=th * (1 + 1e-6), mode=PRE)
    o2.step(1)
    s2 = o2.stats(1)
    # only (0,0) survives: |U10|^2 < |U00 U10| drops (1,1) too
    assert s2["n_amb_theta"] == 0 and s2["n_survivors"] == 1 and 1e-7 < s2["theta_margin"] < 1e-5
