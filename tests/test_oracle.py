"""Pins for the CPU oracle, against facts that do not come from the oracle itself:
known permanents, brute force over permutations, closed forms of the beam
splitter (single photon, Hong-Ou-Mandel, theta = 0 and pi/2), group structure
(sector unitarity and the homomorphism (AB)_P = A_P B_P), the unique path of
depth <= 2 circuits (Eq. (10)), and the paper's own correctness protocol
(Sec. III.A: probabilities of all outputs sum to 1; path sum and Ryser agree)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2510_26408_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2.0 ** -53


def rand_unitary(n, rng):
    z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def brick(m, D, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return workloads.random_brickwork(m, D, rng)


def flat(layers):
    return [bs for l in layers for bs in l]


# ---------------------------------------------------------------- permanents
@pytest.mark.parametrize("n", range(0, 7))
def test_permanent_all_ones_is_factorial(n):
    assert oracle.permanent(np.ones((n, n))) == pytest.approx(math.factorial(n), rel=1e-15)


def test_permanent_diagonal_and_permutation():
    rng = np.random.default_rng(1)
    d = rng.normal(size=5) + 1j * rng.normal(size=5)
    assert abs(oracle.permanent(np.diag(d)) - np.prod(d)) < 1e-14
    P = np.eye(6)[[3, 0, 5, 1, 2, 4]]
    assert abs(oracle.permanent(P) - 1) < 1e-15


@pytest.mark.parametrize("n", range(1, 8))
def test_ryser_matches_bruteforce(n):
    rng = np.random.default_rng(100 + n)
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    r, eb = oracle.permanent(a, with_bound=True)
    b = oracle.permanent_bruteforce(a)
    assert abs(r - b) <= 1e-12 * max(1.0, abs(b))
    assert eb < 1e-12


# ------------------------------------------------------------ single BS (App.)
@pytest.mark.parametrize("theta,phi", [(0.3, 0.7), (1.2, 5.9), (0.05, 3.1)])
def test_single_photon_is_matrix_element(theta, phi):
    # rows = outputs, columns = inputs: <y|BS|x> for one photon is BS[y, x]
    c, s = math.cos(theta), math.sin(theta)
    assert abs(oracle.bs_amplitude(theta, phi, 1, 0, 1, 0) - c) < 1e-15
    assert abs(oracle.bs_amplitude(theta, phi, 1, 0, 0, 1) - np.exp(1j * phi) * s) < 1e-15
    assert abs(oracle.bs_amplitude(theta, phi, 0, 1, 1, 0) + np.exp(-1j * phi) * s) < 1e-15
    assert abs(oracle.bs_amplitude(theta, phi, 0, 1, 0, 1) - c) < 1e-15


@pytest.mark.parametrize("phi", [0.0, 1.0, 2.5, 6.0])
def test_hong_ou_mandel(phi):
    t = math.pi / 4
    assert abs(oracle.bs_amplitude(t, phi, 1, 1, 1, 1)) <= 4 * U64
    assert abs(oracle.bs_amplitude(t, phi, 1, 1, 2, 0)) ** 2 == pytest.approx(0.5, abs=1e-15)
    assert abs(oracle.bs_amplitude(t, phi, 1, 1, 0, 2)) ** 2 == pytest.approx(0.5, abs=1e-15)


@pytest.mark.parametrize("x1,x2", [(0, 0), (1, 0), (2, 3), (4, 1), (3, 3)])
def test_theta_zero_and_half_pi(x1, x2):
    phi = 0.83
    N = x1 + x2
    for y1 in range(N + 1):
        a0 = oracle.bs_amplitude(0.0, phi, x1, x2, y1, N - y1)
        assert a0 == (1.0 if y1 == x1 else 0.0)
        a1 = oracle.bs_amplitude(math.pi / 2, phi, x1, x2, y1, N - y1)
        if y1 == x2:
            want = np.exp(1j * phi) ** x1 * (-np.exp(-1j * phi)) ** x2
            assert abs(a1 - want) < 1e-13
        else:
            assert abs(a1) < 1e-13


@pytest.mark.parametrize("N", range(0, 9))
def test_sector_unitary(N):
    rng = np.random.default_rng(N)
    for _ in range(3):
        th, ph = rng.uniform(0, math.pi / 2), rng.uniform(0, 2 * math.pi)
        W = oracle.bs_sector(th, ph, N)
        assert np.max(np.abs(W.conj().T @ W - np.eye(N + 1))) < 2e-15 * (N + 1)


def test_fock_lift_is_homomorphism_two_modes():
    rng = np.random.default_rng(7)
    for N in range(1, 7):
        A, B = rand_unitary(2, rng), rand_unitary(2, rng)

        def sector(U):
            return np.array([[oracle.fock_amplitude(U, [x1, N - x1], [y1, N - y1])
                              for x1 in range(N + 1)] for y1 in range(N + 1)])

        assert np.max(np.abs(sector(A @ B) - sector(A) @ sector(B))) < 1e-13


def test_fock_lift_is_homomorphism_three_modes():
    rng = np.random.default_rng(8)
    A, B = rand_unitary(3, rng), rand_unitary(3, rng)
    n = 3
    confs = oracle.all_patterns(3, n)
    S = (2, 0, 1)
    for T in confs:
        direct = oracle.fock_amplitude(A @ B, S, T)
        via = sum(oracle.fock_amplitude(A, c, T) * oracle.fock_amplitude(B, S, c) for c in confs)
        assert abs(direct - via) < 1e-13


# --------------------------------------------------------------- full circuit
def test_compose_is_unitary_and_single_photon_entries():
    m, D = 7, 5
    layers = brick(m, D, 3)
    U = oracle.compose(m, flat(layers))
    assert np.max(np.abs(U @ U.conj().T - np.eye(m))) < 1e-14
    for s in range(m):
        for t in range(m):
            S = np.eye(m, dtype=np.int32)[s]
            T = np.eye(m, dtype=np.int32)[t]
            assert abs(oracle.amplitude(m, S, T, flat(layers)) - U[t, s]) < 1e-15


def test_conservation_and_light_cone_give_exact_zero():
    m = 8
    layers = brick(m, 1, 4)
    S = [1, 0, 0, 0, 0, 0, 0, 0]
    assert oracle.amplitude(m, S, [0, 0, 0, 1, 0, 0, 0, 0], flat(layers)) == 0
    assert oracle.amplitude(m, S, [1, 1, 0, 0, 0, 0, 0, 0], flat(layers)) == 0


@pytest.mark.parametrize("m,D,S", [(4, 3, (1, 1, 0, 0)), (4, 4, (2, 0, 1, 0)), (5, 4, (1, 0, 1, 0, 1)),
                                   (5, 5, (0, 2, 0, 1, 0)), (6, 3, (1, 1, 1, 0, 0, 0))])
def test_pathsum_matches_ryser_and_counts(m, D, S):
    layers = brick(m, D, 10 + m + D)
    circ = flat(layers)
    n = sum(S)
    for T in oracle.all_patterns(m, n):
        r = oracle.amplitude(m, S, T, circ)
        p, cnt = oracle.pathsum(m, S, T, circ)
        assert abs(r - p) < 1e-14
        assert cnt == oracle.path_count_bruteforce(m, S, T, circ)


@pytest.mark.parametrize("D", [1, 2])
def test_depth_le_two_has_at_most_one_path(D):
    m = 6
    layers = brick(m, D, 20 + D)
    circ = flat(layers)
    S = (1, 0, 2, 1, 0, 1)
    for T in oracle.all_patterns(m, sum(S)):
        p, cnt = oracle.pathsum(m, S, T, circ)
        assert cnt in (0.0, 1.0)
        assert abs(p - oracle.amplitude(m, S, T, circ)) < 1e-14
        if cnt == 0:
            assert p == 0


def test_paper_correctness_protocol():
    g = json.load(open(os.path.join(GOLDEN, "paper_correctness_inputs.json")))
    m = g["m"]
    for k, case in enumerate(g["cases"]):
        S = np.array(case["S"], dtype=np.int32)
        layers = brick(m, case["depth"], 30 + k)
        circ = flat(layers)
        pats = oracle.all_patterns(m, int(S.sum()))
        amps, eb, _ = oracle.amplitudes(m, S, np.array(pats), circ, with_bound=True)
        p_ryser = np.abs(amps) ** 2
        assert abs(p_ryser.sum() - 1) < 1e-12
        assert eb.max() < 1e-15
        state = oracle.evolve(m, S, circ)
        p_evolve = np.array([abs(state.get(tuple(T), 0)) ** 2 for T in pats])
        assert abs(p_evolve.sum() - 1) < 1e-12
        tvd = 0.5 * np.abs(p_ryser - p_evolve).sum()
        assert tvd <= g["tvd_vs_ryser_max"]


def test_batch_matches_single_and_threads():
    wl = workloads.make("c2", seed=0, batch=16)
    circ = wl.flat_circuit()
    amps, used = oracle.amplitudes(wl.m, wl.S, wl.Ts, circ, nthreads=4)
    for p in range(4):
        assert amps[p] == oracle.amplitude(wl.m, wl.S, wl.Ts[p], circ)
    assert used >= 1


def test_ryser_bound_small_on_workloads():
    for name in ("c2", "c3", "c5"):
        wl = workloads.make(name, seed=0, batch=4)
        _, eb, _ = oracle.amplitudes(wl.m, wl.S, wl.Ts, wl.flat_circuit(), nthreads=4, with_bound=True)
        assert eb.max() < 1e-15


# ------------------------------------------------------------ absolute form
@pytest.mark.parametrize("m,D", [(4, 3), (6, 5), (7, 4)])
def test_absolute_form_single_photon_is_matrix_product(m, D):
    """With one photon every path is a walk of the photon through the modes,
    so the absolute form is an entry of the product of the splitters' mode
    matrices with each entry replaced by |Re| + |Im|."""
    circ = flat(brick(m, D, 40 + m + D))
    P = np.eye(m)
    for (a, b, th, ph) in circ:
        M = np.eye(m)
        for xa in range(2):
            for ya in range(2):
                t = oracle.bs_amplitude(th, ph, xa, 1 - xa, ya, 1 - ya)
                M[(a, b)[1 - ya], (a, b)[1 - xa]] = abs(t.real) + abs(t.imag)
        P = M @ P
    for i in range(m):
        S = [0] * m
        S[i] = 1
        for j in range(m):
            T = [0] * m
            T[j] = 1
            got = oracle.absolute_form(m, S, T, circ)
            assert abs(got - P[j, i]) <= 1e-14 * max(1.0, P[j, i])


def test_absolute_form_bounds_amplitude_and_vanishes_with_paths():
    m, D = 5, 4
    circ = flat(brick(m, D, 50))
    S = (1, 0, 2, 0, 1)
    for T in oracle.all_patterns(m, sum(S)):
        a = oracle.absolute_form(m, S, T, circ)
        amp = oracle.amplitude(m, S, T, circ)
        assert a >= abs(amp) - 1e-14
        assert (a > 0) == (oracle.path_count_bruteforce(m, S, T, circ) > 0)


# ------------------------------------------------ high-precision sectors
def test_high_precision_sector_matches_permanent_form():
    """The closed-form sum in 40 digits equals the permanent-based sector (a
    different formula) for small N."""
    pytest.importorskip("mpmath")
    for (th, ph) in ((0.3, 1.1), (1.2, -0.4), (math.pi / 4, 2.5)):
        for N in range(0, 7):
            a = oracle.bs_sector_hp(th, ph, N)
            b = oracle.bs_sector(th, ph, N)
            assert np.abs(a - b).max() < 1e-15


def test_high_precision_sector_unitary_at_large_n():
    pytest.importorskip("mpmath")
    W = oracle.bs_sector_hp(0.83, 0.6, 30)
    assert np.abs(W @ W.conj().T - np.eye(31)).max() < 1e-14


def test_high_precision_evolution_matches_ryser():
    """The evolution with 40-digit sectors equals Ryser's amplitudes on a
    small circuit (a third route to the same numbers) and conserves norm."""
    pytest.importorskip("mpmath")
    m, D = 4, 3
    circ = flat(brick(m, D, 60))
    S = (2, 0, 1, 1)
    st = oracle.evolve_hp(m, S, circ)
    assert abs(sum(abs(v) ** 2 for v in st.values()) - 1.0) < 1e-13
    for T in oracle.all_patterns(m, sum(S)):
        assert abs(st.get(tuple(T), 0) - oracle.amplitude(m, S, T, circ)) < 1e-14
