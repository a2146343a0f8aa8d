"""Pins for the oracle's state evolution and objective (CPU).

The oracle follows Algorithm 3 (phase then mixer, per-qubit gates).  It is
checked against:
  * scipy.linalg.expm of the dense 2^n x 2^n mixer Hamiltonian (library routine);
  * the p=1 MaxCut closed form of Wang et al. (PRA 97, 022304, 2018);
  * exact special cases and invariants of the QAOA state and objective;
  * math.fsum for the compensated objective sum.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from dense_ref import dense_state, maxcut_p1_closed_form

RNG = np.random.default_rng(1234)


def _rand_state(n, seed):
    r = np.random.default_rng(seed)
    v = r.normal(size=1 << n) + 1j * r.normal(size=1 << n)
    return v / np.linalg.norm(v)


CASES = []
for n in (1, 2, 3, 5, 7):
    for p in (0, 1, 3):
        CASES.append(("random", n, p))
CASES += [("labs", 6, 2), ("labs", 8, 4), ("maxcut", 8, 3)]


@pytest.mark.parametrize("kind,n,p", CASES)
def test_evolve_matches_dense_expm(kind, n, p):
    seed = 100 * n + p
    if kind == "random":
        c = oracle.diag_terms(n, W.random_terms(n, 10, seed=seed, integer=False))
    elif kind == "labs":
        c = oracle.diag_labs(n).astype(np.float64)
    else:
        edges, weights = W.erdos_renyi_graph(n, 0.5, seed=seed)
        c = oracle.diag_maxcut(n, edges, weights)
    r = np.random.default_rng(seed)
    gamma = r.uniform(-np.pi, np.pi, size=p)
    beta = r.uniform(-np.pi, np.pi, size=p)
    ref = dense_state(n, c, gamma, beta)
    got = oracle.evolve(n, c, gamma, beta)
    assert np.max(np.abs(got - ref)) < 1e-11
    # from an arbitrary input state too
    psi0 = _rand_state(n, seed + 1)
    ref = dense_state(n, c, gamma, beta, psi0=psi0)
    got = oracle.evolve(n, c, gamma, beta, psi0=psi0)
    assert np.max(np.abs(got - ref)) < 1e-11


@pytest.mark.parametrize("n", [1, 4, 7])
def test_beta_half_pi_is_global_bit_flip(n):
    # exp(-i pi/2 X) = -i X on every qubit: psi'[x] = (-i)^n psi[x xor (2^n - 1)]
    psi = _rand_state(n, 7 + n)
    out = oracle.apply_mixer(n, np.pi / 2, psi)
    N = 1 << n
    expect = ((-1j) ** n) * psi[np.arange(N) ^ (N - 1)]
    assert np.max(np.abs(out - expect)) < 1e-14


@pytest.mark.parametrize("n,p", [(3, 2), (8, 5)])
def test_gamma_zero_plus_state_eigenvector(n, p):
    # |+> is the +1 eigenvector of every X_i: exp(-i b M)|+> = exp(-i n b)|+>
    c = oracle.diag_labs(n).astype(np.float64)
    beta = RNG.uniform(-2, 2, size=p)
    got = oracle.evolve(n, c, np.zeros(p), beta)
    expect = np.exp(-1j * n * beta.sum()) * np.full(1 << n, 2.0 ** (-n / 2))
    assert np.max(np.abs(got - expect)) < 1e-13


@pytest.mark.parametrize("n", [4, 10])
def test_norm_preserved_and_beta_zero_mean(n):
    c = oracle.diag_labs(n).astype(np.float64)
    p = 4
    g = RNG.uniform(0, 1, size=p)
    psi = oracle.evolve(n, c, g, RNG.uniform(0, 1, size=p))
    E, nrm = oracle.expectation(n, psi, c)
    assert abs(nrm - 1.0) < 1e-13
    # beta = 0: only phases act on |+>, so E = mean(c) = n(n-1)/2 for LABS
    psi0 = oracle.evolve(n, c, g, np.zeros(p))
    E0, _ = oracle.expectation(n, psi0, c)
    assert abs(E0 - n * (n - 1) / 2) < 1e-12 * n * n


def test_zero_weight_problem_gives_zero():
    n = 6
    c = oracle.diag_terms(n, [(0.0, (0, 1)), (0.0, (2, 3, 4))])
    psi = oracle.evolve(n, c, [0.4, 1.3], [0.2, 0.9])
    assert oracle.expectation(n, psi, c)[0] == 0.0


def _k4():
    return 4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def _prism():
    return 6, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 3), (0, 3), (1, 4), (2, 5)]


def _c1():
    cfg = W.C1()
    return cfg["n"], cfg["edges"]


@pytest.mark.parametrize("graph", [_k4, _prism, _c1])
def test_p1_maxcut_closed_form(graph):
    n, edges = graph()
    c = oracle.diag_maxcut(n, edges)
    r = np.random.default_rng(len(edges))
    for _ in range(5):
        g, b = r.uniform(0, np.pi, size=2)
        E = oracle.qaoa_expectation(n, c, [g], [b])
        # our phase exp(-i g c) with c = -cut is the paper-of-Wang phase at -g
        ref = -maxcut_p1_closed_form(n, edges, -g, b)
        assert abs(E - ref) < 1e-12


def test_c1_workload_closed_form():
    cfg = W.C1()
    n, edges = cfg["n"], cfg["edges"]
    c = oracle.diag_maxcut(n, edges)
    E = oracle.qaoa_expectation(n, c, cfg["gamma"], cfg["beta"])
    ref = -maxcut_p1_closed_form(n, edges, -cfg["gamma"][0], cfg["beta"][0])
    assert abs(E - ref) < 1e-12


def test_time_reversal_symmetry():
    # real c: conj(psi(gamma, beta)) = psi(-gamma, -beta) up to the X-basis symmetry,
    # so E(-gamma, -beta) = E(gamma, beta)
    n, p = 7, 3
    c = oracle.diag_terms(n, W.random_terms(n, 12, seed=5))
    g, b = RNG.uniform(-2, 2, size=p), RNG.uniform(-2, 2, size=p)
    assert abs(oracle.qaoa_expectation(n, c, g, b) - oracle.qaoa_expectation(n, c, -g, -b)) < 1e-12


def test_labs_gamma_pi_shift_and_even_order_beta_shift():
    n, p = 7, 3
    c = oracle.diag_labs(n).astype(np.float64)
    g, b = RNG.uniform(0, 1, size=p), RNG.uniform(0, 1, size=p)
    E = oracle.qaoa_expectation(n, c, g, b)
    for l in range(p):
        g2 = g.copy(); g2[l] += np.pi
        assert abs(oracle.qaoa_expectation(n, c, g2, b) - E) < 1e-10
        b2 = b.copy(); b2[l] += np.pi / 2
        assert abs(oracle.qaoa_expectation(n, c, g, b2) - E) < 1e-10


def test_expectation_compensated_against_fsum():
    n = 14
    c = oracle.diag_labs(n).astype(np.float64)
    psi = _rand_state(n, 99)
    E, nrm = oracle.expectation(n, psi, c)
    pr = psi.real * psi.real + psi.imag * psi.imag
    ex = math.fsum((pr * c).tolist())
    assert abs(E - ex) <= 2 * np.spacing(ex)
    assert abs(nrm - math.fsum(pr.tolist())) <= 2 * np.spacing(1.0)
