"""Pins for the oracle's adjoint gradient (CPU).

* central finite differences of the oracle objective (h = 1e-5) on problems with
  small cost values, where the O(h^2 c^3) truncation error is below 1e-8;
* the per-gate parameter-shift rule for beta, exact because every mixer gate is
  exp(-i b X) with X^2 = I:  dE/dbeta_l = sum_i [E(beta_{l,i} + pi/4) - E(beta_{l,i} - pi/4)],
  with only gate i of layer l shifted (built from the oracle's per-gate primitives);
* the complex-step derivative of the p = 1 MaxCut closed form (Wang et al. 2018).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from dense_ref import maxcut_p1_closed_form


def _small_problem(n, seed):
    terms = W.random_terms(n, 12, seed=seed, max_order=3, integer=False, wmax=0.5)
    return oracle.diag_terms(n, terms)


@pytest.mark.parametrize("n,p,seed", [(3, 1, 0), (5, 3, 1), (7, 4, 2)])
def test_grad_matches_central_differences(n, p, seed):
    c = _small_problem(n, seed)
    rng = np.random.default_rng(seed)
    g, b = rng.uniform(-1, 1, size=p), rng.uniform(-1, 1, size=p)
    E, dg, db = oracle.grad(n, c, g, b)
    assert abs(E - oracle.qaoa_expectation(n, c, g, b)) < 1e-13
    h = 1e-5
    scale = max(1.0, np.max(np.abs(np.concatenate([dg, db]))))
    for k in range(p):
        for vec, d in ((g, dg), (b, db)):
            vp, vm = vec.copy(), vec.copy()
            vp[k] += h
            vm[k] -= h
            if vec is g:
                fd = (oracle.qaoa_expectation(n, c, vp, b) - oracle.qaoa_expectation(n, c, vm, b)) / (2 * h)
            else:
                fd = (oracle.qaoa_expectation(n, c, g, vp) - oracle.qaoa_expectation(n, c, g, vm)) / (2 * h)
            assert abs(fd - d[k]) <= 1e-7 * scale, (k, fd, d[k])


def _energy_pergate(n, c, gamma, beta_gates):
    """E for a circuit whose mixer gate i of layer l has its own angle."""
    psi = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
    for l, gl in enumerate(gamma):
        psi = oracle.apply_phase(n, c, gl, psi)
        for q in range(n):
            psi = oracle.apply_rx(n, q, beta_gates[l][q], psi)
    return oracle.expectation(n, psi, c)[0]


@pytest.mark.parametrize("n,p", [(4, 2), (7, 3)])
def test_beta_gradient_equals_parameter_shift(n, p):
    c = oracle.diag_labs(n).astype(np.float64)
    g, b = W.linear_ramp(p, seed=n)
    _, _, db = oracle.grad(n, c, g, b)
    for l in range(p):
        tot = 0.0
        for i in range(n):
            bp = [[b[m]] * n for m in range(p)]
            bm = [[b[m]] * n for m in range(p)]
            bp[l][i] += np.pi / 4
            bm[l][i] -= np.pi / 4
            tot += _energy_pergate(n, c, g, bp) - _energy_pergate(n, c, g, bm)
        assert abs(tot - db[l]) <= 1e-10 * max(1.0, abs(db[l])), (l, tot, db[l])


def test_p1_maxcut_gradient_closed_form():
    cfg = W.C1()
    n, edges = cfg["n"], cfg["edges"]
    c = oracle.diag_maxcut(n, edges)
    rng = np.random.default_rng(3)
    h = 1e-20
    for _ in range(4):
        g, b = rng.uniform(0, np.pi, size=2)
        _, dg, db = oracle.grad(n, c, [g], [b])
        # E(g, b) = -F(-g, b); complex-step derivatives of the closed form
        dg_ref = (-maxcut_p1_closed_form(n, edges, -(g + 1j * h), b)).imag / h
        db_ref = (-maxcut_p1_closed_form(n, edges, -g, b + 1j * h)).imag / h
        assert abs(dg[0] - dg_ref) <= 1e-10 * max(1.0, abs(dg_ref))
        assert abs(db[0] - db_ref) <= 1e-10 * max(1.0, abs(db_ref))


def test_grad_zero_at_trivial_points():
    # gamma = 0 everywhere: |+> is stationary, E = mean(c) for all beta, so dE/dbeta = 0
    n, p = 6, 3
    c = oracle.diag_labs(n).astype(np.float64)
    _, _, db = oracle.grad(n, c, np.zeros(p), np.array([0.3, -0.7, 1.1]))
    assert np.max(np.abs(db)) < 1e-12


def test_grad_does_not_depend_on_thread_count():
    # the inner products are summed over fixed index ranges in a fixed order
    n, p = 11, 3
    c = oracle.diag_terms(n, W.random_terms(n, 20, seed=5, max_order=4, integer=False, wmax=2.0))
    rng = np.random.default_rng(5)
    g, b = rng.uniform(-1, 1, size=p), rng.uniform(-1, 1, size=p)
    saved = oracle.num_threads()
    try:
        results = []
        for t in (1, 3, 8):
            oracle.set_num_threads(t)
            E, dg, db = oracle.grad(n, c, g, b)
            results.append(np.concatenate([[E], dg, db]))
    finally:
        oracle.set_num_threads(saved)
    assert all(np.array_equal(results[0], r) for r in results[1:])
