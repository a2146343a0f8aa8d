"""Adjoint gradient on the GPU (qaoa_grad) against the FP64 oracle's adjoint,
central finite differences, and through torch.autograd.

Tolerances: complex128 |d grad| <= 1e-9 * max(1, ||grad||_inf); complex64
<= 1e-5 * max(1, ||grad||_inf); finite differences (h = 1e-5, truncation
O(h^2 c^3)) <= 1e-5 * max(1, ||grad||_inf).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TD = {"complex64": torch.complex64, "complex128": torch.complex128}


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_04841_amd as q
    return q


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _gpu_grad(q, n, terms, ddt, dtype, g, b):
    diag, off = q.qaoa_precompute_diag(n, terms, ddt, device="cuda")
    psi = torch.empty(1 << n, dtype=TD[dtype], device="cuda")
    adj = torch.empty_like(psi)
    out = q.qaoa_grad(n, g, b, diag, psi, adj, diag_offset=off).cpu().numpy()
    p = len(g)
    return out[0], out[1:1 + p], out[1 + p:], diag, off


CASES = [(3, 2, "complex128", "i32"), (8, 3, "complex128", "u16"), (12, 4, "complex128", "i32"),
         (13, 2, "complex128", "i32"), (16, 3, "complex128", "u16"), (17, 2, "complex128", "f64"),
         (9, 3, "complex64", "i32"), (14, 3, "complex64", "u16"), (18, 2, "complex64", "i32")]


@pytest.mark.parametrize("n,p,dtype,ddt", CASES)
def test_grad_matches_oracle(q, n, p, dtype, ddt):
    _say(f"grad n={n} p={p} {dtype} {ddt}")
    if ddt == "f64":
        terms = [(0.37 * w, e) for w, e in W.labs_terms(n)]
    else:
        terms = W.random_terms(n, 3 * n, seed=n, max_order=4, integer=True, wmax=4)
    rng = np.random.default_rng(100 + n)
    g, b = rng.uniform(-0.5, 0.5, size=p), rng.uniform(-np.pi, np.pi, size=p)
    E, dg, db, _, _ = _gpu_grad(q, n, terms, ddt, dtype, g, b)
    c = oracle.diag_terms(n, terms)
    Er, dgr, dbr = oracle.grad(n, c, g, b)
    scale = max(1.0, np.max(np.abs(np.concatenate([dgr, dbr]))))
    tol = 1e-9 if dtype == "complex128" else 1e-5
    assert abs(E - Er) <= tol * max(1.0, abs(Er))
    assert np.max(np.abs(dg - dgr)) <= tol * scale, (dg, dgr)
    assert np.max(np.abs(db - dbr)) <= tol * scale, (db, dbr)


@pytest.mark.parametrize("n,dtype", [(9, "complex128"), (15, "complex128"), (16, "complex64")])
def test_grad_int32_beyond_two_level_table(q, n, dtype):
    # cost values mostly outside [-2^15, 2^15): the reverse sweeps undo the phase
    # with the two-pass byte tables
    p = 2
    terms = W.random_terms(n, 4 * n, seed=60 + n, max_order=3, integer=True, wmax=9000)
    c = oracle.diag_terms(n, terms)
    assert np.abs(c).max() >= 32768
    rng = np.random.default_rng(300 + n)
    g, b = rng.uniform(-0.02, 0.02, size=p), rng.uniform(-np.pi, np.pi, size=p)
    _say(f"grad int32 wide range n={n} {dtype}")
    E, dg, db, _, _ = _gpu_grad(q, n, terms, "i32", dtype, g, b)
    Er, dgr, dbr = oracle.grad(n, c, g, b)
    scale = max(1.0, np.max(np.abs(np.concatenate([dgr, dbr]))))
    tol = 1e-9 if dtype == "complex128" else 1e-5
    assert abs(E - Er) <= tol * max(1.0, abs(Er))
    assert np.max(np.abs(dg - dgr)) <= tol * scale, (dg, dgr)
    assert np.max(np.abs(db - dbr)) <= tol * scale, (db, dbr)


def test_grad_energy_equals_evolve_and_is_deterministic(q):
    n, p = 15, 3
    terms = W.labs_terms(n)
    g, b = W.linear_ramp(p, seed=1)
    E1, dg1, db1, diag, off = _gpu_grad(q, n, terms, "i32", "complex128", g, b)
    E2, dg2, db2, _, _ = _gpu_grad(q, n, terms, "i32", "complex128", g, b)
    assert E1 == E2 and np.array_equal(dg1, dg2) and np.array_equal(db1, db2)
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    q.qaoa_evolve(n, g, b, diag, psi, diag_offset=off, out=out)
    assert out[0].item() == E1


def test_c4_workload_against_finite_differences(q):
    """LABS n=24, p=20, complex128: adjoint vs central differences of the GPU
    objective (h = 1e-5) on sampled parameters, and the p=20 gradient's
    gamma/beta time-reversal symmetry."""
    cfg = W.C4()
    n, p = cfg["n"], cfg["p"]
    g, b = cfg["gamma"], cfg["beta"]
    _say("C4 gradient")
    E, dg, db, diag, off = _gpu_grad(q, n, cfg["terms"], "i32", "complex128", g, b)
    scale = max(1.0, np.max(np.abs(np.concatenate([dg, db]))))
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")

    def energy(gg, bb):
        q.qaoa_evolve(n, gg, bb, diag, psi, diag_offset=off, out=out)
        return out[0].item()

    assert energy(g, b) == E
    h = 1e-5
    for k in (0, 7, 19):
        gp, gm = g.copy(), g.copy()
        gp[k] += h
        gm[k] -= h
        assert abs((energy(gp, b) - energy(gm, b)) / (2 * h) - dg[k]) <= 1e-5 * scale, k
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        assert abs((energy(g, bp) - energy(g, bm)) / (2 * h) - db[k]) <= 1e-5 * scale, k
    # E(-gamma, -beta) = E(gamma, beta), so the gradient flips sign
    E2, dg2, db2, _, _ = _gpu_grad(q, n, cfg["terms"], "i32", "complex128", -g, -b)
    assert abs(E2 - E) <= 1e-10 * abs(E)
    assert np.max(np.abs(dg2 + dg)) <= 1e-9 * scale and np.max(np.abs(db2 + db)) <= 1e-9 * scale
    del psi
    torch.cuda.empty_cache()


def test_autograd_function(q):
    n, p = 12, 3
    sim = q.Simulator(n, terms=W.labs_terms(n), dtype="complex128")
    g0, b0 = W.linear_ramp(p, seed=9)
    gamma = torch.tensor(g0, dtype=torch.float64, requires_grad=True)
    beta = torch.tensor(b0, dtype=torch.float64, requires_grad=True)
    E = q.qaoa_objective(gamma, beta, sim)
    (3.0 * E).backward()
    c = oracle.diag_labs(n).astype(np.float64)
    Er, dgr, dbr = oracle.grad(n, c, g0, b0)
    assert abs(E.item() - Er) <= 1e-10 * abs(Er)
    assert np.max(np.abs(gamma.grad.numpy() - 3.0 * dgr)) <= 1e-8 * max(1.0, np.max(np.abs(dgr)))
    assert np.max(np.abs(beta.grad.numpy() - 3.0 * dbr)) <= 1e-8 * max(1.0, np.max(np.abs(dbr)))
    # a few small optimiser steps lower E monotonically.  The LABS landscape
    # oscillates in gamma at a frequency of the order of the cost values (|dE/dgamma|
    # ~ 200 here), so the step must stay far below 1e-2 rad: lr = 1e-6 moves gamma
    # by ~1e-3 over five steps.
    opt = torch.optim.SGD([gamma, beta], lr=1e-6)
    energies = []
    for _ in range(5):
        opt.zero_grad()
        e = q.qaoa_objective(gamma, beta, sim)
        energies.append(e.item())
        e.backward()
        opt.step()
    energies.append(q.qaoa_objective(gamma.detach(), beta.detach(), sim).item())
    assert all(b < a for a, b in zip(energies, energies[1:])), energies
