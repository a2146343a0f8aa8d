"""Seeded random configurations against the FP64 oracle: state sizes across the
single-tile, narrow, wide and complex64 plans, random spin polynomials of order
up to 4 (integer and real weights, all three cost storages), random angles of
either sign, p up to 6, from |+>^n or a given state; and adjoint gradients.
Tolerances as in the other parity tests (complex128 1e-10 on the state and E,
1e-9 relative on gradients; complex64 1e-5)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TD = {"complex64": torch.complex64, "complex128": torch.complex128}


def _cases(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(3, 21))
        p = int(rng.integers(1, 7))
        dtype = "complex128" if rng.random() < 0.6 else "complex64"
        ddt = ("i32", "u16", "f64")[int(rng.integers(0, 3))]
        out.append((i, n, p, dtype, ddt, bool(rng.random() < 0.3)))
    return out


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_04841_amd as q
    return q


def _terms(n, ddt, seed):
    # integer weights for the integer storages (bit-exact), real ones for float64
    return W.random_terms(n, 2 * n + 3, seed, max_order=4, integer=ddt != "f64", wmax=5)


@pytest.mark.parametrize("i,n,p,dtype,ddt,given", _cases(24, 2026))
def test_random_evolve(q, i, n, p, dtype, ddt, given):
    print(f"random evolve #{i} n={n} p={p} {dtype} {ddt} given={given}", file=sys.stderr, flush=True)
    rng = np.random.default_rng(1000 + i)
    terms = _terms(n, ddt, seed=2000 + i)
    gamma, beta = rng.uniform(-1.5, 1.5, size=p), rng.uniform(-np.pi, np.pi, size=p)
    psi0 = None
    if given:
        psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        psi0 /= np.linalg.norm(psi0)
        if dtype == "complex64":
            psi0 = psi0.astype(np.complex64).astype(np.complex128)
    diag, off = q.qaoa_precompute_diag(n, terms, ddt, device="cuda")
    psi = torch.empty(1 << n, dtype=TD[dtype], device="cuda")
    if given:
        psi.copy_(torch.from_numpy(psi0).to(TD[dtype]))
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    q.qaoa_evolve(n, gamma, beta, diag, psi, init=not given, diag_offset=off, out=out)
    torch.cuda.synchronize()
    c = oracle.diag_terms(n, terms)
    got_c = diag.cpu().numpy().astype(np.float64) + off
    assert np.array_equal(got_c, c) if ddt != "f64" else np.max(np.abs(got_c - c)) <= 1e-12 * sum(abs(w) for w, _ in terms)
    ref = oracle.evolve(n, c, gamma, beta, psi0=psi0)
    E, nrm = oracle.expectation(n, ref, c)
    tol = 1e-10 if dtype == "complex128" else 1e-5
    got = psi.cpu().numpy().astype(np.complex128)
    eo = out.cpu().numpy()
    assert np.linalg.norm(got - ref) <= tol
    assert abs(eo[0] - E) <= tol * max(1.0, abs(E))
    assert abs(eo[1] - nrm) <= tol


@pytest.mark.parametrize("i,n,p,dtype,ddt,given", _cases(10, 2027))
def test_random_gradient(q, i, n, p, dtype, ddt, given):
    # the gradient entry point always starts from |+>^n: `given` is not used here
    print(f"random gradient #{i} n={n} p={p} {dtype} {ddt}", file=sys.stderr, flush=True)
    rng = np.random.default_rng(3000 + i)
    terms = _terms(n, ddt, seed=4000 + i)
    gamma, beta = rng.uniform(-0.5, 0.5, size=p), rng.uniform(-np.pi, np.pi, size=p)
    diag, off = q.qaoa_precompute_diag(n, terms, ddt, device="cuda")
    psi = torch.empty(1 << n, dtype=TD[dtype], device="cuda")
    adj = torch.empty_like(psi)
    out = q.qaoa_grad(n, gamma, beta, diag, psi, adj, diag_offset=off).cpu().numpy()
    c = oracle.diag_terms(n, terms)
    Er, dgr, dbr = oracle.grad(n, c, gamma, beta)
    scale = max(1.0, np.max(np.abs(np.concatenate([dgr, dbr]))))
    tol = 1e-9 if dtype == "complex128" else 1e-5
    assert abs(out[0] - Er) <= tol * max(1.0, abs(Er))
    assert np.max(np.abs(out[1:1 + p] - dgr)) <= tol * scale
    assert np.max(np.abs(out[1 + p:] - dbr)) <= tol * scale
