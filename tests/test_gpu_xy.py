"""GPU parity of the XY mixers (Section 3.2, ring and complete graph) against the
FP64 oracle: single-tile states (all layers in one launch), multi-sweep states
(the planner's commuted gate order), |+>^n, Dicke and caller-given starts, p = 0,
more than one chunk of prepared layers, and Hamming-weight conservation at the
largest sizes.  Tolerances as for the X mixer: complex128 ||dpsi|| <= 1e-10,
complex64 1e-5; the same relative bounds on E and sum |psi|^2."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"complex128": 1e-10, "complex64": 1e-5}
KIND = {1: oracle.XY_RING, 2: oracle.XY_COMPLETE}


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_04841_amd as q
    return q


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _tdtype(name):
    return {"complex128": torch.complex128, "complex64": torch.complex64}[name]


def _portfolio_terms(n, seed):
    # order <= 2 spin polynomial with real weights: the shape of a
    # mean-variance portfolio objective written in spins
    return W.random_terms(n, 3 * n, seed, max_order=2, integer=False, wmax=2)


def _run(q, n, terms, ddt, gamma, beta, mixer, dtype, init, k=0, psi0=None):
    diag, off = q.qaoa_precompute_diag(n, terms, ddt, device="cuda")
    psi = torch.empty(1 << n, dtype=_tdtype(dtype), device="cuda")
    if psi0 is not None:
        psi.copy_(torch.from_numpy(psi0).to(_tdtype(dtype)))
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    q.qaoa_evolve_xy(n, gamma, beta, diag, psi, mixer=mixer, init=init, k=k, diag_offset=off, out=out)
    torch.cuda.synchronize()
    return psi.cpu().numpy().astype(np.complex128), out.cpu().numpy()


def _check(n, terms, gamma, beta, mixer, dtype, psi, eo, init, k=0, psi0=None):
    c = oracle.diag_terms(n, terms)
    ref = oracle.evolve_xy(n, c, gamma, beta, KIND[mixer], init=init, k=k, psi0=psi0)
    E, nrm = oracle.expectation(n, ref, c)
    tol = TOL[dtype]
    d = np.linalg.norm(psi - ref)
    assert d <= tol, f"||dpsi|| = {d:.3e}"
    assert abs(eo[0] - E) <= tol * max(1.0, abs(E)), f"E gpu {eo[0]!r} oracle {E!r}"
    assert abs(eo[1] - nrm) <= tol * max(1.0, abs(nrm))


@pytest.mark.parametrize("n", [2, 3, 5, 8, 12])
@pytest.mark.parametrize("mixer", [1, 2])
def test_xy_single_tile_labs(q, n, mixer):
    _say(f"xy single tile n={n} mixer={mixer}")
    terms = W.labs_terms(n)
    gamma, beta = W.linear_ramp(3, seed=n)
    psi, eo = _run(q, n, terms, "i32", gamma, beta, mixer, "complex128", q._lib.INIT_PLUS)
    _check(n, terms, gamma, beta, mixer, "complex128", psi, eo, "plus")


@pytest.mark.parametrize("n", [13, 14, 17])
@pytest.mark.parametrize("mixer", [1, 2])
@pytest.mark.parametrize("dtype,ddt", [("complex128", "i32"), ("complex64", "u16")])
def test_xy_multi_sweep_labs(q, n, mixer, dtype, ddt):
    _say(f"xy multi sweep n={n} mixer={mixer} {dtype} {ddt}")
    terms = W.labs_terms(n)
    gamma, beta = W.linear_ramp(2, seed=n + mixer)
    psi, eo = _run(q, n, terms, ddt, gamma, beta, mixer, dtype, q._lib.INIT_PLUS)
    _check(n, terms, gamma, beta, mixer, dtype, psi, eo, "plus")


@pytest.mark.parametrize("n,k", [(6, 0), (6, 3), (6, 6), (14, 4), (15, 7)])
@pytest.mark.parametrize("mixer", [1, 2])
def test_xy_dicke_portfolio(q, n, k, mixer):
    _say(f"xy dicke n={n} k={k} mixer={mixer}")
    terms = _portfolio_terms(n, seed=100 + n)
    gamma, beta = W.linear_ramp(3, seed=k)
    psi, eo = _run(q, n, terms, "f64", gamma, beta, mixer, "complex128", q._lib.INIT_DICKE, k=k)
    _check(n, terms, gamma, beta, mixer, "complex128", psi, eo, "dicke", k=k)
    # the mixer and the phase keep the state inside the weight-k subspace
    w = np.array([bin(x).count("1") for x in range(1 << n)])
    assert np.sum(np.abs(psi[w != k]) ** 2) < 1e-24


@pytest.mark.parametrize("n", [9, 16])
@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_xy_from_given_state(q, n, dtype):
    _say(f"xy given state n={n} {dtype}")
    rng = np.random.default_rng(n)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    if dtype == "complex64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    terms = W.random_terms(n, 20, seed=n)
    gamma, beta = W.linear_ramp(2, seed=3)
    psi, eo = _run(q, n, terms, "i32", gamma, beta, 1, dtype, q._lib.INIT_GIVEN, psi0=psi0)
    _check(n, terms, gamma, beta, 1, dtype, psi, eo, "given", psi0=psi0)


@pytest.mark.parametrize("n", [4, 13])
def test_xy_p0(q, n):
    _say(f"xy p=0 n={n}")
    terms = W.labs_terms(n)
    for init, name, k in ((q._lib.INIT_PLUS, "plus", 0), (q._lib.INIT_DICKE, "dicke", 2)):
        psi, eo = _run(q, n, terms, "i32", [], [], 2, "complex128", init, k=k)
        _check(n, terms, [], [], 2, "complex128", psi, eo, name, k=k)


@pytest.mark.parametrize("n", [10, 13])
def test_xy_more_layers_than_one_prep_chunk(q, n):
    _say(f"xy p=37 n={n}")
    terms = W.labs_terms(n)
    gamma, beta = W.linear_ramp(37, seed=5)
    psi, eo = _run(q, n, terms, "u16", gamma, beta, 1, "complex128", q._lib.INIT_PLUS)
    _check(n, terms, gamma, beta, 1, "complex128", psi, eo, "plus")


@pytest.mark.parametrize("n,mixer", [(24, 1), (22, 2)])
def test_xy_large_state_conserves_weight(q, n, mixer):
    """Larger states: properties that hold at any size (norm 1, all mass in the
    Dicke weight-k subspace), and the whole state against the oracle where it
    finishes in seconds (one layer, n <= 22)."""
    _say(f"xy large n={n} mixer={mixer}")
    k = n // 3
    terms = W.labs_terms(n)
    psi, eo = _run(q, n, terms, "u16", [0.31], [0.77], mixer, "complex128", q._lib.INIT_DICKE, k=k)
    assert abs(eo[1] - 1.0) < 1e-10
    xs = np.arange(1 << n, dtype=np.int64)
    w = np.zeros(1 << n, dtype=np.int64)
    for b in range(n):
        w += (xs >> b) & 1
    assert np.sum(np.abs(psi[w != k]) ** 2) < 1e-24
    if n <= 22:
        c = oracle.diag_terms(n, terms)
        ref = oracle.evolve_xy(n, c, [0.31], [0.77], KIND[mixer], init="dicke", k=k)
        assert np.linalg.norm(psi - ref) <= 1e-10
