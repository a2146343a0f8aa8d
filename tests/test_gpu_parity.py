"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Sizes span the single-tile path (whole state in one workgroup, all layers in
one launch), the multi-sweep path (several tiles, ragged active-bit counts)
and edge cases (n=1..3, p=0, long single-tile chains, odd-order terms).

Tolerances (from the required accuracy):
  cost vector        bit-exact for integer dtypes; F64 exact for dyadic weights,
                     |dc| <= 1e-12 * sum|w| otherwise
  complex128         ||psi - psi_ref||_2 <= 1e-10, |dE| <= 1e-10 * max(1, |E|)
  complex64          ||psi - psi_ref||_2 <= 1e-5,  |dE| <= 1e-5  * max(1, |E|)
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"complex128": (1e-10, 1e-10), "complex64": (1e-5, 1e-5)}


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


def _c_of(q, n, terms, ddt):
    diag, off = q.qaoa_precompute_diag(n, terms, ddt, device="cuda")
    return diag, off


def _run(q, n, diag, off, gamma, beta, dtype, psi0=None):
    psi = torch.empty(1 << n, dtype=_tdtype(dtype), device="cuda")
    if psi0 is not None:
        psi.copy_(torch.from_numpy(psi0).to(_tdtype(dtype)))
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    q.qaoa_evolve(n, gamma, beta, diag, psi, init=psi0 is None, diag_offset=off, out=out)
    torch.cuda.synchronize()
    return psi.cpu().numpy().astype(np.complex128), out.cpu().numpy()


def _compare(n, psi, eo, c, gamma, beta, dtype, psi0=None):
    ref = oracle.evolve(n, c, gamma, beta, psi0=psi0)
    E, nrm = oracle.expectation(n, ref, c)
    tpsi, te = TOL[dtype]
    dpsi = np.linalg.norm(psi - ref)
    assert dpsi <= tpsi, f"||dpsi|| = {dpsi:.3e}"
    assert abs(eo[0] - E) <= te * max(1.0, abs(E)), f"E gpu {eo[0]!r} oracle {E!r}"
    assert abs(eo[1] - nrm) <= te * max(1.0, abs(nrm)), f"norm gpu {eo[1]!r} oracle {nrm!r}"


# ---------------------------------------------------------------------------
# cost vector
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 5, 13, 16, 20])
@pytest.mark.parametrize("ddt", ["i32", "u16", "f64"])
def test_precompute_labs_bit_exact(q, n, ddt):
    _say(f"precompute labs n={n} {ddt}")
    diag, off = _c_of(q, n, W.labs_terms(n), ddt)
    got = diag.cpu().numpy().astype(np.int64) + int(off) if ddt != "f64" else diag.cpu().numpy()
    ref = oracle.diag_labs(n)
    assert np.array_equal(np.asarray(got, dtype=np.float64), ref.astype(np.float64))


@pytest.mark.parametrize("ddt", ["i32", "u16", "f64"])
def test_precompute_weighted_maxcut_bit_exact(q, ddt):
    n = 14
    edges, weights = W.erdos_renyi_graph(n, 0.4, seed=21)
    _say(f"precompute maxcut n={n} {ddt}")
    diag, off = _c_of(q, n, W.maxcut_terms(edges, weights), ddt)
    got = diag.cpu().numpy().astype(np.float64) + off
    assert np.array_equal(got, oracle.diag_maxcut(n, edges, weights))


@pytest.mark.parametrize("ddt", ["i32", "u16", "f64"])
def test_precompute_random_odd_terms_bit_exact(q, ddt):
    n = 15
    terms = W.random_terms(n, 60, seed=3, max_order=5, integer=True, wmax=20)
    _say(f"precompute random n={n} {ddt}")
    diag, off = _c_of(q, n, terms, ddt)
    got = diag.cpu().numpy().astype(np.float64) + off
    assert np.array_equal(got, oracle.diag_terms(n, terms))


def test_precompute_u16_wide_range_uses_workspace(q):
    # 2 sum|w| >= 2^16 but max - min < 2^16: the int32 scratch path must be taken.
    # c = w (s0 + s1 + s0 s1) takes values {3w, -w}: range 4w, sum|w| = 3w.
    n = 12
    w = 12000.0
    terms = [(w, (0,)), (w, (1,)), (w, (0, 1)), (-3.0, (5, 7)), (3.0, ())]
    diag, off = _c_of(q, n, terms, "u16")
    got = diag.cpu().numpy().astype(np.float64) + off
    assert np.array_equal(got, oracle.diag_terms(n, terms))


def test_precompute_non_dyadic_f64_and_i32_range(q):
    n = 10
    terms = [(0.3, (i, j)) for i in range(n) for j in range(i + 1, n)]  # Listing 1 style
    diag, off = _c_of(q, n, terms, "f64")
    ref = oracle.diag_terms(n, terms)
    assert np.max(np.abs(diag.cpu().numpy() - ref)) <= 1e-12 * 0.3 * len(terms)
    with pytest.raises(q.QaoaError, match="RANGE"):
        _c_of(q, n, terms, "i32")
    with pytest.raises(q.QaoaError, match="RANGE"):
        _c_of(q, n, [(70000.0, (0,)), (1.0, ())], "u16")


def test_precompute_degenerate_terms(q):
    n = 7
    for terms in ([], [(5.0, ())], [(2.0, (3, 3))], [(0.0, (1, 2)), (1.0, (0, 0, 4))]):
        for ddt in ("i32", "u16", "f64"):
            diag, off = _c_of(q, n, terms, ddt)
            got = diag.cpu().numpy().astype(np.float64) + off
            assert np.array_equal(got, oracle.diag_terms(n, terms) if terms else np.zeros(1 << n)), (terms, ddt)


# ---------------------------------------------------------------------------
# evolution and objective
# ---------------------------------------------------------------------------
EVOLVE_CASES = []
for n in (1, 2, 3, 4, 5, 8, 11, 12, 13, 14, 17, 20):
    EVOLVE_CASES.append((n, "complex128"))
for n in (1, 3, 7, 13, 14, 15, 18, 21):
    EVOLVE_CASES.append((n, "complex64"))


@pytest.mark.parametrize("n,dtype", EVOLVE_CASES)
def test_evolve_random_terms(q, n, dtype):
    p = 3
    terms = W.random_terms(n, 4 * n + 3, seed=n, max_order=4, integer=True, wmax=6)
    rng = np.random.default_rng(1000 + n)
    gamma, beta = rng.uniform(-1, 1, size=p), rng.uniform(-np.pi, np.pi, size=p)
    _say(f"evolve random n={n} {dtype}")
    diag, off = _c_of(q, n, terms, "i32")
    psi, eo = _run(q, n, diag, off, gamma, beta, dtype)
    _compare(n, psi, eo, oracle.diag_terms(n, terms), gamma, beta, dtype)


@pytest.mark.parametrize("n,dtype,ddt", [(10, "complex128", "u16"), (16, "complex128", "u16"),
                                         (19, "complex128", "i32"), (16, "complex64", "u16"),
                                         (20, "complex64", "i32")])
def test_evolve_labs_ramp(q, n, dtype, ddt):
    p = 4
    gamma, beta = W.linear_ramp(p, seed=n)
    _say(f"evolve labs n={n} {dtype} {ddt}")
    diag, off = _c_of(q, n, W.labs_terms(n), ddt)
    psi, eo = _run(q, n, diag, off, gamma, beta, dtype)
    _compare(n, psi, eo, oracle.diag_labs(n).astype(np.float64), gamma, beta, dtype)


@pytest.mark.parametrize("n,p", [(22, 3), (23, 2), (25, 1)])
def test_evolve_wide_complex128_tiles(q, n, p):
    # 2^22..2^25 complex128 elements run 2^14-element tiles (1024 threads, LDS
    # exchanges split into real and imaginary passes), two sweeps per layer
    from paper_2309_04841_amd import _lib
    assert _lib.plan_describe(n, _lib.QAOA_C128)["wide"]
    gamma, beta = W.linear_ramp(p, seed=n)
    if n % 2:
        terms = W.maxcut_terms(W.random_regular_graph(4, n, seed=n))  # d n must be even
    else:
        terms = W.labs_terms(n)
    _say(f"evolve wide n={n} p={p}")
    diag, off = _c_of(q, n, terms, "i32")
    psi, eo = _run(q, n, diag, off, gamma, beta, "complex128")
    _compare(n, psi, eo, oracle.diag_terms(n, terms), gamma, beta, "complex128")


@pytest.mark.parametrize("n,dtype", [(10, "complex128"), (16, "complex128"), (22, "complex128"),
                                     (12, "complex64"), (18, "complex64")])
def test_evolve_int32_beyond_two_level_table(q, n, dtype):
    # most int32 cost values lie outside [-2^15, 2^15): those workgroups take the
    # two-pass byte-table phase (single tile, narrow, wide and complex64 tiles)
    p = 3
    terms = W.random_terms(n, 4 * n, seed=50 + n, max_order=3, integer=True, wmax=9000)
    c = oracle.diag_terms(n, terms)
    assert np.abs(c).max() >= 32768
    rng = np.random.default_rng(77 + n)
    gamma, beta = rng.uniform(-0.05, 0.05, size=p), rng.uniform(-np.pi, np.pi, size=p)
    _say(f"evolve int32 wide range n={n} {dtype}")
    diag, off = _c_of(q, n, terms, "i32")
    psi, eo = _run(q, n, diag, off, gamma, beta, dtype)
    _compare(n, psi, eo, c, gamma, beta, dtype)


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_evolve_weighted_maxcut_f64_diag(q, dtype):
    n = 16
    edges, weights = W.erdos_renyi_graph(n, 0.3, seed=8)
    terms = [(0.37 * w, e) for (w, e) in W.maxcut_terms(edges, weights)]  # non-dyadic: F64 cost vector
    gamma, beta = W.uniform_angles(3, seed=9)
    diag, off = _c_of(q, n, terms, "f64")
    psi, eo = _run(q, n, diag, off, gamma, beta, dtype)
    # the oracle uses its own term-by-term cost vector (rounding may differ by ~1 ulp)
    _compare(n, psi, eo, oracle.diag_terms(n, terms), gamma, beta, dtype)


def test_c1_workload_and_closed_form(q):
    from dense_ref import maxcut_p1_closed_form
    cfg = W.C1()
    n = cfg["n"]
    diag, off = _c_of(q, n, cfg["terms"], "i32")
    psi, eo = _run(q, n, diag, off, cfg["gamma"], cfg["beta"], "complex128")
    _compare(n, psi, eo, oracle.diag_maxcut(n, cfg["edges"]), cfg["gamma"], cfg["beta"], "complex128")
    ref = -maxcut_p1_closed_form(n, cfg["edges"], -cfg["gamma"][0], cfg["beta"][0])
    assert abs(eo[0] - ref) < 1e-12


@pytest.mark.parametrize("n,dtype", [(9, "complex128"), (18, "complex128"), (16, "complex64")])
def test_evolve_from_given_state(q, n, dtype):
    rng = np.random.default_rng(n)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    if dtype == "complex64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    terms = W.random_terms(n, 30, seed=2 * n, integer=True)
    gamma, beta = rng.uniform(-1, 1, size=2), rng.uniform(-1, 1, size=2)
    diag, off = _c_of(q, n, terms, "i32")
    psi, eo = _run(q, n, diag, off, gamma, beta, dtype, psi0=psi0)
    _compare(n, psi, eo, oracle.diag_terms(n, terms), gamma, beta, dtype, psi0=psi0)


@pytest.mark.parametrize("n,p", [(6, 40), (12, 33), (5, 0), (15, 0)])
def test_evolve_layer_counts(q, n, p):
    # p > 32 chains several single-tile launches; p = 0 is |+> (or the input) alone
    rng = np.random.default_rng(p + n)
    gamma, beta = rng.uniform(-1, 1, size=p), rng.uniform(-1, 1, size=p)
    diag, off = _c_of(q, n, W.labs_terms(n), "i32")
    psi, eo = _run(q, n, diag, off, gamma, beta, "complex128")
    _compare(n, psi, eo, oracle.diag_labs(n).astype(np.float64), gamma, beta, "complex128")


def test_special_angles(q):
    n = 15
    diag, off = _c_of(q, n, W.labs_terms(n), "i32")
    c = oracle.diag_labs(n).astype(np.float64)
    # beta = 0: E is the mean of c = n(n-1)/2
    _, eo = _run(q, n, diag, off, [0.3, 0.9], [0.0, 0.0], "complex128")
    assert abs(eo[0] - n * (n - 1) / 2) < 1e-10 * n * n
    # gamma = 0: |+> is an eigenvector, psi = exp(-i n sum beta) |+>
    psi, _ = _run(q, n, diag, off, [0.0, 0.0], [0.4, -1.1], "complex128")
    assert np.max(np.abs(psi - np.exp(-1j * n * (0.4 - 1.1)) * 2 ** (-n / 2))) < 1e-14
    # beta = pi/2 on a given state: global bit flip times (-i)^n
    rng = np.random.default_rng(5)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    zero_diag = torch.zeros(1 << n, dtype=torch.int32, device="cuda")
    psi, _ = _run(q, n, zero_diag, 0.0, [0.0], [np.pi / 2], "complex128", psi0=psi0)
    N = 1 << n
    assert np.max(np.abs(psi - (-1j) ** n * psi0[np.arange(N) ^ (N - 1)])) < 1e-14
    del c


# complex64 sweeps compute in FP32 while every layer a launch applies has
# |tan beta| <= 64 and in FP64 otherwise (the tangent-form gates let a tile grow
# by 1/|cos beta| per gate before its rescale).  Layers on both sides of the
# bound, beta = pi/2 exactly, and fused launches that pair a large and a small
# tangent; ragged 2^13-element tiles (n = 18, 21) in both cost dtypes, and the
# single-tile kernel (n = 10), whose FP64 registers exchange through FP32 LDS.
@pytest.mark.parametrize("n,ddt", [(10, "u16"), (18, "u16"), (21, "i32")])
def test_complex64_precision_switch(q, n, ddt):
    _say(f"complex64 precision switch n={n} {ddt}")
    beta = [np.pi / 2, np.arctan(63.9), 0.3, np.pi / 2 - 1e-3, np.arctan(64.1), np.pi / 2 + 0.01, -np.arctan(63.9)]
    gamma = list(np.linspace(0.05, 0.35, len(beta)))
    if ddt == "u16":
        terms, c = W.labs_terms(n), oracle.diag_labs(n).astype(np.float64)
    else:
        edges = W.random_regular_graph(4, n, seed=n)
        weights = list(np.random.default_rng(n).integers(1, 11, size=len(edges)))
        terms = W.maxcut_terms(edges, weights)
        c = oracle.diag_maxcut(n, edges, weights)
    diag, off = _c_of(q, n, terms, ddt)
    psi, eo = _run(q, n, diag, off, gamma, beta, "complex64")
    _compare(n, psi, eo, c, gamma, beta, "complex64")
    # beta = pi/2 alone: the global bit flip times (-i)^n, in FP64 sweeps
    rng = np.random.default_rng(n)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 = (psi0 / np.linalg.norm(psi0)).astype(np.complex64).astype(np.complex128)
    zero_diag = torch.zeros(1 << n, dtype=torch.int32, device="cuda")
    got, _ = _run(q, n, zero_diag, 0.0, [0.0], [np.pi / 2], "complex64", psi0=psi0)
    N = 1 << n
    assert np.max(np.abs(got - (-1j) ** n * psi0[np.arange(N) ^ (N - 1)])) < 1e-6


def test_zero_weight_problem(q):
    n = 14
    diag, off = _c_of(q, n, [(0.0, (0, 1)), (0.0, (2, 5, 7))], "i32")
    _, eo = _run(q, n, diag, off, [0.5, 1.0], [0.3, 0.2], "complex128")
    assert eo[0] == 0.0


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_expectation_standalone(q, dtype):
    n = 17
    rng = np.random.default_rng(17)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    if dtype == "complex64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    t = torch.from_numpy(psi0).to(_tdtype(dtype)).cuda()
    c = oracle.diag_labs(n)
    for ddt, tdt in (("i32", torch.int32), ("f64", torch.float64)):
        diag = torch.from_numpy(c).to(tdt).cuda()
        out = q.qaoa_expectation(n, t, diag).cpu().numpy()
        E, nrm = oracle.expectation(n, psi0, c.astype(np.float64))
        assert abs(out[0] - E) <= 1e-12 * abs(E), ddt
        assert abs(out[1] - nrm) <= 1e-12
    # u16 with an offset: c = stored + offset
    diag16 = torch.from_numpy((c - 3).astype(np.uint16)).cuda()
    out = q.qaoa_expectation(n, t, diag16, diag_offset=3.0).cpu().numpy()
    assert abs(out[0] - oracle.expectation(n, psi0, c.astype(np.float64))[0]) <= 1e-12 * abs(out[0])


@pytest.mark.parametrize("n,dtype", [(12, "complex128"), (20, "complex128"), (21, "complex64")])
def test_deterministic(q, n, dtype):
    diag, off = _c_of(q, n, W.labs_terms(n), "i32")
    gamma, beta = W.linear_ramp(5, seed=1)
    a_psi, a_e = _run(q, n, diag, off, gamma, beta, dtype)
    b_psi, b_e = _run(q, n, diag, off, gamma, beta, dtype)
    assert np.array_equal(a_psi, b_psi) and np.array_equal(a_e, b_e)


def test_simulator_api(q):
    n = 14
    terms = W.labs_terms(n)
    sim = q.Simulator(n, terms=terms, dtype="complex128", diag_dtype="u16")
    c = oracle.diag_labs(n).astype(np.float64)
    assert np.array_equal(sim.get_cost_diagonal(), c)
    gamma, beta = W.linear_ramp(3, seed=4)
    res = sim.simulate_qaoa(gamma, beta)
    ref = oracle.evolve(n, c, gamma, beta)
    assert np.linalg.norm(sim.get_statevector(res) - ref) < 1e-10
    E = sim.get_expectation(res)
    assert abs(E - oracle.expectation(n, ref, c)[0]) < 1e-10 * abs(E)
    # costs= override (Section 4): any vector of the right length
    other = np.arange(1 << n, dtype=np.float64)
    assert abs(sim.get_expectation(res, costs=other) - oracle.expectation(n, ref, other)[0]) < 1e-9 * (1 << n)
    sim2 = q.Simulator(n, costs=c, dtype="complex64")
    res2 = sim2.simulate_qaoa(gamma, beta)
    assert abs(sim2.get_expectation(res2) - E) < 1e-5 * abs(E)
    p = sim.get_probabilities(res)
    assert abs(p.sum() - 1.0) < 1e-12
