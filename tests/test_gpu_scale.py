"""Full-size GPU checks at the benchmark's sizes that complement the element-wise
oracle comparisons of the benchmarked evaluations (LABS n=26 p=10 complex128 and
n=31 p=10 complex64, in test_gpu_bench_parity.py):
  * cost vector at sampled basis states against the oracle's direct LABS sum,
    including n=33 (indices above 2^32);
  * a full element-by-element oracle comparison at n=26 for p=1 (unfused plan);
  * properties that hold at any size: norm conservation, beta=0 gives the mean
    of c (= n(n-1)/2 for LABS), gamma=0 gives exp(-i n sum beta)|+>,
    E(-gamma, -beta) = E(gamma, beta), LABS E(gamma_l + pi) = E,
    complex64 and complex128 agree, and repeated runs are bitwise identical.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_04841_amd as q
    return q


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _E(q, n, diag, off, gamma, beta, psi, out):
    q.qaoa_evolve(n, gamma, beta, diag, psi, init=True, diag_offset=off, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy().copy()


@pytest.fixture(scope="module")
def labs26(q):
    cfg = W.C2A()
    n = cfg["n"]
    _say("precompute LABS n=26 i32")
    diag, off = q.qaoa_precompute_diag(n, cfg["terms"], "i32", device="cuda")
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    yield cfg, diag, off, psi, out
    del diag, psi, out
    torch.cuda.empty_cache()


def test_n26_cost_vector_sampled(q, labs26):
    cfg, diag, off, _, _ = labs26
    n = cfg["n"]
    rng = np.random.default_rng(26)
    xs = np.concatenate([[0, (1 << n) - 1], rng.integers(0, 1 << n, size=8192)])
    got = diag[torch.from_numpy(xs).cuda()].cpu().numpy().astype(np.int64) + int(off)
    assert np.array_equal(got, oracle.diag_labs_at(n, xs))
    # sum over all x equals N * n(n-1)/2 (the mean of each C_k^2 is n - k)
    assert int(diag.to(torch.int64).sum().item()) == (1 << n) * n * (n - 1) // 2


def test_n26_p1_full_oracle(q, labs26):
    cfg, diag, off, psi, out = labs26
    n = cfg["n"]
    gamma, beta = cfg["gamma"][:1], cfg["beta"][:1]
    _say("n=26 p=1 GPU")
    eo = _E(q, n, diag, off, gamma, beta, psi, out)
    _say("n=26 p=1 oracle")
    c = oracle.diag_labs(n).astype(np.float64)
    ref = oracle.evolve(n, c, gamma, beta)
    E, nrm = oracle.expectation(n, ref, c)
    got = psi.cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-10
    assert abs(eo[0] - E) <= 1e-10 * abs(E)
    assert abs(eo[1] - nrm) <= 1e-10


def test_n26_p10_properties(q, labs26):
    cfg, diag, off, psi, out = labs26
    n, g, b = cfg["n"], cfg["gamma"], cfg["beta"]
    _say("n=26 p=10 properties")
    e1 = _E(q, n, diag, off, g, b, psi, out)
    h1 = psi[:: 4099].clone()
    e2 = _E(q, n, diag, off, g, b, psi, out)
    assert np.array_equal(e1, e2) and torch.equal(h1, psi[:: 4099])
    assert abs(e1[1] - 1.0) <= 1e-10
    # E is a convex combination of cost values: 0 <= E <= max c = sum_k (n-k)^2
    assert 0.0 <= e1[0] <= sum((n - k) ** 2 for k in range(1, n))
    er = _E(q, n, diag, off, -g, -b, psi, out)
    assert abs(er[0] - e1[0]) <= 1e-10 * e1[0]
    g2 = g.copy(); g2[3] += np.pi
    es = _E(q, n, diag, off, g2, b, psi, out)
    assert abs(es[0] - e1[0]) <= 1e-10 * e1[0]
    e0 = _E(q, n, diag, off, g, np.zeros_like(b), psi, out)
    assert abs(e0[0] - n * (n - 1) / 2) <= 1e-10 * e0[0]
    _E(q, n, diag, off, np.zeros_like(g), b, psi, out)
    ref = np.exp(-1j * n * b.sum()) * 2.0 ** (-n / 2)
    assert torch.max(torch.abs(psi - torch.tensor(ref, dtype=torch.complex128, device="cuda"))).item() < 1e-14


def test_n31_c64_properties(q):
    cfg = W.C2B()
    n, g, b = cfg["n"], cfg["gamma"], cfg["beta"]
    _say("precompute LABS n=31 u16")
    diag, off = q.qaoa_precompute_diag(n, cfg["terms"], "u16", device="cuda")
    rng = np.random.default_rng(31)
    xs = np.concatenate([[0, (1 << n) - 1], rng.integers(0, 1 << n, size=4096)])
    # torch has no uint16 gather on the GPU: gather the bits as int16
    raw = diag.view(torch.int16)[torch.from_numpy(xs).cuda()].cpu().numpy().astype(np.int64) & 0xFFFF
    assert np.array_equal(raw + int(off), oracle.diag_labs_at(n, xs))
    psi = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    _say("n=31 c64 p=10")
    e1 = _E(q, n, diag, off, g, b, psi, out)
    h1 = psi[:: 1000003].clone()
    e2 = _E(q, n, diag, off, g, b, psi, out)
    assert np.array_equal(e1, e2) and torch.equal(h1, psi[:: 1000003])
    assert abs(e1[1] - 1.0) <= 1e-5
    er = _E(q, n, diag, off, -g, -b, psi, out)
    assert abs(er[0] - e1[0]) <= 1e-5 * e1[0]
    e0 = _E(q, n, diag, off, g, np.zeros_like(b), psi, out)
    assert abs(e0[0] - n * (n - 1) / 2) <= 1e-5 * e0[0]
    del psi
    torch.cuda.empty_cache()
    _say("n=31 c128 p=10 (cross-check of the complex64 path)")
    psi128 = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    e128 = _E(q, n, diag, off, g, b, psi128, out)
    assert abs(e128[1] - 1.0) <= 1e-10
    assert abs(e1[0] - e128[0]) <= 1e-5 * e128[0]
    del psi128, diag
    torch.cuda.empty_cache()


def test_n33_c64_beyond_32bit_indices(q):
    """2^33 elements (64 GiB complex64 state): every index computation above
    2^32.  Cost values at sampled high indices against the oracle; beta=0 gives
    E = n(n-1)/2 exactly in exact arithmetic; gamma=0 gives the same amplitude
    exp(-i n sum beta) 2^{-n/2} at every index, checked at sampled high ones."""
    n = 33
    _say("precompute LABS n=33 u16")
    diag, off = q.qaoa_precompute_diag(n, W.labs_terms(n), "u16", device="cuda")
    rng = np.random.default_rng(33)
    xs = np.concatenate([[0, (1 << 32) - 1, 1 << 32, (1 << n) - 1],
                         rng.integers(1 << 32, 1 << n, size=2048), rng.integers(0, 1 << 32, size=1024)])
    idx = torch.from_numpy(xs).cuda()
    raw = diag.view(torch.int16)[idx].cpu().numpy().astype(np.int64) & 0xFFFF
    assert np.array_equal(raw + int(off), oracle.diag_labs_at(n, xs))
    psi = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    g, b = np.array([0.21, 0.33]), np.array([0.61, 0.17])
    _say("n=33 c64 p=2 beta=0")
    e0 = _E(q, n, diag, off, g, np.zeros(2), psi, out)
    assert abs(e0[0] - n * (n - 1) / 2) <= 1e-5 * e0[0] and abs(e0[1] - 1.0) <= 1e-5
    _say("n=33 c64 p=2 gamma=0")
    _E(q, n, diag, off, np.zeros(2), b, psi, out)
    ref = np.exp(-1j * n * b.sum()) * 2.0 ** (-n / 2)
    got = psi[idx].cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - ref)) <= 1e-5 * abs(ref)
    _say("n=33 c64 p=2")
    e1 = _E(q, n, diag, off, g, b, psi, out)
    assert abs(e1[1] - 1.0) <= 1e-5
    assert 0.0 <= e1[0] <= sum((n - k) ** 2 for k in range(1, n))
    del psi, diag
    torch.cuda.empty_cache()
