"""qaoa_evolve_noalloc (no workspace argument, static per-GPU scratch) against
qaoa_evolve with a caller workspace: same kernels and reduction order, so the
state and (E, sum |psi|^2) must be bitwise equal.  Two calls in a row share the
static scratch, the second on a smaller input, then a third on a one-tile
state; the first call's scratch contents must not leak into the later ones."""
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_04841_amd as q
    return q


def _run(q, n, terms, ddt, sdt, gamma, beta, noalloc):
    diag, off = q.qaoa_precompute_diag(n, terms, ddt, device="cuda")
    psi = torch.empty(1 << n, dtype=sdt, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    if noalloc:
        q.qaoa_evolve_noalloc(n, gamma, beta, diag, psi, init=True, diag_offset=off, out=out)
    else:
        q.qaoa_evolve(n, gamma, beta, diag, psi, init=True, diag_offset=off, out=out)
    torch.cuda.synchronize()
    return psi.cpu(), out.cpu()


CASES = [  # (n, problem, cost dtype, state dtype, p): large first, then smaller
    (26, "labs", "u16", torch.complex128, 4),  # qaoa_evolve's workspace holds a second state here; noalloc runs in place
    (24, "labs", "u16", torch.complex128, 5),
    (17, "random", "i32", torch.complex64, 3),
    (11, "labs", "i32", torch.complex128, 2),
]


def test_noalloc_matches_evolve(q):
    for n, problem, ddt, sdt, p in CASES:
        print(f"noalloc: n={n} {problem} {ddt} {sdt} p={p}", file=sys.stderr, flush=True)
        if problem == "labs":
            terms = W.labs_terms(n)
            gamma, beta = W.linear_ramp(p, seed=40 + n)
        else:
            terms = W.random_terms(n, 2 * n, seed=41 + n, max_order=4, integer=True, wmax=5)
            rng = np.random.default_rng(42 + n)
            gamma, beta = rng.uniform(-1, 1, size=p), rng.uniform(-np.pi, np.pi, size=p)
        psi_ref, out_ref = _run(q, n, terms, ddt, sdt, gamma, beta, noalloc=False)
        psi, out = _run(q, n, terms, ddt, sdt, gamma, beta, noalloc=True)
        assert torch.equal(out, out_ref), (out, out_ref)
        assert torch.equal(psi, psi_ref)
        assert abs(float(out[1]) - 1.0) < 1e-5


def test_noalloc_rejects_oversize(q):
    from paper_2309_04841_amd import _lib
    diag = torch.empty(1 << 10, dtype=torch.int32, device="cuda")
    psi = torch.empty(1 << 10, dtype=torch.complex128, device="cuda")
    # a state of 2^32 complex128 entries is never allocated: the size check
    # fails on the host before anything is enqueued
    g = (np.array([0.1]),)
    rc = _lib.lib.qaoa_evolve_noalloc(32, 1, _lib._f64(g[0]), _lib._f64(g[0]), diag.data_ptr(), _lib.QAOA_DIAG_I32,
                                      0.0, 4 << 32, psi.data_ptr(), _lib.QAOA_C128, 16 << 32, 1, None,
                                      _lib._stream(psi.device))
    assert rc == _lib.QAOA_ERR_NOMEM
