"""Request loop (continuous batching): objective and gradient requests of mixed
n and p, admitted by device footprint, overlapping on several streams.

* every result equals the same request run alone through qaoa_evolve /
  qaoa_grad (bitwise: each request owns its buffers, reductions are fixed-order);
* with an arena that fits only a few requests, all complete and the peak use
  stays within the arena (requests wait for memory instead of failing);
* a request that can never fit is rejected at submit;
* latency percentiles are reported.
"""
import threading
import time

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


TD = {"complex64": torch.complex64, "complex128": torch.complex128}


def _problems(ns):
    probs = []
    for i, n in enumerate(ns):
        if i % 2 == 0:
            probs.append((n, W.labs_terms(n)))
        else:
            probs.append((n, W.maxcut_terms(W.random_regular_graph(3, n, seed=n))))
    return probs


def _requests(probs, count, seed, pmax=12):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        k = int(rng.integers(0, len(probs)))
        p = int(rng.integers(1, pmax + 1))
        grad = bool(rng.random() < 0.4)
        g, b = rng.uniform(0, 1, size=p), rng.uniform(0, np.pi, size=p)
        reqs.append((k, g, b, grad))
    return reqs


def _alone(q, n, terms, g, b, grad, dtype):
    diag, off = q.qaoa_precompute_diag(n, terms, "i32", device="cuda")
    psi = torch.empty(1 << n, dtype=TD[dtype], device="cuda")
    if grad:
        adj = torch.empty_like(psi)
        return q.qaoa_grad(n, g, b, diag, psi, adj, diag_offset=off).cpu().numpy()
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    q.qaoa_evolve(n, g, b, diag, psi, diag_offset=off, out=out)
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype", ["complex64", "complex128"])
def test_mix_equals_alone(q, dtype):
    probs = _problems([14, 16, 17, 18, 13, 20])
    reqs = _requests(probs, 48, seed=7)
    results = {}
    with q.QAOAServer(arena_bytes=2 << 30, num_streams=4, max_in_flight=8) as srv:
        pids = [srv.add_problem(n, terms) for n, terms in probs]
        tickets = []

        def submitter():
            rng = np.random.default_rng(11)
            for i, (k, g, b, grad) in enumerate(reqs):
                tickets.append((i, srv.submit(pids[k], g, b, gradient=grad, dtype=dtype)))
                time.sleep(float(rng.exponential(0.0005)))  # Poisson arrivals

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        for i, t in tickets:
            out, lat = srv.wait(t)
            assert lat > 0
            results[i] = out
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert 0 < st["p50_s"] <= st["p99_s"] <= st["max_s"]
    for i, (k, g, b, grad) in enumerate(reqs):
        n, terms = probs[k]
        ref = _alone(q, n, terms, g, b, grad, dtype)
        got = results[i][:len(ref)]
        if grad:
            assert np.array_equal(got, ref), i
        else:
            assert np.array_equal(got, ref), i


def test_tight_arena_admission(q):
    n = 18
    terms = W.labs_terms(n)
    state = 8 << n
    arena = (4 << n) + 3 * state + (2 << 20)  # cost vector + about two requests at a time
    reqs = _requests([(n, terms)], 24, seed=3, pmax=6)
    with q.QAOAServer(arena_bytes=arena, num_streams=3, max_in_flight=16) as srv:
        pid = srv.add_problem(n, terms)
        tickets = [srv.submit(pid, g, b, gradient=grad) for (_, g, b, grad) in reqs]
        outs = [srv.wait(t)[0] for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["peak_bytes"] <= st["arena_bytes"]
    for (k, g, b, grad), out in zip(reqs, outs):
        ref = _alone(q, n, terms, g, b, grad, "complex64")
        assert np.array_equal(out[:len(ref)], ref)


def test_oversize_request_rejected(q):
    n = 16
    with q.QAOAServer(arena_bytes=(2 << n) + (1 << 20), num_streams=1, max_in_flight=2) as srv:
        pid = srv.add_problem(n, W.labs_terms(n), diag_dtype="u16")
        with pytest.raises(q.QaoaError, match="NOMEM"):
            srv.submit(pid, [0.1], [0.2], dtype="complex128")
