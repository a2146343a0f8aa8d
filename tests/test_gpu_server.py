"""Request loop (continuous batching): objective and gradient requests of mixed
n and p, admitted by device footprint, overlapping on several streams.

* every result equals the same request run alone through qaoa_evolve /
  qaoa_grad (bitwise: each request owns its buffers, reductions are fixed-order);
* a sample of served objective and gradient results equals the FP64 oracle's
  (complex128: 1e-10 on E, 1e-9 of the largest gradient component; complex64:
  1e-5);
* with an arena that fits only a few requests, all complete and the peak use
  stays within the arena (requests wait for memory instead of failing);
* a request that can never fit is rejected at submit;
* destroying the server with requests still queued returns (they are dropped);
* latency percentiles are reported.
"""
import threading
import time

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


TD = {"complex64": torch.complex64, "complex128": torch.complex128}


def _problems(ns):
    probs = []
    for i, n in enumerate(ns):
        if i % 2 == 0:
            probs.append((n, W.labs_terms(n)))
        else:
            d = 3 if n % 2 == 0 else 4  # a d-regular graph on n vertices needs d n even
            probs.append((n, W.maxcut_terms(W.random_regular_graph(d, n, seed=n))))
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


def test_served_results_match_oracle(q):
    probs = _problems([12, 15, 17, 13])
    reqs = _requests(probs, 20, seed=21, pmax=8)
    dtypes = ["complex64" if i % 2 == 0 else "complex128" for i in range(len(reqs))]
    with q.QAOAServer(arena_bytes=1 << 30, num_streams=4, max_in_flight=8) as srv:
        pids = [srv.add_problem(n, terms) for n, terms in probs]
        tickets = [srv.submit(pids[k], g, b, gradient=grad, dtype=dt) for (k, g, b, grad), dt in zip(reqs, dtypes)]
        outs = [srv.wait(t)[0] for t in tickets]
    assert any(r[3] for r in reqs) and not all(r[3] for r in reqs)
    for i, ((k, g, b, grad), dt, out) in enumerate(zip(reqs, dtypes, outs)):
        n, terms = probs[k]
        c = oracle.diag_terms(n, terms)
        p = len(g)
        if grad:
            Er, dgr, dbr = oracle.grad(n, c, g, b)
            tol = 1e-9 if dt == "complex128" else 1e-5
            scale = max(1.0, float(np.max(np.abs(np.concatenate([dgr, dbr])))))
            assert abs(out[0] - Er) <= tol * max(1.0, abs(Er)), i
            assert np.max(np.abs(out[1:1 + p] - dgr)) <= tol * scale, i
            assert np.max(np.abs(out[1 + p:1 + 2 * p] - dbr)) <= tol * scale, i
        else:
            Er, nrm = oracle.expectation(n, oracle.evolve(n, c, g, b), c)
            tol = 1e-10 if dt == "complex128" else 1e-5
            assert abs(out[0] - Er) <= tol * max(1.0, abs(Er)), i
            assert abs(out[1] - nrm) <= tol, i


def test_destroy_with_queued_requests_returns(q):
    n = 20
    srv = q.QAOAServer(arena_bytes=1 << 30, num_streams=2, max_in_flight=2)
    pid = srv.add_problem(n, W.labs_terms(n))
    for i in range(40):
        srv.submit(pid, [0.1, 0.2, 0.3], [0.4, 0.5, 0.6], gradient=(i % 3 == 0))
    t0 = time.perf_counter()
    srv.close()  # waits for the (at most two) running requests, drops the rest
    assert time.perf_counter() - t0 < 30.0
