"""Batched evaluation (many (gamma, beta) sets against one cost vector).

* each state of a batch is bitwise equal to a single qaoa_evolve with its angles
  (same kernels, same reduction order), for every sets_per_pass grouping;
* batch results match the FP64 oracle (complex64 tolerance 1e-5, complex128 1e-10);
* the call captured in a HIP graph replays correctly after new angles are
  written into the same device buffers (every replay checked against eager
  results, with other eager GPU work between replays).
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
    from paper_2309_04841_amd import _lib
    return q, _lib


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


TD = {"complex64": torch.complex64, "complex128": torch.complex128}


def _single(q, n, g, b, diag, off, dtype):
    psi = torch.empty(1 << n, dtype=TD[dtype], device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    q.qaoa_evolve(n, g, b, diag, psi, init=True, diag_offset=off, out=out)
    return psi, out


@pytest.mark.parametrize("n,dtype,ddt,batch,p", [(10, "complex128", "i32", 7, 3), (10, "complex64", "u16", 5, 40),
                                                 (16, "complex128", "u16", 6, 3), (17, "complex64", "i32", 9, 2),
                                                 (15, "complex128", "f64", 4, 2)])
def test_batch_equals_singles_bitwise(q, n, dtype, ddt, batch, p):
    q, _lib = q
    _say(f"batch n={n} {dtype} {ddt} B={batch} p={p}")
    terms = W.labs_terms(n) if ddt != "f64" else [(0.37 * w, e) for w, e in W.labs_terms(n)]
    diag, off = q.qaoa_precompute_diag(n, terms, ddt, device="cuda")
    rng = np.random.default_rng(n + batch)
    gam = rng.uniform(0, 1, size=(batch, p))
    bet = rng.uniform(0, np.pi, size=(batch, p))
    dg = torch.from_numpy(gam).cuda()
    db = torch.from_numpy(bet).cuda()
    for spp in (0, 1, 3):
        states = torch.empty(batch, 1 << n, dtype=TD[dtype], device="cuda")
        out = torch.empty(batch, 2, dtype=torch.float64, device="cuda")
        _lib.qaoa_evolve_batch(n, dg, db, diag, states, init=True, diag_offset=off, out=out, sets_per_pass=spp)
        for s in range(batch):
            psi, o = _single(q, n, gam[s], bet[s], diag, off, dtype)
            assert torch.equal(states[s], psi), (spp, s)
            assert torch.equal(out[s], o), (spp, s)


def test_batch_complex64_precision_switch(q):
    """complex64 sets whose layers straddle the FP32 bound |tan beta| = 64 (and
    beta = pi/2 exactly), several sets per launch with different choices: each
    workgroup decides from its own set's parameter rows, so the batch equals the
    single calls bitwise, and both match the oracle."""
    q, _lib = q
    n, p = 18, 3
    diag, off = q.qaoa_precompute_diag(n, W.labs_terms(n), "u16", device="cuda")
    bet = np.array([[0.3, 0.5, 0.7], [np.pi / 2, 0.4, np.arctan(63.9)], [np.arctan(64.1), np.pi / 2 + 0.01, 0.2],
                    [np.arctan(63.9), -np.arctan(63.9), np.pi / 2 - 1e-3], [1.0, 1.2, 1.4]])
    gam = np.tile(np.array([0.11, 0.23, 0.31]), (bet.shape[0], 1))
    batch = bet.shape[0]
    c = oracle.diag_labs(n).astype(np.float64)
    for spp in (0, 2):
        states = torch.empty(batch, 1 << n, dtype=torch.complex64, device="cuda")
        out = torch.empty(batch, 2, dtype=torch.float64, device="cuda")
        _lib.qaoa_evolve_batch(n, torch.from_numpy(gam).cuda(), torch.from_numpy(bet).cuda(), diag, states,
                               init=True, diag_offset=off, out=out, sets_per_pass=spp)
        got = states.cpu().numpy().astype(np.complex128)
        o = out.cpu().numpy()
        for s in range(batch):
            psi, o1 = _single(q, n, gam[s], bet[s], diag, off, "complex64")
            assert torch.equal(states[s], psi) and torch.equal(out[s], o1), (spp, s)
            ref = oracle.evolve(n, c, gam[s], bet[s])
            E, nrm = oracle.expectation(n, ref, c)
            assert np.linalg.norm(got[s] - ref) <= 1e-5, (spp, s)
            assert abs(o[s, 0] - E) <= 1e-5 * max(1.0, abs(E)), (spp, s)
            assert abs(o[s, 1] - nrm) <= 1e-5, (spp, s)


@pytest.mark.parametrize("n,dtype", [(12, "complex128"), (18, "complex64"), (19, "complex128")])
def test_batch_matches_oracle(q, n, dtype):
    q, _lib = q
    edges, weights = W.erdos_renyi_graph(n, 0.3, seed=n)
    terms = W.maxcut_terms(edges, weights)
    diag, off = q.qaoa_precompute_diag(n, terms, "i32", device="cuda")
    gam, bet = W.uniform_angles(3, seed=n, batch=4)
    states = torch.empty(4, 1 << n, dtype=TD[dtype], device="cuda")
    out = torch.empty(4, 2, dtype=torch.float64, device="cuda")
    _lib.qaoa_evolve_batch(n, torch.from_numpy(gam).cuda(), torch.from_numpy(bet).cuda(), diag, states,
                           diag_offset=off, out=out)
    c = oracle.diag_maxcut(n, edges, weights)
    tol = 1e-10 if dtype == "complex128" else 1e-5
    got = states.cpu().numpy().astype(np.complex128)
    o = out.cpu().numpy()
    for s in range(4):
        ref = oracle.evolve(n, c, gam[s], bet[s])
        E, nrm = oracle.expectation(n, ref, c)
        assert np.linalg.norm(got[s] - ref) <= tol
        assert abs(o[s, 0] - E) <= tol * max(1.0, abs(E))
        assert abs(o[s, 1] - nrm) <= tol


@pytest.mark.parametrize("n,dtype", [(11, "complex128"), (16, "complex64")])
def test_batch_graph_replay(q, n, dtype):
    q, _lib = q
    batch, p = 6, 3
    diag, off = q.qaoa_precompute_diag(n, W.labs_terms(n), "u16", device="cuda")
    dg = torch.zeros(batch, p, dtype=torch.float64, device="cuda")
    db = torch.zeros(batch, p, dtype=torch.float64, device="cuda")
    states = torch.empty(batch, 1 << n, dtype=TD[dtype], device="cuda")
    out = torch.empty(batch, 2, dtype=torch.float64, device="cuda")
    work = torch.empty(_lib.batch_workspace_bytes(n, p, batch, _lib.state_dtype_code(states),
                                                  _lib.diag_dtype_code(diag)), dtype=torch.uint8, device="cuda")

    def call():
        _lib.qaoa_evolve_batch(n, dg, db, diag, states, init=True, diag_offset=off, out=out, work=work)

    call()  # warm (kernel loading happens outside capture)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    for rep in range(4):
        gam = rng.uniform(0, 1, size=(batch, p))
        bet = rng.uniform(0, np.pi, size=(batch, p))
        dg.copy_(torch.from_numpy(gam))
        db.copy_(torch.from_numpy(bet))
        graph.replay()
        torch.cuda.synchronize()
        got_states, got_out = states.clone(), out.clone()
        # unrelated eager GPU work between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        call()
        torch.cuda.synchronize()
        assert torch.equal(got_states, states), rep
        assert torch.equal(got_out, out), rep
        del junk


def test_c3_workload_batch(q):
    """Weighted MaxCut G(22, 0.3), p=6, 512 sets, complex64: batch vs singles
    (bitwise) on a sample of sets, and vs the oracle on two sets."""
    q, _lib = q
    cfg = W.C3()
    n, p = cfg["n"], cfg["p"]
    gam, bet = cfg["gamma"], cfg["beta"]
    batch = gam.shape[0]
    diag, off = q.qaoa_precompute_diag(n, cfg["terms"], "i32", device="cuda")
    states = torch.empty(batch, 1 << n, dtype=torch.complex64, device="cuda")
    out = torch.empty(batch, 2, dtype=torch.float64, device="cuda")
    _say("C3 batch")
    _lib.qaoa_evolve_batch(n, torch.from_numpy(gam).cuda(), torch.from_numpy(bet).cuda(), diag, states,
                           diag_offset=off, out=out, sets_per_pass=8)
    o = out.cpu().numpy()
    for s in (0, 1, 255, 511):
        psi, os_ = _single(q, n, gam[s], bet[s], diag, off, "complex64")
        assert torch.equal(states[s], psi) and torch.equal(out[s], os_), s
    assert np.all(np.abs(o[:, 1] - 1.0) < 1e-5)
    c = oracle.diag_maxcut(n, cfg["edges"], cfg["weights"])
    for s in (0, 300):
        ref = oracle.evolve(n, c, gam[s], bet[s])
        E, _ = oracle.expectation(n, ref, c)
        assert abs(o[s, 0] - E) <= 1e-5 * abs(E)
    del states
    torch.cuda.empty_cache()


def test_autotuned_settings_match_oracle(q, tmp_path, monkeypatch):
    """The tuner's joint choice of tile size, layer fusion and group size runs
    the same evaluation: every state matches the oracle under the chosen knobs,
    and the knobs are restored afterwards."""
    q, _lib = q
    from paper_2309_04841_amd import tune
    monkeypatch.setenv("QAOA_TUNE_CACHE", str(tmp_path / "tune.json"))
    n, batch = 16, 8
    diag, off = q.qaoa_precompute_diag(n, W.labs_terms(n), "u16", device="cuda")
    gam, bet = W.uniform_angles(3, seed=16, batch=batch)
    dg, db = torch.from_numpy(gam).cuda(), torch.from_numpy(bet).cuda()
    states = torch.empty(batch, 1 << n, dtype=torch.complex128, device="cuda")
    out = torch.empty(batch, 2, dtype=torch.float64, device="cuda")
    before = (_lib.get_tuning(_lib.TUNE_WIDE_TILES), _lib.get_tuning(_lib.TUNE_FUSE_LAYERS))
    best = tune.best_settings(n, 3, batch, diag, off, states, out, dg, db, reps=1)
    assert (_lib.get_tuning(_lib.TUNE_WIDE_TILES), _lib.get_tuning(_lib.TUNE_FUSE_LAYERS)) == before
    assert set(best) == {"wide_tiles", "fuse_layers", "sets_per_pass"} and 1 <= best["sets_per_pass"] <= batch
    assert tune.best_settings(n, 3, batch, diag, off, states, out, dg, db) == best  # cached
    with tune.settings(best):
        work = torch.empty(_lib.batch_workspace_bytes(n, 3, batch, _lib.QAOA_C128, _lib.QAOA_DIAG_U16),
                           dtype=torch.uint8, device="cuda")
        _lib.qaoa_evolve_batch(n, dg, db, diag, states, diag_offset=off, out=out,
                               sets_per_pass=best["sets_per_pass"], work=work)
        torch.cuda.synchronize()
    c = oracle.diag_labs(n).astype(np.float64)
    got = states.cpu().numpy()
    o = out.cpu().numpy()
    for s in range(batch):
        ref = oracle.evolve(n, c, gam[s], bet[s])
        E, _ = oracle.expectation(n, ref, c)
        assert np.linalg.norm(got[s] - ref) <= 1e-10
        assert abs(o[s, 0] - E) <= 1e-10 * max(1.0, abs(E))
