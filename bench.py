"""Throughput benchmark: QAOA expectation evaluations per second on one MI355X.

Workload (default): LABS n=26, p=10, complex128 state, uint16 cost vector,
linear-ramp schedule (seeded).  One "step" is one full evaluation of the hot
path: |+>^n generated in-kernel, p layers of phase + mixer sweeps, E fused into
the last sweep and reduced in FP64.  The cost vector is precomputed once before
the timed region (as in the paper, precompute is reported separately).

Prints ONE JSON line.  `roofline` describes the dominant kernel (the fused
sweep kernel): algorithmic bytes per launch / average launch duration, both per
launch of that kernel, timed with HIP events on the stream the kernels run on.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "QAOA expectation evals/s, LABS n=26 p=10; % HBM peak; served p50/p99"

CONFIGS = {
    # LABS energies are integers in [0, sum_k (n-k)^2] (12529 at n=34), so uint16 holds the cost
    # vector exactly (int32 and float64 are available through --diag)
    "labs26": dict(make="C2A", diag="u16"),
    "labs31": dict(make="C2B", diag="u16"),
    # the same LABS n=26 p=10 evaluation with the Hamming-weight-preserving XY
    # mixers (ring / complete graph on the qubits) in place of the X mixer
    "xy_ring26": dict(make="C2A", diag="u16", mixer="xy_ring"),
    "xy_complete26": dict(make="C2A", diag="u16", mixer="xy_complete"),
}


def _sweep_bytes(sched, n, state_bytes, diag_bytes):
    """Algorithmic HBM bytes of one evaluation, per sweep launch of its schedule.

    Every launch reads and writes the state once (S bytes each way per element),
    except the first, which generates |+> in registers and only writes.  A
    launch that applies a phase (the opening sweep, and each fused sweep that
    joins two layers) reads the cost vector (D bytes per element); so does the
    last launch, which reduces E.
    """
    from paper_2309_04841_amd import _lib
    N = 1 << n
    per_launch = []
    for _sw, _layer, flags in sched:
        b = (1 if flags & _lib.F_INIT else 2) * state_bytes * N
        if flags & (_lib.F_PHASE | _lib.F_FUSE | _lib.F_EXPV):
            b += diag_bytes * N
        per_launch.append(b)
    return per_launch


def _xy_sweep_bytes(n, p, nsweeps, state_bytes, diag_bytes):
    """Algorithmic HBM bytes per launch of an XY-mixer evaluation: p layers of
    `nsweeps` launches; the first generates |+> and only writes the state, every
    other reads and writes it; each layer's first launch applies the phase and
    reads the cost vector, and so does the last launch, which reduces E."""
    N = 1 << n
    per_launch = []
    for l in range(p):
        for sw in range(nsweeps):
            b = (1 if (l == 0 and sw == 0) else 2) * state_bytes * N
            if sw == 0 or (l == p - 1 and sw == nsweeps - 1):
                b += diag_bytes * N
            per_launch.append(b)
    return per_launch


KERNEL_SOURCES = ("tile.hpp", "kernels.hpp", "qaoa.hip")


def kernel_source_hash() -> str:
    """sha256 over the HIP sources that define the kernels and their launches,
    with comments and blank space removed (an edit to a comment leaves the
    measured kernels unchanged)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2309_04841_amd", "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per sweep launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
    (scaled by the copy-kernel calibration) and recorded in profiles/, or None
    when no record exists for this workload or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg, budget_s=12.0, mixer=None):
    """Time the FP64 oracle on whole QAOA layers of the same workload, repeating
    evaluations from |+> until about `budget_s` of work is done (at least one
    layer); scale to evaluations per second."""
    import numpy as np

    import oracle
    n, p = cfg["n"], cfg["p"]
    xy_kind = {None: None, "xy_ring": oracle.XY_RING, "xy_complete": oracle.XY_COMPLETE}[mixer]
    t0 = time.perf_counter()
    c = oracle.diag_labs(n)
    c = c.astype(np.float64)
    t_diag = time.perf_counter() - t0
    layers = 0
    if xy_kind is None:
        # Algorithm 3 one layer at a time on one state (no copies: at n=31 it holds 32 GiB)
        psi = np.empty(1 << n, dtype=np.complex128)
        t0 = time.perf_counter()
        while True:
            l = layers % p
            oracle.evolve_inplace(n, c, cfg["gamma"][l:l + 1], cfg["beta"][l:l + 1], psi, init=(l == 0))
            layers += 1
            if time.perf_counter() - t0 >= budget_s:
                break
    else:
        plus = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
        psi = plus
        t0 = time.perf_counter()
        while True:
            l = layers % p
            if l == 0:
                psi = plus.copy()
            psi = oracle.apply_phase(n, c, cfg["gamma"][l], psi)
            psi = oracle.apply_xy_mixer(n, xy_kind, cfg["beta"][l], psi)
            layers += 1
            if time.perf_counter() - t0 >= budget_s:
                break
    t_layers = time.perf_counter() - t0
    evals_per_s = layers / (t_layers * p)
    return dict(value=evals_per_s, unit="evals/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"{layers} layers ({layers / p:.1f} evaluations of {p} layers) of the same workload "
                       f"(n={n}, FP64 complex128 state, phase + "
                       f"{'%d single-qubit' % n if xy_kind is None else len(oracle.xy_edges(n, xy_kind))} "
                       f"{'mixer' if xy_kind is None else mixer + ' two-qubit'} passes per layer) in "
                       f"{t_layers:.2f} s, scaled to evaluations/s; cost vector built separately in "
                       f"{t_diag:.2f} s and excluded like the GPU precompute")


def _replay_ms(graph, steps, stream):
    """Average time of one replay of a captured graph, HIP events on `stream`."""
    import torch
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record(stream)
    for _ in range(steps):
        graph.replay()
    e.record(stream)
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def bench_batch(args):
    """Batched parameter sweep: weighted MaxCut G(22, 0.3), p=6, 512 (gamma, beta)
    sets, complex64.  The batched call and, for comparison, the loop of 512
    single qaoa_evolve calls are each captured once in a HIP graph and timed by
    replaying it (one submission per batch); eager timings are reported beside."""
    import numpy as np
    import torch

    import paper_2309_04841_amd as q
    from paper_2309_04841_amd import _lib, tune
    import workloads as W
    cfg = W.C3()
    n, p = cfg["n"], cfg["p"]
    gam, bet = cfg["gamma"], cfg["beta"]
    batch = gam.shape[0]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    diag, off = q.qaoa_precompute_diag(n, cfg["terms"], "i32", device=dev)
    dg, db = torch.from_numpy(gam).to(dev), torch.from_numpy(bet).to(dev)
    states = torch.empty(batch, 1 << n, dtype=torch.complex64, device=dev)
    out = torch.empty(batch, 2, dtype=torch.float64, device=dev)
    if args.sets_per_pass:
        best = {"wide_tiles": _lib.get_tuning(_lib.TUNE_WIDE_TILES),
                "fuse_layers": _lib.get_tuning(_lib.TUNE_FUSE_LAYERS), "sets_per_pass": args.sets_per_pass}
    else:
        best = tune.best_settings(n, p, batch, diag, off, states, out, dg, db)
    spp = best["sets_per_pass"]
    psi = torch.empty(1 << n, dtype=torch.complex64, device=dev)
    o1 = torch.empty(batch, 2, dtype=torch.float64, device=dev)
    w1 = _lib.alloc_workspace(_lib.QAOA_OP_EVOLVE, n, _lib.QAOA_C64, _lib.QAOA_DIAG_I32, dev)
    with tune.settings(best):
        work = torch.empty(_lib.batch_workspace_bytes(n, p, batch, _lib.QAOA_C64, _lib.QAOA_DIAG_I32),
                           dtype=torch.uint8, device=dev)

        def run_batch():
            _lib.qaoa_evolve_batch(n, dg, db, diag, states, diag_offset=off, out=out, sets_per_pass=spp, work=work)

        def run_singles():
            for s_ in range(batch):
                q.qaoa_evolve(n, gam[s_], bet[s_], diag, psi, diag_offset=off, out=o1[s_], work=w1)

        for _ in range(max(1, args.warmup)):
            run_batch()
        run_singles()
        torch.cuda.synchronize()
        ref_out = out.clone()
        # eager: one library call per batch / per set
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run_batch()
        torch.cuda.synchronize()
        t_batch_eager = (time.perf_counter() - t0) / args.steps
        t0 = time.perf_counter()
        run_singles()
        torch.cuda.synchronize()
        t_single_eager = time.perf_counter() - t0
        # captured: one graph replay per batch (kernels only, so the call is capturable)
        g_batch, g_single = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_batch):
            run_batch()
        with torch.cuda.graph(g_single):
            run_singles()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream(dev)
        ms_batch = _replay_ms(g_batch, args.steps, stream)
        ms_single = _replay_ms(g_single, max(1, args.steps // 4), stream)
        if not (torch.equal(out, ref_out) and torch.equal(o1, ref_out)):
            raise RuntimeError("graph replay, eager batch and single calls disagree")
        sched = _lib.schedule_describe(n, p, _lib.QAOA_C64)
    t_batch = ms_batch * 1e-3
    per_launch = _sweep_bytes(sched, n, 8, 4)  # one state, under the tuned schedule
    groups = -(-batch // spp)
    launches = len(per_launch) * groups  # each launch advances one group of spp states
    achieved = sum(per_launch) * batch / t_batch / 1e9
    return {"metric": "batched QAOA evals/s, weighted MaxCut G(22,0.3) p=6, 512 sets", "value": batch / t_batch,
            "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_batch, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": cfg["name"], "n": n, "p": p, "sets": batch, "state": "complex64",
                       "cost_vector": "int32", "sets_per_pass": spp, "fuse_layers": best["fuse_layers"],
                       "wide_tiles": best["wide_tiles"], "timing": "HIP graph replay"},
            "single_path_evals_per_s": batch / (ms_single * 1e-3), "speedup_vs_single": ms_single / ms_batch,
            "eager_batch_evals_per_s": batch / t_batch_eager, "eager_single_evals_per_s": batch / t_single_eager,
            "roofline": {"bound": "hbm", "kernel": "qaoa_sweep_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                         "traffic": measured_traffic(f"{cfg['name']}_spp{spp}"),
                         "bytes_per_launch": sum(per_launch) * batch / launches, "launches_per_step": launches,
                         "avg_launch_ms": ms_batch / launches}}


def _adjoint_bytes(sched, n, state_bytes, diag_bytes):
    """Algorithmic HBM bytes per reverse-pass launch of the gradient: every
    launch reads and writes psi and lambda, except the first, which reads psi
    and the cost vector and writes both (lambda = c psi); launches that undo a
    phase (A_PHASE, or A_FUSE joining two layers) read the cost vector."""
    from paper_2309_04841_amd import _lib
    N = 1 << n
    out = []
    for _sw, _layer, flags in sched:
        if flags & _lib.A_FIRST:
            b = 3 * state_bytes * N + diag_bytes * N
        else:
            b = 4 * state_bytes * N
            if flags & (_lib.A_PHASE | _lib.A_FUSE):
                b += diag_bytes * N
        out.append(b)
    return out


def bench_grad(args):
    """Adjoint gradient (E, dE/dgamma, dE/dbeta): LABS n=24, p=20, complex128,
    uint16 cost vector.  One step = one qaoa_grad call (forward evaluation +
    reverse pass); the reverse pass's time is the gradient's time minus that of
    the same forward evaluation timed alone."""
    import numpy as np
    import torch

    import paper_2309_04841_amd as q
    from paper_2309_04841_amd import _lib
    import workloads as W
    cfg = W.C4()
    n, p = cfg["n"], cfg["p"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    gamma, beta = np.asarray(cfg["gamma"]), np.asarray(cfg["beta"])
    diag, off = q.qaoa_precompute_diag(n, cfg["terms"], "u16", device=dev)
    psi = torch.empty(1 << n, dtype=torch.complex128, device=dev)
    adj = torch.empty_like(psi)
    out = torch.empty(1 + 2 * p, dtype=torch.float64, device=dev)
    eo = torch.empty(2, dtype=torch.float64, device=dev)
    gw = torch.empty(_lib.grad_workspace_bytes(n, p, _lib.QAOA_C128, _lib.QAOA_DIAG_U16), dtype=torch.uint8, device=dev)
    ew = _lib.alloc_workspace(_lib.QAOA_OP_EVOLVE, n, _lib.QAOA_C128, _lib.QAOA_DIAG_U16, dev)
    stream = torch.cuda.current_stream(dev)

    def grad():
        q.qaoa_grad(n, gamma, beta, diag, psi, adj, diag_offset=off, out=out, work=gw)

    def fwd():
        q.qaoa_evolve(n, gamma, beta, diag, psi, init=True, diag_offset=off, out=eo, work=ew)

    def timed(fn, k):
        for _ in range(max(1, args.warmup)):
            fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record(stream)
        for _ in range(k):
            fn()
        e.record(stream)
        torch.cuda.synchronize()
        return s.elapsed_time(e) / k

    ms_grad = timed(grad, args.steps)
    g_first = out.cpu().numpy().copy()
    ms_fwd = timed(fwd, args.steps)
    grad()
    torch.cuda.synchronize()
    if not np.array_equal(g_first, out.cpu().numpy()) or not np.isfinite(g_first).all():
        raise RuntimeError("non-reproducible or non-finite gradient")
    sched = _lib.schedule_describe(n, p, _lib.QAOA_C128, kind=_lib.SCHED_ADJOINT)
    per = _adjoint_bytes(sched, n, 16, 2)
    ms_rev = ms_grad - ms_fwd
    achieved = (sum(per) / len(per)) / (ms_rev / len(per) * 1e-3) / 1e9
    res = {
        "metric": f"QAOA gradient evals/s (adjoint), LABS n={n} p={p}",
        "value": 1e3 / ms_grad, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps,
        "warmup": max(1, args.warmup), "ms_per_step": ms_grad, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "problem": "LABS", "n": n, "p": p, "state": "complex128",
                   "cost_vector": "uint16", "schedule": "linear ramp + N(0, 0.05), seeded",
                   "forward_ms": ms_fwd, "reverse_ms": ms_rev, "reverse_launches": len(per),
                   "E": float(g_first[0])},
        "roofline": {"bound": "hbm", "kernel": "qaoa_adjoint_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(cfg["name"]),
                     "bytes_per_launch": sum(per) / len(per), "launches_per_step": len(per),
                     "avg_launch_ms": ms_rev / len(per)},
    }
    if not args.no_cpu_baseline:
        import oracle
        c = oracle.diag_labs(n).astype(np.float64)
        t0 = time.perf_counter()
        oracle.grad(n, c, gamma, beta)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = dict(value=1.0 / dt, unit="gradients/s", cores=oracle.num_threads(), kind="oracle",
                                   sample=f"one full gradient of the same workload (forward + adjoint, FP64) in "
                                          f"{dt:.2f} s")
    return res


SERVE_MIXES = {
    # the configured serving workload: n ~ U{16..30}, p ~ U{1..20}
    "mix": dict(ns=range(16, 31), pmax=20, count=96),
    # requests small enough that one does not fill the GPU (n ~ U{16..22}):
    # the case where overlapping admitted requests pays
    "small": dict(ns=range(16, 23), pmax=20, count=600),
}


def _serve_workload(name, seed):
    """Problems and requests of a serving mix: 60 % objective / 40 % gradient,
    LABS or regular MaxCut (3-regular for even n, 4-regular for odd n)."""
    import numpy as np

    import workloads as W
    spec = SERVE_MIXES[name]
    rng = np.random.default_rng(seed)
    probs = {}
    for n in spec["ns"]:
        probs[("labs", n)] = (n, W.labs_terms(n))
        d = 3 if n % 2 == 0 else 4  # d n must be even
        probs[("maxcut", n)] = (n, W.maxcut_terms(W.random_regular_graph(d, n, seed=100 + n)))
    keys = list(probs)
    reqs = []
    for _ in range(spec["count"]):
        k = keys[int(rng.integers(0, len(keys)))]
        p = int(rng.integers(1, spec["pmax"] + 1))
        reqs.append((k, rng.uniform(0, 1, size=p), rng.uniform(0, np.pi, size=p), bool(rng.random() < 0.4)))
    return probs, reqs


def _serve_run(probs, reqs, arrivals=None, streams=4, max_in_flight=16, arena_bytes=160 << 30):
    """Run the requests through a fresh server; `arrivals` (seconds from the
    start) paces the submissions, None submits them all at once.  Returns the
    server's stats, the wall time from the first submission to the last result,
    and the results in request order."""
    import threading

    import paper_2309_04841_amd as q
    srv = q.QAOAServer(arena_bytes=arena_bytes, num_streams=streams, max_in_flight=max_in_flight)
    try:
        pids = {k: srv.add_problem(n, terms) for k, (n, terms) in probs.items()}
        tickets = []

        def submitter():
            t0 = time.perf_counter()
            for i, (k, g, b, grad) in enumerate(reqs):
                if arrivals is not None:
                    dt = arrivals[i] - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                tickets.append(srv.submit(pids[k], g, b, gradient=grad))

        t0 = time.perf_counter()
        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        results = [srv.wait(t)[0] for t in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
    finally:
        srv.close()
    return st, wall, results


def serve_summary(name, seed=7, load=0.6):
    """Capacity (all requests submitted at once, four streams, 16 in flight),
    one-at-a-time rate (one stream, one in flight), and latency under Poisson
    arrivals at `load` times the capacity, where the queue stays bounded."""
    import numpy as np
    probs, reqs = _serve_workload(name, seed)
    _serve_run(probs, reqs[:8])  # warm the kernels and the allocator
    st_cap, wall_cap, _ = _serve_run(probs, reqs)
    capacity = len(reqs) / wall_cap
    _, wall_seq, _ = _serve_run(probs, reqs, streams=1, max_in_flight=1)
    sequential = len(reqs) / wall_seq
    rate = load * capacity
    arrivals = np.cumsum(np.random.default_rng(seed + 1).exponential(1.0 / rate, size=len(reqs)))
    st, wall, _ = _serve_run(probs, reqs, arrivals=arrivals)
    spec = SERVE_MIXES[name]
    return {"requests": len(reqs), "n_range": [min(spec["ns"]), max(spec["ns"])], "p_range": [1, spec["pmax"]],
            "capacity_requests_per_s": capacity, "sequential_requests_per_s": sequential,
            "overlap_gain": capacity / sequential, "offered_requests_per_s": rate,
            "served_requests_per_s": len(reqs) / wall, "p50_ms": 1e3 * st["p50_s"], "p99_ms": 1e3 * st["p99_s"],
            "mean_ms": 1e3 * st["mean_s"], "max_ms": 1e3 * st["max_s"],
            "peak_arena_GB": max(st["peak_bytes"], st_cap["peak_bytes"]) / 1e9}


def bench_serve(args):
    """Served mixes (60 % objective / 40 % gradient, LABS or regular MaxCut,
    complex64): capacity, one-at-a-time rate, and p50/p99 latency of Poisson
    arrivals at 0.6 of capacity; n ~ U{16..30} and the small-request mix
    n ~ U{16..22}."""
    mixes = {name: serve_summary(name) for name in SERVE_MIXES}
    main_mix = mixes["mix"]
    return {"metric": "served QAOA requests/s (60% objective / 40% gradient, n 16..30, p 1..20)",
            "value": main_mix["capacity_requests_per_s"], "unit": "requests/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "serve_mix", "state": "complex64", "streams": 4, "max_in_flight": 16,
                       "arithmetic": "forward sweeps FP32, gradient sweeps FP64"},
            "p50_ms": main_mix["p50_ms"], "p99_ms": main_mix["p99_ms"], "mixes": mixes}


MALL_BYTES = 256 << 20  # memory-side (Infinity) cache of one MI355X


def bench_layer_curve(args):
    """Time per QAOA layer against n (LABS, uint16 cost vector, linear ramp),
    complex128 n = 18..32 and complex64 n = 18..33: per-layer time
    (T(p=10) - T(p=2)) / 8 removes the fixed first and last launches and the
    parameter preparation; its algorithmic bytes come from the same schedules.
    Flags the sizes whose state and cost vector fit the 256 MB memory-side
    cache (bandwidth there can exceed HBM's)."""
    import numpy as np
    import torch

    import paper_2309_04841_amd as q
    from paper_2309_04841_amd import _lib
    import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    rows = []
    for dtype, sdt, S, ns in (("complex128", torch.complex128, 16, range(18, 33)),
                              ("complex64", torch.complex64, 8, range(18, 34))):
        for n in ns:
            gamma, beta = W.linear_ramp(10, seed=n)
            diag, off = q.qaoa_precompute_diag(n, W.labs_terms(n), "u16", device=dev)
            psi = torch.empty(1 << n, dtype=sdt, device=dev)
            out = torch.empty(2, dtype=torch.float64, device=dev)
            work = _lib.alloc_workspace(_lib.QAOA_OP_EVOLVE, n, _lib.state_dtype_code(psi), _lib.QAOA_DIAG_U16, dev)
            reps = 3 if n >= 30 else 10
            t = {}
            for p in (2, 10):
                g, b = gamma[:p], beta[:p]
                q.qaoa_evolve(n, g, b, diag, psi, diag_offset=off, out=out, work=work)
                s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                s0.record(stream)
                for _ in range(reps):
                    q.qaoa_evolve(n, g, b, diag, psi, diag_offset=off, out=out, work=work)
                s1.record(stream)
                torch.cuda.synchronize()
                t[p] = s0.elapsed_time(s1) / reps
            code = _lib.state_dtype_code(psi)
            plan = _lib.plan_describe(n, code)
            if plan["single"]:
                b_layer = None
            else:
                b2 = sum(_sweep_bytes(_lib.schedule_describe(n, 2, code), n, S, 2))
                b10 = sum(_sweep_bytes(_lib.schedule_describe(n, 10, code), n, S, 2))
                b_layer = (b10 - b2) / 8
            ms_layer = (t[10] - t[2]) / 8
            gbs = b_layer / (ms_layer * 1e-3) / 1e9 if b_layer else None
            rows.append({"state": dtype, "n": n, "sweeps_per_layer": len(plan["sweeps"]), "wide": plan["wide"],
                         "ms_per_layer": ms_layer, "ms_eval_p10": t[10], "bytes_per_layer": b_layer,
                         "GBps": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS if gbs else None,
                         "mall_resident": (1 << n) * (S + 2) <= MALL_BYTES})
            print(f"layer_curve {dtype} n={n} {ms_layer:.4f} ms/layer", file=sys.stderr, flush=True)
            del psi, diag, work
            torch.cuda.empty_cache()
    return {"metric": "time per QAOA layer vs n, LABS, uint16 cost vector", "unit": "ms/layer",
            "higher_is_better": False, "n_gpus": 1, "data": "synthetic", "rows": rows}


def _progress(msg):
    """One line per finished part of the run, on stderr (stdout holds the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", choices=sorted(CONFIGS) + ["batch", "serve", "grad", "layer_curve"],
                    default="labs26")
    ap.add_argument("--sets-per-pass", type=int, default=0, help="batch: states advanced together (0 = autotune)")
    ap.add_argument("--wide-tiles", type=int, choices=(0, 1), default=1,
                    help="complex128: 2^14-element tiles when they save a sweep (library tuning knob)")
    ap.add_argument("--fuse-layers", type=int, choices=(0, 1), default=1,
                    help="join adjacent layers in one sweep launch (library tuning knob)")
    ap.add_argument("--diag", choices=("u16", "i32", "f64"), default=None,
                    help="cost-vector storage (default: the configuration's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="labs26: skip the nested complex64 n=31 evaluation and the served mixes")
    ap.add_argument("--c2b-steps", type=int, default=10, help="labs26: timed evaluations of the nested n=31 run")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (torch), the reference for HBM counter scaling")
    args = ap.parse_args(argv)

    if args.copy_calibration:
        import torch
        nbytes = 1 << 30
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes, "dispatches": 3}}))
        return 0

    if args.config in ("batch", "serve", "grad", "layer_curve") and args.gpus == 1:
        import torch  # noqa: F401
        res = {"batch": bench_batch, "serve": bench_serve, "grad": bench_grad,
               "layer_curve": bench_layer_curve}[args.config](args)
        print(json.dumps(res), flush=True)
        return 0

    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (--gpus {args.gpus} requested); the hot path is "
              "single-device and no multi-GPU path exists", file=sys.stderr)
        return 2

    from paper_2309_04841_amd import _lib
    _lib.set_tuning(_lib.TUNE_WIDE_TILES, args.wide_tiles)
    _lib.set_tuning(_lib.TUNE_FUSE_LAYERS, args.fuse_layers)
    res = measure_eval(args.config, args.diag, args.steps, args.warmup,
                       None if args.no_cpu_baseline else args.cpu_budget)
    if res is None:
        return 1
    _progress(f"{args.config}: {res['value']:.2f} {res['unit']}")
    if args.config == "labs26" and not args.headline_only:
        # the rest of the metric: the complex64 n=31 evaluation and the served mix
        c2b = measure_eval("labs31", None, args.c2b_steps, 2, None if args.no_cpu_baseline else args.cpu_budget)
        if c2b is None:
            return 1
        _progress(f"labs31: {c2b['value']:.3f} {c2b['unit']}")
        res["c2b"] = {k: c2b[k] for k in ("metric", "value", "unit", "ms_per_step", "dtype", "config", "roofline")
                      if k in c2b}
        if "cpu_baseline" in c2b:
            res["c2b"]["cpu_baseline"] = c2b["cpu_baseline"]
        res["serve"] = {}
        for name in SERVE_MIXES:
            res["serve"][name] = serve_summary(name)
            _progress(f"serve {name}: {res['serve'][name]['capacity_requests_per_s']:.1f} requests/s capacity")
    print(json.dumps(res), flush=True)
    return 0


def measure_eval(config, diag_name, steps, warmup, cpu_budget):
    """One workload of CONFIGS: precompute (timed apart), `warmup` evaluations,
    then `steps` evaluations timed with HIP events on the stream they run on.
    Returns the result dict (roofline and, unless cpu_budget is None, the
    oracle's sampled rate), or None if the objective is not reproducible."""
    import numpy as np
    import torch

    import paper_2309_04841_amd as q
    from paper_2309_04841_amd import _lib
    import workloads as W

    spec = dict(CONFIGS[config])
    if diag_name:
        spec["diag"] = diag_name
    cfg = getattr(W, spec["make"])()
    n, p = cfg["n"], cfg["p"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sdt = torch.complex128 if cfg["dtype"] == "complex128" else torch.complex64
    S = 16 if sdt == torch.complex128 else 8
    D = {"i32": 4, "u16": 2, "f64": 8}[spec["diag"]]
    gamma, beta = np.asarray(cfg["gamma"]), np.asarray(cfg["beta"])

    stream = torch.cuda.current_stream(dev)
    # precompute (timed separately, excluded from the metric)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    q.qaoa_precompute_diag(n, cfg["terms"], spec["diag"], device=dev)  # warm
    torch.cuda.synchronize()
    ev0.record(stream)
    diag, off = q.qaoa_precompute_diag(n, cfg["terms"], spec["diag"], device=dev)
    ev1.record(stream)
    torch.cuda.synchronize()
    precompute_ms = ev0.elapsed_time(ev1)

    psi = torch.empty(1 << n, dtype=sdt, device=dev)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    work = _lib.alloc_workspace(_lib.QAOA_OP_EVOLVE, n, _lib.state_dtype_code(psi), _lib.diag_dtype_code(diag), dev)

    mixer = spec.get("mixer")
    if mixer:
        mcode = _lib.MIXER_NAMES[mixer]
        work = torch.empty(max(16, _lib.xy_workspace_bytes(n, mcode, _lib.state_dtype_code(psi))),
                           dtype=torch.uint8, device=dev)

        def step():
            q.qaoa_evolve_xy(n, gamma, beta, diag, psi, mixer=mcode, init=_lib.INIT_PLUS, diag_offset=off, out=out,
                             work=work)
    else:
        def step():
            q.qaoa_evolve(n, gamma, beta, diag, psi, init=True, diag_offset=off, out=out, work=work)

    for _ in range(max(1, warmup)):  # at least one evaluation, the reference for reproducibility
        step()
    torch.cuda.synchronize()
    e_first = out.cpu().numpy().copy()

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        step()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(end)
    ms_per_step = ms_total / steps
    e_last = out.cpu().numpy()
    if not (np.isfinite(e_last).all() and np.array_equal(e_first, e_last)):
        print(f"bench.py: non-reproducible or non-finite objective {e_first} vs {e_last}", file=sys.stderr)
        return None

    if mixer:
        plan = _lib.xy_plan_describe(n, mcode, _lib.state_dtype_code(psi))
        per_launch = _xy_sweep_bytes(n, p, len(plan["sweeps"]), S, D)
        kernel = "qaoa_xy_kernel"
    else:
        plan = _lib.plan_describe(n, _lib.state_dtype_code(psi))
        sched = _lib.schedule_describe(n, p, _lib.state_dtype_code(psi))
        per_launch = _sweep_bytes(sched, n, S, D)
        kernel = "qaoa_sweep_kernel"
    launches = len(per_launch)
    bytes_per_eval = float(sum(per_launch))
    # the timed region holds `launches` sweep launches and one tiny finalize
    # kernel per evaluation; charging the whole time to the sweeps is conservative
    avg_launch_ms = ms_per_step / launches
    achieved = (bytes_per_eval / launches) / (avg_launch_ms * 1e-3) / 1e9

    res = {
        "metric": METRIC if config == "labs26" else
        f"QAOA expectation evals/s, LABS n={n} p={p}" + (f", {mixer} mixer" if mixer else ""),
        "value": steps / (ms_total * 1e-3),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(1, warmup),
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # complex64 transverse-field sweeps compute in FP32 (FP64 for layers
        # with |tan beta| > 64, none in these ramps); the rest in FP64
        "dtype": "f32" if (cfg["dtype"] == "complex64" and not mixer) else "f64",
        "data": "synthetic",
        "config": {
            "workload": cfg["name"] + (f"+{mixer}" if mixer else ""), "problem": "LABS", "n": n, "p": p,
            "state": cfg["dtype"], "mixer": mixer or "x",
            "cost_vector": {"i32": "int32", "u16": "uint16", "f64": "float64"}[spec["diag"]],
            "schedule": "linear ramp, seeded", "sweeps_per_layer": len(plan["sweeps"]),
            "tile_bits": plan["sweeps"][0]["tb"], "wide_tiles": _lib.get_tuning(_lib.TUNE_WIDE_TILES),
            "fuse_layers": _lib.get_tuning(_lib.TUNE_FUSE_LAYERS), "launches_per_eval": launches,
            "precompute_ms": precompute_ms, "E": float(e_last[0]), "norm": float(e_last[1]),
            "wall_s_timed": wall,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(cfg["name"] + (f"_{mixer}" if mixer else "")),
            "bytes_per_launch": bytes_per_eval / launches,
            "launches_per_step": launches,
            "avg_launch_ms": avg_launch_ms,
        },
    }
    del psi, diag, work
    torch.cuda.empty_cache()
    if cpu_budget is not None:
        res["cpu_baseline"] = cpu_baseline(cfg, cpu_budget, mixer)
    return res


if __name__ == "__main__":
    sys.exit(main())
