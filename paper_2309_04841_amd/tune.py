"""Autotuner for the batched evaluation: how many states advance together.

A group of `sets_per_pass` states goes through all layers before the next
group starts.  Small groups keep their states in the memory-side cache between
sweeps; large groups give each launch more workgroups.  The best value depends
on n, p, the dtype and the device, so it is measured: every candidate runs the
real batched call (same kernels, same results), the fastest is cached in a JSON
file (QAOA_TUNE_CACHE, default ~/.cache/paper_2309_04841_amd/tune.json).
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import _lib

_DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2309_04841_amd", "tune.json")


def cache_path() -> str:
    return os.environ.get("QAOA_TUNE_CACHE", _DEFAULT_CACHE)


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def key(n, p, batch, states, diag) -> str:
    dev = torch.cuda.get_device_properties(states.device).gcnArchName
    return f"{dev}|n={n}|p={p}|batch={batch}|{states.dtype}|{diag.dtype}"


def best_sets_per_pass(n, p, batch, diag, offset, states, out, gamma, beta, candidates=None, reps=2,
                       use_cache=True) -> int:
    """Fastest sets_per_pass for qaoa_evolve_batch on these buffers (states and
    out are overwritten while timing)."""
    k = key(n, p, batch, states, diag)
    cache = _load() if use_cache else {}
    if k in cache:
        return int(cache[k]["sets_per_pass"])
    if candidates is None:
        candidates = sorted({min(batch, 1 << i) for i in range(0, 16) if (1 << i) <= 2 * batch})
    work = torch.empty(_lib.batch_workspace_bytes(n, p, batch, _lib.state_dtype_code(states),
                                                  _lib.diag_dtype_code(diag)), dtype=torch.uint8,
                       device=states.device)
    timings = {}
    for spp in candidates:
        _lib.qaoa_evolve_batch(n, gamma, beta, diag, states, diag_offset=offset, out=out, sets_per_pass=spp,
                               work=work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _lib.qaoa_evolve_batch(n, gamma, beta, diag, states, diag_offset=offset, out=out, sets_per_pass=spp,
                                   work=work)
        torch.cuda.synchronize()
        timings[spp] = (time.perf_counter() - t0) / reps
    best = min(timings, key=timings.get)
    if use_cache:
        cache[k] = {"sets_per_pass": best, "seconds": timings}
        _store(cache)
    return best
