"""Autotuner for the batched evaluation: how many states advance together,
and which sweep plan and launch schedule they use.

A group of `sets_per_pass` states goes through all layers before the next
group starts.  Small groups keep their states in the memory-side cache between
sweeps; large groups give each launch more workgroups.  The library's tuning
knobs choose the tile size (2^14-element complex128 tiles or not) and whether
adjacent layers share a sweep.  The best choice depends on n, p, the dtype and
the device, so it is measured: every candidate runs the real batched call (the
same result up to rounding order), the fastest is cached in a JSON file
(QAOA_TUNE_CACHE, default ~/.cache/paper_2309_04841_amd/tune.json).
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


def _time_batch(n, p, batch, diag, offset, states, out, gamma, beta, spp, reps):
    work = torch.empty(max(16, _lib.batch_workspace_bytes(n, p, batch, _lib.state_dtype_code(states),
                                                          _lib.diag_dtype_code(diag))),
                       dtype=torch.uint8, device=states.device)
    _lib.qaoa_evolve_batch(n, gamma, beta, diag, states, diag_offset=offset, out=out, sets_per_pass=spp, work=work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _lib.qaoa_evolve_batch(n, gamma, beta, diag, states, diag_offset=offset, out=out, sets_per_pass=spp,
                               work=work)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def best_settings(n, p, batch, diag, offset, states, out, gamma, beta, reps=2, use_cache=True) -> dict:
    """Fastest (wide_tiles, fuse_layers, sets_per_pass) for qaoa_evolve_batch on
    these buffers: every knob setting with group sizes 1, 4, 16, 64, ... up to
    the batch.  Apply the result with `settings(result)`.  The knobs are
    process-wide; the previous values are restored before returning."""
    k = "settings|" + key(n, p, batch, states, diag)
    cache = _load() if use_cache else {}
    if k in cache:
        return dict(cache[k]["best"])
    spps = sorted({min(batch, 4 ** i) for i in range(0, 10) if 4 ** i <= 4 * batch})
    wides = (0, 1) if states.dtype == torch.complex128 else (_lib.get_tuning(_lib.TUNE_WIDE_TILES),)
    timings = {}
    for wide in wides:
        for fuse in (0, 1):
            with _lib.tuning(wide_tiles=wide, fuse_layers=fuse):
                for spp in spps:
                    timings[(wide, fuse, spp)] = _time_batch(n, p, batch, diag, offset, states, out, gamma, beta,
                                                             spp, reps)
    wide, fuse, spp = min(timings, key=timings.get)
    best = {"wide_tiles": wide, "fuse_layers": fuse, "sets_per_pass": spp}
    if use_cache:
        cache[k] = {"best": best, "seconds": {f"{w},{f},{g}": t for (w, f, g), t in timings.items()}}
        _store(cache)
    return best


def settings(best: dict):
    """Context manager that applies the knobs of a best_settings result."""
    return _lib.tuning(wide_tiles=best["wide_tiles"], fuse_layers=best["fuse_layers"])
