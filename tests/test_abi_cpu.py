"""CPU checks of the C ABI: exports, argument validation, and the sweep plans.

No compute calls are made here.  The plan checks emulate, on the CPU, the index
arithmetic every sweep kernel uses (tile element -> global element, register
window mapping, LDS swizzle), so a plan that would read or write out of bounds,
touch an element twice, or skip or repeat a qubit fails here before any GPU run.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2309_04841_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qaoa.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qaoa_\w+)\s*\(", src)))


def test_header_symbols_exported():
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    raw = ctypes.CDLL(_lib.LIB_PATH)
    for name in names:
        assert hasattr(raw, name), name


def test_version_and_last_error():
    assert re.match(r"\d+\.\d+\.\d+", _lib.version())
    size = ctypes.c_size_t(0)
    assert _lib.lib.qaoa_workspace_bytes(_lib.QAOA_OP_EVOLVE, 0, 1, 1, ctypes.byref(size)) == _lib.QAOA_ERR_INVALID
    assert b"out of range" in _lib.lib.qaoa_last_error()


def test_workspace_bytes():
    # per-block (E, norm) partials of the last sweep + parameter rows (4 doubles, 256-byte aligned) and
    # phase tables (3 x 256 + 4 x 16 entries) of 33 layers (a chunk of 32 and the next one) + the
    # first stage of the two-stage reduction.  The partials cover the most workgroups of either plan
    # (2^12-element tiles: 2^14 workgroups at n=26), so the size does not depend on the tuning knobs.
    want = 16 * (1 << 14) + 1280 + 33 * 832 * 16 + 16 * 1024
    grad_sizes = set()
    for wide in (0, 1):
        for fuse in (0, 1):
            with _lib.tuning(wide_tiles=wide, fuse_layers=fuse):
                assert _lib.workspace_bytes(_lib.QAOA_OP_EVOLVE, 26, _lib.QAOA_C128) == want
                grad_sizes.add(_lib.grad_workspace_bytes(24, 20, _lib.QAOA_C128, _lib.QAOA_DIAG_I32))
    assert len(grad_sizes) == 1
    assert _lib.workspace_bytes(_lib.QAOA_OP_PRECOMPUTE, 20, diag_dtype=_lib.QAOA_DIAG_F64) == 0
    assert _lib.workspace_bytes(_lib.QAOA_OP_PRECOMPUTE, 20, diag_dtype=_lib.QAOA_DIAG_U16) >= 4 << 20
    with pytest.raises(_lib.QaoaError):
        _lib.workspace_bytes(9, 10)


# ---------------------------------------------------------------------------
# validation: every case fails before anything is enqueued
# ---------------------------------------------------------------------------
FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: each call fails validation first


def _evolve(n=10, p=1, gamma=(0.1,), beta=(0.2,), diag=FAKE, ddt=1, off=0.0, dbytes=None,
            state=FAKE, sdt=1, sbytes=None, init=1, out=None, work=None, wbytes=0):
    N = 1 << max(n, 0) if 0 <= n < 40 else 0
    dbytes = 4 * N if dbytes is None else dbytes
    sbytes = 16 * N if sbytes is None else sbytes
    g = (ctypes.c_double * max(1, len(gamma)))(*gamma) if gamma is not None else None
    b = (ctypes.c_double * max(1, len(beta)))(*beta) if beta is not None else None
    return _lib.lib.qaoa_evolve(n, p, g, b, diag, ddt, off, dbytes, state, sdt, sbytes, init, out, work, wbytes, None)


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), _lib.QAOA_ERR_INVALID),
    (dict(n=35), _lib.QAOA_ERR_INVALID),
    (dict(p=-1), _lib.QAOA_ERR_INVALID),
    (dict(sdt=7), _lib.QAOA_ERR_INVALID),
    (dict(ddt=7), _lib.QAOA_ERR_INVALID),
    (dict(state=None), _lib.QAOA_ERR_INVALID),
    (dict(diag=None), _lib.QAOA_ERR_INVALID),
    (dict(gamma=None), _lib.QAOA_ERR_INVALID),
    (dict(gamma=(float("nan"),)), _lib.QAOA_ERR_INVALID),
    (dict(beta=(float("inf"),)), _lib.QAOA_ERR_INVALID),
    (dict(off=0.5), _lib.QAOA_ERR_INVALID),
    (dict(init=2), _lib.QAOA_ERR_INVALID),
    (dict(sbytes=100), _lib.QAOA_ERR_NOMEM),
    (dict(dbytes=100), _lib.QAOA_ERR_NOMEM),
    (dict(out=FAKE), _lib.QAOA_ERR_NOMEM),
    (dict(out=FAKE, work=FAKE, wbytes=8), _lib.QAOA_ERR_NOMEM),
])
def test_evolve_rejects(kw, code):
    assert _evolve(**kw) == code
    assert _lib.lib.qaoa_last_error() != b""


def _evolve_noalloc(n=10, p=1, sdt=1, out=FAKE, init=1, off=0.0):
    N = 1 << n
    g = (ctypes.c_double * max(1, p))(*([0.1] * max(1, p)))
    return _lib.lib.qaoa_evolve_noalloc(n, p, g, g, FAKE, 1, off, 4 * N, FAKE, sdt, (16 if sdt else 8) * N, init,
                                        out, None)


def test_evolve_noalloc_limits():
    """The static scratch covers complex64 up to n=32 and complex128 up to n=31;
    beyond that (and for invalid arguments) the call fails before touching the GPU."""
    for sdt, nmax in ((_lib.QAOA_C64, 32), (_lib.QAOA_C128, 31)):
        assert _lib.workspace_bytes(_lib.QAOA_OP_EVOLVE, nmax, sdt) <= _lib.QAOA_NOALLOC_SCRATCH_BYTES
        assert _lib.workspace_bytes(_lib.QAOA_OP_EVOLVE, nmax + 1, sdt) > _lib.QAOA_NOALLOC_SCRATCH_BYTES
        assert _evolve_noalloc(n=nmax + 1, sdt=sdt) == _lib.QAOA_ERR_NOMEM
        assert b"static" in _lib.lib.qaoa_last_error()
    assert _evolve_noalloc(init=3) == _lib.QAOA_ERR_INVALID
    assert _evolve_noalloc(off=0.5) == _lib.QAOA_ERR_INVALID
    assert _evolve_noalloc(p=-1) == _lib.QAOA_ERR_INVALID


def _precompute(n=6, w=(1.0,), ptr=(0, 2), idx=(0, 1), ddt=1, diag=FAKE, dbytes=None, work=None, wbytes=0,
                offset=True):
    N = 1 << n if 0 < n < 40 else 0
    dbytes = 8 * N if dbytes is None else dbytes
    wa = (ctypes.c_double * max(1, len(w)))(*w)
    pa = (ctypes.c_int64 * len(ptr))(*ptr)
    ia = (ctypes.c_int32 * max(1, len(idx)))(*idx) if idx is not None else None
    off = ctypes.c_double(0) if offset else None
    return _lib.lib.qaoa_precompute_diag(n, len(w), wa, pa, ia, ddt, diag, dbytes,
                                         ctypes.byref(off) if offset else None, work, wbytes, None)


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), _lib.QAOA_ERR_INVALID),
    (dict(idx=(0, 6)), _lib.QAOA_ERR_INVALID),
    (dict(idx=(-1, 2)), _lib.QAOA_ERR_INVALID),
    (dict(ptr=(1, 2)), _lib.QAOA_ERR_INVALID),
    (dict(w=(1.0, 2.0), ptr=(0, 2, 1)), _lib.QAOA_ERR_INVALID),
    (dict(w=(float("nan"),)), _lib.QAOA_ERR_INVALID),
    (dict(ddt=9), _lib.QAOA_ERR_INVALID),
    (dict(diag=None), _lib.QAOA_ERR_INVALID),
    (dict(offset=False), _lib.QAOA_ERR_INVALID),
    (dict(dbytes=10), _lib.QAOA_ERR_NOMEM),
    (dict(w=(0.3,)), _lib.QAOA_ERR_RANGE),                  # not dyadic: not an integer vector
    (dict(w=(2.0 ** 31,)), _lib.QAOA_ERR_RANGE),            # beyond int32
    (dict(w=(1.0,), ddt=2, wbytes=0, idx=(0, 1)), None),   # placeholder, replaced below
])
def test_precompute_rejects(kw, code):
    if code is None:
        # U16 needing the int32 scratch (half-integer weight) without a workspace
        assert _precompute(w=(0.5,), ddt=2) == _lib.QAOA_ERR_NOMEM
        return
    assert _precompute(**kw) == code


def test_grad_validates():
    N = 1 << 8
    g = (ctypes.c_double * 1)(0.1)
    # no adjoint buffer, aliasing buffers, p = 0, missing workspace
    assert _lib.lib.qaoa_grad(8, 1, g, g, FAKE, 1, 0.0, 4 * N, FAKE, None, 1, 16 * N, FAKE, None, 0, None) \
        == _lib.QAOA_ERR_INVALID
    assert _lib.lib.qaoa_grad(8, 1, g, g, FAKE, 1, 0.0, 4 * N, FAKE, FAKE, 1, 16 * N, FAKE, None, 0, None) \
        == _lib.QAOA_ERR_INVALID
    other = ctypes.c_void_p(0x2000)
    assert _lib.lib.qaoa_grad(8, 0, g, g, FAKE, 1, 0.0, 4 * N, FAKE, other, 1, 16 * N, FAKE, None, 0, None) \
        == _lib.QAOA_ERR_INVALID
    assert _lib.lib.qaoa_grad(8, 1, g, g, FAKE, 1, 0.0, 4 * N, FAKE, other, 1, 16 * N, FAKE, None, 0, None) \
        == _lib.QAOA_ERR_NOMEM


# ---------------------------------------------------------------------------
# sweep plans: emulate the kernels' index arithmetic
# ---------------------------------------------------------------------------
def tmap(tid, k, w, eb):
    return (tid & ((1 << w) - 1)) | (k << w) | ((tid >> w) << (w + eb))


def tile_off(t, s):
    t = np.asarray(t)
    R, hA, qA, qB = s["R"], s["hA"], s["qA"], s["qB"]
    return (t & ((1 << R) - 1)) | (((t >> R) & ((1 << hA) - 1)) << qA) | ((t >> (R + hA)) << qB)


def block_base(b, s):
    R, hA, qA, qB, tb = s["R"], s["hA"], s["qA"], s["qB"], s["tb"]
    g1, g2 = qA - R, qB - (qA + hA)
    top = qB + (tb - R - hA)
    b = np.asarray(b)
    lo = b & ((1 << g1) - 1)
    b = b >> g1
    mid = b & ((1 << g2) - 1)
    b = b >> g2
    return (lo << R) | (mid << (qA + hA)) | (b << top)


def global_bit(s, t):
    R, hA, qA, qB = s["R"], s["hA"], s["qA"], s["qB"]
    if t < R:
        return t
    if t < R + hA:
        return qA + (t - R)
    return qB + (t - R - hA)


# LDS swizzle for tiles of 2^eb elements per thread: pos = t ^ ((t >> eb) & m)
# (m = 31 for 8-byte entries, 15 for 16-byte ones); cost-vector tiles of 4- and
# 2-byte entries use pos = t ^ ((t >> 5) & 31)
def swz(t, elem_bytes, eb=4):
    t = np.asarray(t)
    if elem_bytes >= 8:
        return t ^ ((t >> eb) & (31 if elem_bytes == 8 else 15))
    return t ^ ((t >> 5) & 31)


# gfx950 LDS service groups, (lanes served together, 4-byte banks), measured
# with the bank-conflict counter on strided and permuted lane patterns:
# ds_read_b64 32 lanes / 64 banks, ds_write_b64 16 / 32, ds_write_b128 8 / 32;
# ds_read_b128 is modelled as 16 lanes / 64 banks (its counter reads zero for
# every window of the 16-byte map)
LDS_GROUPS = {8: {"read": (32, 64), "write": (16, 32)}, 16: {"read": (16, 64), "write": (8, 32)}}


def bank_conflict_degree(elem_bytes, tb, w, eb=4, direction="read"):
    """Worst number of distinct 4-byte words that one bank serves within a group
    of lanes served together, over all registers k (1 = conflict free)."""
    group, nbanks = LDS_GROUPS[elem_bytes][direction]
    nthreads = 1 << (tb - eb)
    worst = 1
    for k in range(1 << eb):
        for g0 in range(0, min(64, nthreads), group):
            tid = np.arange(g0, min(g0 + group, nthreads))
            pos = swz(tmap(tid, k, w, eb), elem_bytes, eb)
            words = (pos * elem_bytes // 4)[:, None] + np.arange(max(1, elem_bytes // 4))[None, :]
            counts = np.bincount((words % nbanks).ravel(), minlength=nbanks)
            worst = max(worst, int(counts.max()))
    return worst


def test_bank_model_reproduces_measured_conflicts():
    """The group model against counter readings taken on the hardware: lanes
    writing 8-byte entries at a stride of 2 entries cost 4 extra cycles per
    instruction (2-way in each 16-lane group), reading them 2 (2-way in each
    32-lane group); lanes l and l + 16 on the same bank conflict for reads only."""
    def extra(pos, elem_bytes, direction):
        group, nbanks = LDS_GROUPS[elem_bytes][direction]
        e = 0
        for g0 in range(0, 64, group):
            words = np.asarray(pos[g0:g0 + group]) * (elem_bytes // 4)
            words = (words[:, None] + np.arange(elem_bytes // 4)[None, :]).ravel()
            e += np.bincount(words % nbanks, minlength=nbanks).max() - 1
        return e
    lanes = np.arange(64)
    assert extra(lanes * 2, 8, "write") == 4 and extra(lanes * 2, 8, "read") == 2
    assert extra(lanes * 4, 8, "write") == 12 and extra(lanes * 4, 8, "read") == 6
    pair16 = (lanes % 16) | ((lanes // 16) << 5)
    assert extra(pair16, 8, "write") == 0 and extra(pair16, 8, "read") == 2
    assert extra(lanes * 2, 16, "write") == 8 and extra(lanes * 4, 16, "write") == 24
    assert extra(lanes, 8, "write") == extra(lanes, 8, "read") == extra(lanes, 16, "write") == 0
    # a map searched against reads alone, pos = t ^ L(t >> 5) with these columns, read
    # zero conflicts but 4 extra cycles per 8-byte write in window 0 (16 elements per
    # thread) on the counter; the model must tell it from the map in use
    cols = [26, 14, 19, 24, 6, 23, 3, 20, 8]

    def old_map(t):
        x = np.zeros_like(t)
        for j, c in enumerate(cols):
            x ^= ((t >> (5 + j)) & 1) * c
        return t ^ x
    t0 = tmap(lanes, 0, 0, 4)
    assert extra(old_map(t0), 8, "write") == 4 and extra(old_map(t0), 8, "read") == 0
    assert extra(swz(t0, 8, 4), 8, "write") == 0 and extra(swz(t0, 8, 4), 8, "read") == 0


def _check_plan(n, plan, elem_bytes, emulate):
    eb = plan["eb"]
    wide = plan.get("wide", False)
    # wide complex128 tiles pass through LDS as 8-byte halves, 1024 threads
    lds_elem, max_thread_bits, lds_cap = (8, 10, 131072) if wide else (elem_bytes, 9, 65536)
    if wide:
        assert elem_bytes == 16 and n > 14
    seen = []
    for si, s in enumerate(plan["sweeps"]):
        tb, R, hA, qA, qB, act_lo = s["tb"], s["R"], s["hA"], s["qA"], s["qB"], s["act_lo"]
        hB = tb - R - hA
        assert 1 <= tb <= n and 0 <= R <= tb and 0 <= hA and hB >= 0
        assert tb - eb <= max_thread_bits, "too many threads"
        assert (1 << tb) * lds_elem <= lds_cap, "tile exceeds its LDS buffer"
        assert R <= qA and qA + hA <= qB and qB + hB <= n, "segments must be ordered and inside n"
        if si == 0:
            assert act_lo == 0
        else:
            assert act_lo == R and (1 << R) * elem_bytes >= (64 if wide else 128), "contiguous bytes per run"
        gbits = [global_bit(s, t) for t in range(tb)]
        assert len(set(gbits)) == tb and max(gbits) < n
        assert 0 <= s["w_store"] <= tb - eb
        # the first chunk's window is the load mapping: the top window, or (wide
        # tiles) window 6, whose lanes are tile bits [0, 6) as in the top window
        assert s["chunks"][0][0] == tb - eb or (wide and s["chunks"][0][0] == 6), "first window must load coalesced"
        for (w, jlo, jhi) in s["chunks"]:
            assert 0 <= w <= tb - eb and 0 <= jlo < jhi <= eb
            for j in range(jlo, jhi):
                t = w + j
                assert t >= act_lo, "butterfly on a passenger bit"
                seen.append(gbits[t])
        if emulate:
            nthreads = 1 << (tb - eb)
            tid = np.arange(nthreads)[:, None]
            k = np.arange(1 << eb)[None, :]
            windows = {c[0] for c in s["chunks"]} | {s["w_store"]}
            for w in windows:
                t = tmap(tid, k, w, eb).ravel()
                assert np.array_equal(np.sort(t), np.arange(1 << tb))
                pos = swz(t, lds_elem, eb)
                assert np.array_equal(np.sort(pos), np.arange(1 << tb))
                off = tile_off(t, s)
                blocks = np.arange(1 << (n - tb))[:, None]
                g = (block_base(blocks, s) | off[None, :]).ravel()
                assert g.min() >= 0 and g.max() < (1 << n)
                assert np.array_equal(np.sort(g), np.arange(1 << n)), "sweep does not cover every element once"
                # the split into per-thread and per-register parts used by the kernels
                thr = (tid & ((1 << w) - 1)) | ((tid >> w) << (w + eb))
                assert np.array_equal(tile_off(thr | (k << w), s), tile_off(thr, s) + tile_off(k << w, s))
            # window changes between windows <= 6 keep every element in its wave
            # (the kernels skip the workgroup barrier for them)
            local = sorted(x for x in windows | {s["tb"] - eb} if x <= 6)
            owner = {}
            for w in local:
                t = tmap(tid, k, w, eb)
                o = np.empty(1 << tb, dtype=np.int64)
                o[t.ravel()] = np.broadcast_to(tid >> 6, t.shape).ravel()
                owner[w] = o
            for w in local[1:]:
                assert np.array_equal(owner[w], owner[local[0]]), (n, si, local)
    assert sorted(seen) == list(range(n)), "every qubit must be butterflied exactly once per layer"


def _page_bits_per_sweep(plan, elem_bytes):
    pb = 0
    while (1 << (pb + 1)) * elem_bytes <= (2 << 20):
        pb += 1
    return [sum(1 for t in range(s["tb"]) if global_bit(s, t) >= pb) for s in plan["sweeps"]]


def test_page_bits_are_spread():
    # LABS n=26 complex128 (two sweeps) and n=31 complex64 (three sweeps): no
    # sweep's tile spans more than 2^5 pages of 2 MiB (a plain split, one
    # contiguous high segment per sweep, spans up to 2^9)
    p26 = _lib.plan_describe(26, _lib.QAOA_C128)
    p31 = _lib.plan_describe(31, _lib.QAOA_C64)
    assert max(_page_bits_per_sweep(p26, 16)) <= 5
    assert max(_page_bits_per_sweep(p31, 8)) <= 5


@pytest.mark.parametrize("sdt,eb", [(_lib.QAOA_C128, 16), (_lib.QAOA_C64, 8)])
def test_state_plans(sdt, eb):
    for n in range(1, _lib.QAOA_MAX_QUBITS + 1):
        plan = _lib.plan_describe(n, sdt)
        _check_plan(n, plan, eb, emulate=n <= 17 or (plan["wide"] and n <= 22))
        if plan["single"]:
            assert len(plan["sweeps"]) == 1


@pytest.mark.parametrize("sdt", [_lib.QAOA_C128, _lib.QAOA_C64])
def test_short_last_chunks_sit_at_the_window_top(sdt):
    # the sweep kernels apply a short last chunk with specialised code when it
    # holds the top register bits of its window (jhi = eb, jlo in 1..3)
    for n in range(16, _lib.QAOA_MAX_QUBITS + 1):
        plan = _lib.plan_describe(n, sdt)
        for s in plan["sweeps"]:
            w, jlo, jhi = s["chunks"][-1]
            if jhi - jlo < plan["eb"]:
                assert jhi == plan["eb"] and 1 <= jlo <= 3, (n, s["chunks"])


@pytest.mark.parametrize("elem", [2, 4, 8])
def test_transform_plans(elem):
    for n in range(1, _lib.QAOA_MAX_QUBITS + 1):
        _check_plan(n, _lib.plan_describe(n, -1, elem), elem, emulate=n <= 16)


@pytest.mark.parametrize("sdt,eb", [(_lib.QAOA_C128, 16), (_lib.QAOA_C64, 8)])
def test_adjoint_plans(sdt, eb):
    for n in range(1, _lib.QAOA_MAX_QUBITS + 1):
        plan = _lib.plan_describe(n, sdt, kind=_lib.PLAN_ADJOINT)
        assert plan["eb"] <= 3
        _check_plan(n, plan, eb, emulate=n <= 16)


def test_headline_plans_sweep_counts():
    # LABS n=26 complex128: two sweeps per layer with 2^14-element tiles and
    # 64-byte runs; n=31 complex64: three sweeps
    p26 = _lib.plan_describe(26, _lib.QAOA_C128)
    assert p26["wide"] and len(p26["sweeps"]) == 2
    assert len(_lib.schedule_describe(26, 10, _lib.QAOA_C128)) == 11
    assert len(_lib.plan_describe(31, _lib.QAOA_C64)["sweeps"]) == 3
    assert _lib.plan_describe(12, _lib.QAOA_C128)["single"]
    # wide tiles only where they save a sweep
    for n in range(1, _lib.QAOA_MAX_QUBITS + 1):
        pl = _lib.plan_describe(n, _lib.QAOA_C128)
        if pl["wide"]:
            assert n > 14 and len(pl["sweeps"]) < len(_lib.plan_describe(n, _lib.QAOA_C64)["sweeps"]) + 1
    assert [n for n in range(15, 35) if _lib.plan_describe(n, _lib.QAOA_C128)["wide"]] == [22, 23, 24, 25, 26] + \
        list(range(31, 35))


@pytest.mark.parametrize("elem_bytes", [8, 16])
@pytest.mark.parametrize("eb", [3, 4])
def test_lds_swizzle_is_a_linear_permutation(elem_bytes, eb):
    # the kernels split pos(thr | k << w) into pos(thr) ^ pos(k << w): the map
    # must be XOR-linear, and a permutation of every tile size it serves
    for tb in range(eb + 1, 15):
        t = np.arange(1 << tb)
        pos = swz(t, elem_bytes, eb)
        assert np.array_equal(np.sort(pos), t)
    rng = np.random.default_rng(elem_bytes + eb)
    a, b = rng.integers(0, 1 << 14, size=(2, 4096))
    assert np.array_equal(swz(a ^ b, elem_bytes, eb), swz(a, elem_bytes, eb) ^ swz(b, elem_bytes, eb))


@pytest.mark.parametrize("elem_bytes,tbmax", [(8, 14), (16, 12)])
@pytest.mark.parametrize("eb", [3, 4])
def test_lds_swizzle_conflict_free_in_every_window(elem_bytes, tbmax, eb):
    # not only the windows today's plans use: every window of every multi-wave tile
    for tb in range(eb + 6, tbmax + 1):
        for w in range(0, tb - eb + 1):
            for direction in ("read", "write"):
                assert bank_conflict_degree(elem_bytes, tb, w, eb=eb, direction=direction) == 1, \
                    (elem_bytes, tb, w, eb, direction)


@pytest.mark.parametrize("sdt", [_lib.QAOA_C128, _lib.QAOA_C64])
@pytest.mark.parametrize("kind", [_lib.PLAN_EVOLVE, _lib.PLAN_ADJOINT])
def test_lds_swizzle_conflict_free(sdt, kind):
    # every register window that any plan uses is free of LDS bank conflicts:
    # complex64 exchanges 8-byte entries, complex128 16-byte ones, or 8-byte
    # real and imaginary passes in wide tiles
    used = set()
    for n in range(1, _lib.QAOA_MAX_QUBITS + 1):
        plan = _lib.plan_describe(n, sdt, kind=kind)
        eb = plan["eb"]
        lds_elem = 8 if (sdt == _lib.QAOA_C64 or plan["wide"]) else 16
        for sw in plan["sweeps"]:
            if sw["tb"] - eb < 6:
                continue  # fewer than 64 threads: single partial wave
            for w in {c[0] for c in sw["chunks"]} | {sw["w_store"], sw["tb"] - eb}:
                used.add((lds_elem, sw["tb"], w, eb))
    assert used
    for lds_elem, tb, w, eb in sorted(used):
        for direction in ("read", "write"):
            assert bank_conflict_degree(lds_elem, tb, w, eb=eb, direction=direction) == 1, \
                (lds_elem, tb, w, eb, direction)


def test_server_validation():
    h = ctypes.c_void_p()
    lib = _lib.lib
    lib.qaoa_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    assert lib.qaoa_server_create(0, 1, 1, ctypes.byref(h)) == _lib.QAOA_ERR_INVALID
    assert lib.qaoa_server_create(1 << 30, 0, 1, ctypes.byref(h)) == _lib.QAOA_ERR_INVALID
    assert lib.qaoa_server_create(1 << 30, 1, 0, ctypes.byref(h)) == _lib.QAOA_ERR_INVALID
    assert b"max_in_flight" in lib.qaoa_last_error()
    lib.qaoa_server_destroy.argtypes = [ctypes.c_void_p]
    assert lib.qaoa_server_destroy(None) == _lib.QAOA_ERR_INVALID


def _sweep_qubits(s):
    return {global_bit(s, t) for t in range(s["act_lo"], s["tb"])}


@pytest.mark.parametrize("n,sdt", [(13, _lib.QAOA_C128), (20, _lib.QAOA_C128), (26, _lib.QAOA_C128),
                                   (31, _lib.QAOA_C64), (34, _lib.QAOA_C64), (14, _lib.QAOA_C64)])
@pytest.mark.parametrize("p", [1, 2, 3, 10, 33, 64])
@pytest.mark.parametrize("init,reduce", [(True, True), (False, False)])
@pytest.mark.parametrize("fuse,wide", [(1, 1), (0, 1), (1, 0)])
def test_schedule_is_a_reordering_of_the_layers(n, sdt, p, init, reduce, fuse, wide):
    with _lib.tuning(wide_tiles=wide, fuse_layers=fuse):
        _check_schedule(n, sdt, p, init, reduce, fuse)


def _check_schedule(n, sdt, p, init, reduce, fuse):
    """Flattened, the launches must apply phase(l) then one gate per qubit of
    layer l, for l = 0..p-1 in order; gates of one layer may come in any order
    (they commute), nothing else may move (Sections 3.1-3.2)."""
    plan = _lib.plan_describe(n, sdt)
    sched = _lib.schedule_describe(n, p, sdt, init, reduce)
    if plan["single"]:
        assert sched == []
        return
    nsw = len(plan["sweeps"])
    assert len(sched) == (1 + (nsw - 1) * p if fuse else nsw * p)
    ops = []
    for i, (sw, layer, flags) in enumerate(sched):
        qs = _sweep_qubits(plan["sweeps"][sw])
        assert bool(flags & _lib.F_INIT) == (init and i == 0)
        assert bool(flags & _lib.F_EXPV) == (reduce and i == len(sched) - 1)
        assert not (flags & _lib.F_FUSE and flags & (_lib.F_PHASE | _lib.F_EXPV | _lib.F_INIT))
        if flags & _lib.F_PHASE:
            ops.append(("phase", layer))
        ops += [("mix", layer, q) for q in qs]
        if flags & _lib.F_FUSE:
            assert layer + 1 < p
            ops.append(("phase", layer + 1))
            ops += [("mix", layer + 1, q) for q in qs]
    # canonical grouping
    pos = 0
    for layer in range(p):
        assert ops[pos] == ("phase", layer), (layer, ops[pos])
        pos += 1
        gates = ops[pos:pos + n]
        assert sorted(gates) == [("mix", layer, q) for q in range(n)]
        pos += n
    assert pos == len(ops)


def test_schedule_counts_and_fusion():
    # LABS n=31 complex64, p=10: 3 sweeps per layer fused to 21 launches;
    # n=26 complex128: 2 sweeps per layer, 11 launches
    sched = _lib.schedule_describe(31, 10, _lib.QAOA_C64)
    assert len(sched) == 21
    assert sum(1 for s in sched if s[2] & _lib.F_FUSE) == 9
    sched = _lib.schedule_describe(26, 10, _lib.QAOA_C128)
    assert len(sched) == 11 and sum(1 for s in sched if s[2] & _lib.F_FUSE) == 9
    with pytest.raises(_lib.QaoaError):
        _lib.schedule_describe(0, 1)
    with pytest.raises(_lib.QaoaError):
        _lib.schedule_describe(20, 1, kind=2)


@pytest.mark.parametrize("n,sdt", [(12, _lib.QAOA_C128), (18, _lib.QAOA_C128), (26, _lib.QAOA_C128),
                                   (31, _lib.QAOA_C64), (16, _lib.QAOA_C64)])
@pytest.mark.parametrize("p", [1, 2, 3, 10, 40])
@pytest.mark.parametrize("fuse", [1, 0])
def test_adjoint_schedule_undoes_layers_in_reverse(n, sdt, p, fuse):
    with _lib.tuning(fuse_layers=fuse):
        _check_adjoint_schedule(n, sdt, p, fuse)


def _check_adjoint_schedule(n, sdt, p, fuse):
    """Flattened, the reverse pass must undo, for l = p-1 .. 0, one gate per
    qubit of layer l (any order) and then layer l's phase; lambda = c psi is
    formed by the first launch only; every (layer, sweep) partial slot is
    written exactly once, and the gamma term of layer l by the launch that
    undoes its phase."""
    plan = _lib.plan_describe(n, sdt, kind=_lib.PLAN_ADJOINT)
    sched = _lib.schedule_describe(n, p, sdt, kind=_lib.SCHED_ADJOINT)
    if plan["single"]:
        assert sched == []
        return
    nsw = len(plan["sweeps"])
    assert len(sched) == (1 + (nsw - 1) * p if fuse else nsw * p)
    ops, slots = [], []
    for i, (sw, layer, flags) in enumerate(sched):
        qs = _sweep_qubits(plan["sweeps"][sw])
        assert bool(flags & _lib.A_FIRST) == (i == 0)
        assert flags in (0, _lib.A_FIRST, _lib.A_PHASE, _lib.A_FUSE)
        ops += [("undo", layer, q) for q in qs]
        slots.append((layer, sw))
        if flags & (_lib.A_PHASE | _lib.A_FUSE):
            ops.append(("unphase", layer))
        if flags & _lib.A_FUSE:
            assert layer >= 1
            ops += [("undo", layer - 1, q) for q in qs]
            slots.append((layer - 1, sw))
    assert sorted(slots) == [(l, s) for l in range(p) for s in range(nsw)]
    pos = 0
    for layer in range(p - 1, -1, -1):
        assert sorted(ops[pos:pos + n]) == [("undo", layer, q) for q in range(n)]
        pos += n
        assert ops[pos] == ("unphase", layer)
        pos += 1
    assert pos == len(ops)


def test_tuning_knobs():
    assert _lib.get_tuning(_lib.TUNE_WIDE_TILES) == 1 and _lib.get_tuning(_lib.TUNE_FUSE_LAYERS) == 1
    with _lib.tuning(wide_tiles=0):
        assert not _lib.plan_describe(26, _lib.QAOA_C128)["wide"]
        assert len(_lib.plan_describe(26, _lib.QAOA_C128)["sweeps"]) == 3
    assert _lib.plan_describe(26, _lib.QAOA_C128)["wide"]
    with _lib.tuning(fuse_layers=0):
        assert len(_lib.schedule_describe(26, 10, _lib.QAOA_C128)) == 20
    for bad in ((2, 1), (0, 2), (-1, 0)):
        with pytest.raises(_lib.QaoaError):
            _lib.set_tuning(*bad)
    with pytest.raises(_lib.QaoaError):
        _lib.get_tuning(7)


def test_lower_windows_are_wave_local():
    # in the headline plans only the top window (tb - 4) is not wave-local: the
    # other chunks use windows <= 6, and the top chunk comes either first (the
    # load window) or, when a plan loads in window 6, last
    for n, sdt in ((26, _lib.QAOA_C128), (31, _lib.QAOA_C64), (20, _lib.QAOA_C128)):
        for sw in _lib.plan_describe(n, sdt)["sweeps"]:
            top = sw["tb"] - 4
            ws = [w for (w, _, _) in sw["chunks"]]
            assert all(w <= 6 for w in ws if w != top), (n, sw["chunks"])
            assert ws.count(top) == 1 and (ws[0] == top or ws[-1] == top), (n, sw["chunks"])
    a, b = _lib.plan_describe(26, _lib.QAOA_C128)["sweeps"]
    assert [w for (w, _, _) in a["chunks"]] == [6, 0, 2, 10] and a["chunks"][2] == (2, 2, 4)
    assert [w for (w, _, _) in b["chunks"]] == [6, 2, 10] and b["w_store"] == 10


def test_tile_kernels_have_no_static_lds(tmp_path):
    """The tile kernels address their LDS tiles by absolute byte address, which
    is right only when their dynamic LDS starts at 0, i.e. they declare no
    static LDS: read .group_segment_fixed_size from the built code object."""
    import shutil
    import subprocess
    tools = "/opt/rocm/llvm/bin"
    objcopy, bundler, readelf = (os.path.join(tools, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf"))
    if not all(os.path.exists(t) for t in (objcopy, bundler, readelf)):
        pytest.skip("LLVM tools not found")
    fat, co = tmp_path / "fatbin.bin", tmp_path / "dev.co"
    subprocess.check_call([objcopy, f"--dump-section=.hip_fatbin={fat}", _lib.LIB_PATH, str(tmp_path / "host.so")])
    subprocess.check_call([bundler, "--unbundle", "--type=o", f"--input={fat}",
                           "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"])
    notes = subprocess.check_output([readelf, "--notes", str(co)], text=True)
    sizes, last = {}, None
    for line in notes.splitlines():
        line = line.strip()
        if line.startswith(".group_segment_fixed_size:"):
            last = int(line.split(":")[1])
        elif line.startswith(".name:") and last is not None:
            sizes[line.split(":", 1)[1].strip()] = last
            last = None
    tile = {k: v for k, v in sizes.items() if any(s in k for s in ("qaoa_sweep_kernel", "qaoa_tile_kernel", "qaoa_adjoint"))}
    assert len(tile) > 20
    assert all(v == 0 for v in tile.values()), {k: v for k, v in tile.items() if v}
    shutil.rmtree(tmp_path, ignore_errors=True)
