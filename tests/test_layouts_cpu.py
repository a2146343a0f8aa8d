"""CPU checks of the state layouts between sweep launches (no GPU calls).

With a second state buffer, a launch whose contiguous run is shorter than a
128-byte line writes a rotated bit order of the element positions into that
buffer and the next launch reads it there.  Here the kernels' position
arithmetic (Layout form: run, two segments, block bits in the gaps) is
re-evaluated in Python for every launch of many schedules, and the bit maps
are checked: each is a permutation of the n position bits; every launch reads
exactly the buffer and order the previous one wrote; a launch that reads and
writes the same buffer uses one order for both (so each workgroup writes back
exactly the positions it read: in-place safe); the first launch reads and the
last writes the caller's buffer in natural order (position = index); and every
store of the wide complex128 plans covers whole 128-byte lines.
"""
import pytest

from paper_2309_04841_amd import _lib


def _tile_off(t, lay):
    R, hA, qA, qB = lay
    return (t & ((1 << R) - 1)) | (((t >> R) & ((1 << hA) - 1)) << qA) | ((t >> (R + hA)) << qB)


def _block_base(b, tb, lay):
    R, hA, qA, qB = lay
    g1, g2, top = qA - R, qB - (qA + hA), qB + (tb - R - hA)
    lo = b & ((1 << g1) - 1)
    b >>= g1
    mid = b & ((1 << g2) - 1)
    b >>= g2
    return (lo << R) | (mid << (qA + hA)) | (b << top)


def _tile_global_bits(sw):
    R, hA, qA, qB, tb = sw["R"], sw["hA"], sw["qA"], sw["qB"], sw["tb"]
    return list(range(R)) + [qA + j for j in range(hA)] + [qB + j for j in range(tb - R - hA)]


def _position_bits(n, sw, lay):
    """Position bit of every global bit for sweep `sw` read or written in layout `lay`."""
    tbits = _tile_global_bits(sw)
    bbits = [i for i in range(n) if i not in tbits]
    pos = [None] * n
    for j, g in enumerate(tbits):
        off = _tile_off(1 << j, lay)
        assert off and off & (off - 1) == 0
        pos[g] = off.bit_length() - 1
    for r, g in enumerate(bbits):
        off = _block_base(1 << r, sw["tb"], lay)
        assert off and off & (off - 1) == 0
        pos[g] = off.bit_length() - 1
    return pos


def _natural(sw):
    return (sw["R"], sw["hA"], sw["qA"], sw["qB"])


def _store_run_bytes(sw, lay, w, elem_bytes, eb=4):
    """Bytes of the contiguous runs one wave writes per store instruction in window w."""
    # lane bits 0..5 of the thread index are tile bits [0, w) and [w + eb, w + eb + 6 - w)
    lanes = list(range(min(w, 6))) + [w + eb + j for j in range(max(0, 6 - w))]
    pbits = sorted(_tile_off(1 << t, lay).bit_length() - 1 for t in lanes if t < sw["tb"])
    run = 0
    while run < len(pbits) and pbits[run] == run:
        run += 1
    return (1 << run) * elem_bytes


CASES = [(n, p, sdt) for sdt in (_lib.QAOA_C128, _lib.QAOA_C64) for n in range(13, 35)
         for p in (1, 2, 3, 10)]


@pytest.mark.parametrize("alt", [0, 1])
@pytest.mark.parametrize("wide", [0, 1])
@pytest.mark.parametrize("fuse", [0, 1])
def test_layouts_chain(wide, fuse, alt):
    rotated = 0
    with _lib.tuning(wide_tiles=wide, fuse_layers=fuse):
        for n, p, sdt in CASES:
            plan = _lib.plan_describe(n, sdt)
            sched = _lib.schedule_describe(n, p, sdt)
            lays = _lib.layout_describe(n, p, sdt, alt=bool(alt))
            assert len(lays) == len(sched)
            if not sched:
                continue
            S = 16 if sdt == _lib.QAOA_C128 else 8
            prev, prev_alt = list(range(n)), False  # the caller's state is in natural order
            for i, ((sw_i, _layer, flags), (ld, ld_alt, st, st_alt)) in enumerate(zip(sched, lays)):
                sw = plan["sweeps"][sw_i]
                pin, pout = _position_bits(n, sw, ld), _position_bits(n, sw, st)
                assert sorted(pin) == list(range(n)) and sorted(pout) == list(range(n))
                if not flags & _lib.F_INIT:
                    assert pin == prev and ld_alt == prev_alt, (n, p, sdt, i)
                if ld_alt == st_alt:
                    assert ld == st, (n, p, sdt, i)  # in place: the same positions are read and written
                w_out = sw["tb"] - 4 if flags & (_lib.F_FUSE | _lib.F_EXPV) else sw["w_store"]
                if st != _natural(sw):
                    rotated += 1
                    assert alt and st_alt
                    assert _store_run_bytes(sw, st, w_out, S) >= 128
                    assert _store_run_bytes(sw, st, w_out, S) > _store_run_bytes(sw, _natural(sw), w_out, S)
                prev, prev_alt = pout, st_alt
            assert prev == list(range(n)) and not prev_alt, (n, p, sdt)  # ends in the caller's buffer, natural
    if wide and alt:
        assert rotated > 0  # the wide complex128 plans use the rotated order
    if not alt:
        assert rotated == 0


def test_labs26_c128_stores_whole_lines():
    """The benchmarked schedule: every launch stores runs of at least 128 bytes
    (the 12-qubit sweep writes 8 KiB runs in its rotated order instead of 64-byte
    runs), and only its loads keep 64-byte runs."""
    n, p = 26, 10
    plan = _lib.plan_describe(n, _lib.QAOA_C128)
    lays = _lib.layout_describe(n, p, _lib.QAOA_C128)
    for (sw_i, _layer, flags), (ld, ld_alt, st, st_alt) in zip(_lib.schedule_describe(n, p, _lib.QAOA_C128), lays):
        sw = plan["sweeps"][sw_i]
        w_out = sw["tb"] - 4 if flags & (_lib.F_FUSE | _lib.F_EXPV) else sw["w_store"]
        assert _store_run_bytes(sw, st, w_out, 16) >= 128
    assert lays[1][2] == (9, 5, 17, 22) and lays[1][3] and lays[2][1] and not lays[2][3]


def test_workspace_holds_second_buffer_only_where_used():
    """The evolve workspace has room for a second state exactly for the plans
    that rotate (of n = 13..34, only complex128 at n = 26, whose 2^14-element
    tiles keep 64-byte runs); everywhere else it is the plain workspace."""
    with_alt = set()
    for sdt, S in ((_lib.QAOA_C128, 16), (_lib.QAOA_C64, 8)):
        for n in range(13, 35):
            rot = False
            for wide in (0, 1):
                for fuse in (0, 1):
                    with _lib.tuning(wide_tiles=wide, fuse_layers=fuse):
                        rot |= any(l[3] for l in _lib.layout_describe(n, 3, sdt, alt=True))
            full = _lib.workspace_bytes(_lib.QAOA_OP_EVOLVE, n, sdt)
            base = _lib.workspace_bytes(_lib.QAOA_OP_EXPECTATION, n, sdt)
            if rot:
                with_alt.add((n, sdt))
                assert full == (base + 255) // 256 * 256 + (1 << n) * S
            else:
                assert full == base
    assert with_alt == {(26, _lib.QAOA_C128)}
