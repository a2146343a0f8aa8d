"""Host-side checks of the XY mixer path (Section 3.2): the sweep planner's gate
order, its tile geometry, an emulation of the tile kernel's index arithmetic
against the oracle, and argument validation of qaoa_evolve_xy.  No GPU."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2309_04841_amd import _lib
from test_abi_cpu import block_base, global_bit, tile_off

FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: each call fails validation first
MIXERS = [(_lib.MIXER_XY_RING, oracle.XY_RING), (_lib.MIXER_XY_COMPLETE, oracle.XY_COMPLETE)]


def _edges(n, mixer):
    if mixer == _lib.MIXER_XY_RING:
        e = [(i, i + 1) for i in range(0, n - 1, 2)] + [(i, i + 1) for i in range(1, n - 1, 2)]
        return e + ([(n - 1, 0)] if n > 2 else [])
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def _plan_gates(n, plan):
    """The plan's gates as qubit pairs, in application order."""
    out = []
    for s in plan["sweeps"]:
        for ti, tj in s["gates"]:
            out.append((global_bit(s, ti), global_bit(s, tj)))
    return out


def _passengers(elem_bytes):
    p = 0
    while (1 << p) * elem_bytes < 128:
        p += 1
    return p


@pytest.mark.parametrize("sdt,elem", [(_lib.QAOA_C128, 16), (_lib.QAOA_C64, 8)])
@pytest.mark.parametrize("mixer", [_lib.MIXER_XY_RING, _lib.MIXER_XY_COMPLETE])
def test_xy_plan_is_a_valid_reordering(sdt, elem, mixer):
    for n in range(2, 31):
        plan = _lib.xy_plan_describe(n, mixer, sdt)
        edges = _edges(n, mixer)
        assert plan["single"] == (n <= 12)
        if plan["single"]:
            assert len(plan["sweeps"]) == 1
        for s in plan["sweeps"]:
            tb, R, hA, qA, qB = s["tb"], s["R"], s["hA"], s["qA"], s["qB"]
            hB = tb - R - hA
            assert tb == min(n, 12) and hA >= 0 and hB >= 0
            assert R >= min(n, _passengers(elem)), "coalesced runs need the low passenger bits"
            assert qA >= R and (hA == 0 or qB >= qA + hA) and qB + hB <= n
            assert len(s["gates"]) <= 128
            for ti, tj in s["gates"]:
                assert 0 <= ti < tb and 0 <= tj < tb and ti != tj
        got = _plan_gates(n, plan)
        # every edge exactly once, with its orientation
        assert sorted(got) == sorted(edges)
        # gates that share a qubit keep their relative order (disjoint ones commute)
        pos = {e: k for k, e in enumerate(got)}
        for a in range(len(edges)):
            for b in range(a + 1, len(edges)):
                if set(edges[a]) & set(edges[b]):
                    assert pos[edges[a]] < pos[edges[b]], (n, edges[a], edges[b])


def test_xy_plan_sweep_counts():
    # ring: 3 sweeps per layer at n = 26 (X mixer: 2); complete graph: 13 sweeps
    # for its 325 two-qubit gates at n = 26 (taking gates in the fixed order
    # while they fit needed 28)
    assert len(_lib.xy_plan_describe(26, _lib.MIXER_XY_RING)["sweeps"]) <= 3
    assert len(_lib.xy_plan_describe(20, _lib.MIXER_XY_RING)["sweeps"]) <= 2
    assert len(_lib.xy_plan_describe(26, _lib.MIXER_XY_COMPLETE)["sweeps"]) <= 13
    assert len(_lib.xy_plan_describe(30, _lib.MIXER_XY_COMPLETE)["sweeps"]) <= 17


def _insert_two_zeros(q, lo, hi):
    q = ((q >> lo) << (lo + 1)) | (q & ((1 << lo) - 1))
    return ((q >> hi) << (hi + 1)) | (q & ((1 << hi) - 1))


def _emulate_xy_layer(n, plan, beta, psi):
    """The tile kernel's index arithmetic in numpy: each sweep gathers every tile
    (block_base + tile_off), applies its gate list on tile bits, scatters back."""
    psi = psi.copy()
    ca, sb = np.cos(beta), np.sin(beta)
    for s in plan["sweeps"]:
        tb = s["tb"]
        t = np.arange(1 << tb)
        offs = tile_off(t, s)
        q = np.arange(1 << (tb - 2))
        for b in range((1 << n) >> tb):
            idx = block_base(b, s) + offs
            tile = psi[idx]
            for ti, tj in s["gates"]:
                lo, hi = min(ti, tj), max(ti, tj)
                x = _insert_two_zeros(q, lo, hi)
                x0, x1 = x | (1 << tj), x | (1 << ti)
                u, v = tile[x0].copy(), tile[x1].copy()
                tile[x0] = ca * u - 1j * sb * v
                tile[x1] = ca * v - 1j * sb * u
            psi[idx] = tile
    return psi


@pytest.mark.parametrize("n", [5, 13, 15])
@pytest.mark.parametrize("mixer,kind", MIXERS)
def test_xy_plan_emulation_matches_oracle(n, mixer, kind):
    rng = np.random.default_rng(7 * n + mixer)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    plan = _lib.xy_plan_describe(n, mixer, _lib.QAOA_C128)
    # the tiles of one sweep partition the state
    for s in plan["sweeps"]:
        idx = np.concatenate([block_base(b, s) + tile_off(np.arange(1 << s["tb"]), s)
                              for b in range((1 << n) >> s["tb"])])
        assert np.array_equal(np.sort(idx), np.arange(1 << n))
    got = _emulate_xy_layer(n, plan, 0.43, psi)
    ref = oracle.apply_xy_mixer(n, kind, 0.43, psi)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_xy_workspace_bytes():
    for n in (2, 12, 13, 26, 30):
        for mixer in (_lib.MIXER_XY_RING, _lib.MIXER_XY_COMPLETE):
            nb = _lib.xy_workspace_bytes(n, mixer, _lib.QAOA_C128)
            blocks = max(1, (1 << n) >> 12)
            assert nb >= 16 * blocks + 33 * 832 * 16
    for bad in ((1, 1), (31, 1), (10, 0), (10, 3)):
        with pytest.raises(_lib.QaoaError):
            _lib.xy_workspace_bytes(bad[0], bad[1], _lib.QAOA_C128)


def _evolve_xy(n=10, p=1, gamma=(0.1,), beta=(0.2,), mixer=1, diag=FAKE, ddt=1, off=0.0, dbytes=None,
               state=FAKE, sdt=1, sbytes=None, init=1, k=0, out=None, work=FAKE, wbytes=None):
    dbytes = (4 << n) if dbytes is None else dbytes
    sbytes = (16 << n) if sbytes is None else sbytes
    if wbytes is None:
        try:
            wbytes = _lib.xy_workspace_bytes(n, mixer, sdt)
        except _lib.QaoaError:
            wbytes = 1 << 30
    g = (ctypes.c_double * max(1, len(gamma)))(*gamma)
    b = (ctypes.c_double * max(1, len(beta)))(*beta)
    return _lib.lib.qaoa_evolve_xy(n, p, g, b, mixer, diag, ddt, off, dbytes, state, sdt, sbytes, init, k, out,
                                   work, wbytes, None)


@pytest.mark.parametrize("kw,code", [
    (dict(mixer=0), _lib.QAOA_ERR_INVALID),           # the X mixer has its own entry point
    (dict(mixer=7), _lib.QAOA_ERR_INVALID),
    (dict(n=1), _lib.QAOA_ERR_INVALID),
    (dict(n=31), _lib.QAOA_ERR_INVALID),
    (dict(sdt=5), _lib.QAOA_ERR_INVALID),
    (dict(init=3), _lib.QAOA_ERR_INVALID),
    (dict(init=2, k=11), _lib.QAOA_ERR_INVALID),     # Dicke weight above n
    (dict(init=2, k=-1), _lib.QAOA_ERR_INVALID),
    (dict(p=-1), _lib.QAOA_ERR_INVALID),
    (dict(diag=None), _lib.QAOA_ERR_INVALID),
    (dict(state=None), _lib.QAOA_ERR_INVALID),
    (dict(sbytes=16), _lib.QAOA_ERR_NOMEM),
    (dict(dbytes=16), _lib.QAOA_ERR_NOMEM),
    (dict(gamma=(float("nan"),)), _lib.QAOA_ERR_INVALID),
    (dict(wbytes=64), _lib.QAOA_ERR_NOMEM),
    (dict(work=None), _lib.QAOA_ERR_NOMEM),
])
def test_evolve_xy_rejects(kw, code):
    assert _evolve_xy(**kw) == code
    assert _lib.lib.qaoa_last_error().decode()
