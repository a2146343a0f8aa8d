"""Pins of the oracle's XY mixers (Section 3.2: M = sum over ring or complete-
graph edges of (X_i X_j + Y_i Y_j)/2, one layer = the product of the two-qubit
exponentials in a fixed edge order; the paper leaves the order open, the one used here is a stated reading).

The edge orders are written out here from their definition (not taken from the
oracle), and every layer is compared with the product of scipy expm of dense
Kronecker-product generators."""
import math

import numpy as np
import pytest

import oracle
from dense_ref import xy_generator, xy_layer_dense


def ring_order(n):
    even = [(i, i + 1) for i in range(0, n - 1, 2)]
    odd = [(i, i + 1) for i in range(1, n - 1, 2)]
    wrap = [(n - 1, 0)] if n > 2 else []
    return even + odd + wrap


def complete_order(n):
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def _rand_state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("kind,order", [(oracle.XY_RING, ring_order), (oracle.XY_COMPLETE, complete_order)])
def test_xy_layer_matches_dense_expm(n, kind, order):
    psi = _rand_state(n, 10 * n + kind)
    for beta in (0.37, -1.1, np.pi / 2):
        ref = xy_layer_dense(n, order(n), beta) @ psi
        got = oracle.apply_xy_mixer(n, kind, beta, psi)
        assert np.max(np.abs(got - ref)) < 1e-12, (n, kind, beta)


def test_single_gate_matches_dense_expm():
    n = 4
    psi = _rand_state(n, 3)
    for (i, j) in [(0, 1), (3, 0), (1, 3), (2, 1)]:
        U = __import__("scipy.linalg").linalg.expm(-1j * 0.8 * xy_generator(n, i, j))
        assert np.max(np.abs(oracle.apply_xy(n, i, j, 0.8, psi) - U @ psi)) < 1e-12


def test_two_qubit_closed_form():
    # exp(-i b (XX+YY)/2): |00>, |11> fixed; |01> -> cos b |01> - i sin b |10>
    b = 0.61
    for x, want in [(0, {0: 1.0}), (3, {3: 1.0}), (2, {2: np.cos(b), 1: -1j * np.sin(b)}),
                    (1, {1: np.cos(b), 2: -1j * np.sin(b)})]:
        psi = np.zeros(4, dtype=np.complex128)
        psi[x] = 1.0
        got = oracle.apply_xy(2, 0, 1, b, psi)
        ref = np.zeros(4, dtype=np.complex128)
        for k, v in want.items():
            ref[k] = v
        assert np.max(np.abs(got - ref)) < 1e-15


@pytest.mark.parametrize("kind", [oracle.XY_RING, oracle.XY_COMPLETE])
def test_hamming_weight_and_norm_preserved(kind):
    n = 7
    w = np.array([bin(x).count("1") for x in range(1 << n)])
    for k in (0, 2, 3, 7):
        psi = _rand_state(n, k) * (w == k)
        psi /= np.linalg.norm(psi)
        out = oracle.apply_xy_mixer(n, kind, 0.9, psi)
        assert abs(np.linalg.norm(out) - 1.0) < 1e-13
        assert np.max(np.abs(out[w != k])) == 0.0


def test_ring_groups_commute_internally():
    # gates inside the even group act on disjoint pairs: any order gives the same layer
    n = 8
    psi = _rand_state(n, 5)
    a = psi.copy()
    for i, j in [(0, 1), (2, 3), (4, 5), (6, 7)]:
        a = oracle.apply_xy(n, i, j, 0.4, a)
    b = psi.copy()
    for i, j in [(6, 7), (2, 3), (0, 1), (4, 5)]:
        b = oracle.apply_xy(n, i, j, 0.4, b)
    assert np.max(np.abs(a - b)) < 1e-14


@pytest.mark.parametrize("n,k", [(4, 2), (6, 3), (7, 1), (5, 0), (5, 5)])
def test_dicke_state(n, k):
    d = oracle.dicke_state(n, k)
    w = np.array([bin(x).count("1") for x in range(1 << n)])
    assert np.all(d[w != k] == 0)
    assert np.allclose(d[w == k], 1 / math.sqrt(math.comb(n, k)), atol=1e-15, rtol=0)
    assert abs(np.linalg.norm(d) - 1) < 1e-14


@pytest.mark.parametrize("kind,order", [(oracle.XY_RING, ring_order), (oracle.XY_COMPLETE, complete_order)])
@pytest.mark.parametrize("init", ["plus", "dicke"])
def test_evolve_xy_matches_dense(kind, order, init):
    n, k, p = 5, 2, 3
    rng = np.random.default_rng(17)
    c = rng.integers(-4, 5, size=1 << n).astype(np.float64)
    g, b = rng.uniform(-1, 1, p), rng.uniform(-np.pi, np.pi, p)
    psi = np.full(1 << n, 2 ** (-n / 2), dtype=np.complex128)
    if init == "dicke":
        w = np.array([bin(x).count("1") for x in range(1 << n)])
        psi = (w == k) / math.sqrt(math.comb(n, k)) + 0j
    for l in range(p):
        psi = xy_layer_dense(n, order(n), b[l]) @ (np.exp(-1j * g[l] * c) * psi)
    got = oracle.evolve_xy(n, c, g, b, kind, init=init, k=k)
    assert np.max(np.abs(got - psi)) < 1e-12
