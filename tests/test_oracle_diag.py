"""Pins for the oracle's cost vectors (CPU).

Each check ties the oracle to something other than itself: a second,
independent formulation (direct definition vs term expansion), closed forms,
textbook values (Barker codes, small-graph max cuts) and brute force.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _bits_from_spins(spins):
    return sum((1 << i) for i, s in enumerate(spins) if s == -1)


@pytest.mark.parametrize("n", list(range(2, 15)))
def test_labs_direct_equals_term_expansion(n):
    # Section 2: the 4-body/2-body polynomial (rescaled) == sum_k C_k^2, bit-exact
    direct = oracle.diag_labs(n)
    terms = oracle.diag_terms(n, W.labs_terms(n))
    assert np.array_equal(direct.astype(np.float64), terms)


@pytest.mark.parametrize("n", [3, 6, 9, 12])
def test_labs_closed_forms(n):
    c = oracle.diag_labs(n)
    N = 1 << n
    # all-equal sequences: every C_k = n - k
    top = sum((n - k) ** 2 for k in range(1, n))
    assert c[0] == top and c[N - 1] == top and c.max() == top
    # mean over x: E[C_k^2] = n - k (independent +-1 products), so mean = n(n-1)/2
    assert c.sum() == N * n * (n - 1) // 2
    # symmetries: global flip, reversal, alternating flip s_i -> (-1)^i s_i
    x = np.arange(N)
    flip = x ^ (N - 1)
    rev = np.zeros(N, dtype=np.int64)
    for i in range(n):
        rev |= ((x >> i) & 1) << (n - 1 - i)
    alt = x ^ sum(1 << i for i in range(1, n, 2))
    assert np.array_equal(c, c[flip])
    assert np.array_equal(c, c[rev])
    assert np.array_equal(c, c[alt])
    # parity: C_k = n - k (mod 2) so c = n(n-1)/2 (mod 2) for every x
    assert np.all(c % 2 == (n * (n - 1) // 2) % 2)


@pytest.mark.parametrize("n", [2, 5, 9, 14])
def test_labs_at_equals_full_vector(n):
    # the sampled entry point returns the full vector's entries, in any order
    rng = np.random.default_rng(n)
    xs = np.concatenate([np.arange(1 << n), rng.integers(0, 1 << n, size=257)])
    assert np.array_equal(oracle.diag_labs_at(n, xs), oracle.diag_labs(n)[xs])


@pytest.mark.parametrize("n", [26, 31, 33])
def test_labs_at_against_numpy_autocorrelation(n):
    # sizes used by the full-size GPU checks: C_k from numpy's correlate of the
    # spin sequence (a library routine), including indices at and above 2^32
    rng = np.random.default_rng(1000 + n)
    xs = np.concatenate([[0, (1 << n) - 1, (1 << n) // 3, (1 << (n - 1)) | 1],
                         rng.integers(0, 1 << n, size=200)])
    if n > 32:
        xs = np.concatenate([xs, [1 << 32, (1 << 32) - 1, (1 << 32) + 12345]])
    got = oracle.diag_labs_at(n, xs)
    for x, e in zip(xs.tolist(), got.tolist()):
        s = np.array([1 - 2 * ((x >> i) & 1) for i in range(n)], dtype=np.int64)
        ac = np.correlate(s, s, mode="full")[n:]          # C_1 .. C_{n-1}
        assert int(np.sum(ac * ac)) == e, x


def test_labs_barker_golden():
    d = json.load(open(os.path.join(GOLD, "labs_barker.json")))
    for case in d["cases"]:
        n = case["n"]
        c = oracle.diag_labs(n)
        x = _bits_from_spins(case["spins"])
        assert c[x] == case["energy"], case
        # Barker sequences are optimal: brute-force minimum equals their energy
        assert c.min() == case["energy"], case


def test_labs_term_count_matches_paper():
    # Section 6 (related work): at n=31 the LABS cost has about 75n terms.
    t = W.labs_terms(31)
    nonconst = [x for x in t if len(x[1]) > 0]
    assert abs(len(nonconst) / 31.0 - 75.0) < 0.05 * 75.0
    assert len(nonconst) == 2360


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_maxcut_direct_equals_terms(seed):
    rng = np.random.default_rng(seed)
    n = 9
    edges, weights = W.erdos_renyi_graph(n, 0.5, seed=seed)
    direct = oracle.diag_maxcut(n, edges, weights)
    terms = oracle.diag_terms(n, W.maxcut_terms(edges, weights))
    assert np.array_equal(direct, terms)
    assert direct[0] == 0.0
    assert np.array_equal(direct, direct[np.arange(1 << n) ^ ((1 << n) - 1)])
    del rng


def test_maxcut_golden_graphs():
    d = json.load(open(os.path.join(GOLD, "maxcut_small_graphs.json")))
    for case in d["cases"]:
        c = oracle.diag_maxcut(case["n"], case["edges"])
        assert -c.min() == case["maxcut"], case["name"]
        assert oracle.diag_terms(case["n"], W.maxcut_terms(case["edges"])).min() == -case["maxcut"]


def test_terms_repeated_indices_cancel():
    # s_i^2 = 1: (w, (i, i, j)) is the same function as (w, (j,))
    n = 5
    a = oracle.diag_terms(n, [(3.0, (1, 1, 4)), (2.0, (0, 2, 0, 2))])
    b = oracle.diag_terms(n, [(3.0, (4,)), (2.0, ())])
    assert np.array_equal(a, b)


def test_spin_convention_odd_term():
    # reading of the bijection: s_i = +1 for bit 0, -1 for bit 1
    c = oracle.diag_terms(3, [(1.0, (0,)), (10.0, (2,))])
    x = np.arange(8)
    expect = np.where(x & 1, -1.0, 1.0) + 10.0 * np.where(x & 4, -1.0, 1.0)
    assert np.array_equal(c, expect)


def test_empty_term_is_offset_and_zero_weights():
    c = oracle.diag_terms(4, [(7.5, ())])
    assert np.all(c == 7.5)
    z = oracle.diag_terms(4, [(0.0, (0, 1)), (0.0, (2,))])
    assert np.all(z == 0.0)


def test_brute_force_tiny_terms():
    # brute force over x with Python integers, n = 4, random odd/even terms
    n = 4
    terms = W.random_terms(n, 12, seed=11)
    c = oracle.diag_terms(n, terms)
    for x in range(1 << n):
        tot = 0.0
        for w, idx in terms:
            v = w
            for i in idx:
                v *= -1.0 if (x >> i) & 1 else 1.0
            tot += v
        assert c[x] == tot
