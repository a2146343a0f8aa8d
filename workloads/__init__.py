"""Seeded synthetic problem instances and parameter schedules.

This module is shared by the CPU oracle and by the GPU path as their common
source of inputs.  It builds problem descriptions (weighted spin terms, graphs)
and QAOA parameter vectors; it performs none of the simulation arithmetic
(no cost-vector evaluation, no state evolution, no expectation values).

Term format (Eq. (1) of the paper): a list of ``(w, idx)`` pairs, where ``w`` is
a real weight and ``idx`` a tuple of 0-based variable indices; the empty tuple
is the constant offset.  Variable ``i`` is bit ``i`` of the basis-state index.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "labs_terms",
    "maxcut_terms",
    "random_regular_graph",
    "erdos_renyi_graph",
    "linear_ramp",
    "uniform_angles",
    "random_terms",
    "terms_to_csr",
    "C1", "C2A", "C2B", "C3", "C4",
]


# ---------------------------------------------------------------------------
# Problems
# ---------------------------------------------------------------------------

def labs_terms(n: int):
    """LABS cost ``sum_{k=1}^{n-1} C_k^2`` with ``C_k = sum_i s_i s_{i+k}`` as spin terms.

    Section 2 (Background) writes the LABS objective as a 4-body sum over index
    sets ``{i, i+t, i+k, i+k+t}`` (1 <= t < k) with factor 2 plus a 2-body sum
    over pairs ``{i, i+2k}``.  That polynomial equals
    ``(sum_k C_k^2 - n(n-1)/2) / 2``, so the squared-autocorrelation form used
    here has 4-body weight 4, 2-body weight 2 and constant ``n(n-1)/2``.
    Indices are 0-based.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    terms = []
    # 4-body: i + t < i + k < i + k + t <= n - 1, t >= 1, k >= t + 1
    for i in range(n):
        for t in range(1, n):
            for k in range(t + 1, n):
                if i + k + t > n - 1:
                    break
                terms.append((4.0, (i, i + t, i + k, i + k + t)))
    # 2-body: (i, i + 2k)
    for i in range(n):
        for k in range(1, n):
            if i + 2 * k > n - 1:
                break
            terms.append((2.0, (i, i + 2 * k)))
    terms.append((float(n * (n - 1) // 2), ()))
    return terms


def maxcut_terms(edges, weights=None):
    """Weighted MaxCut in minimisation form, ``c(x) = -cut_w(x)``.

    Section 2 gives the unweighted form ``sum_{(i,j) in E} s_i s_j / 2 - |E|/2``;
    with edge weights every edge contributes ``w/2 * s_i s_j`` and the constant
    is ``-sum(w)/2``.
    """
    edges = [(int(u), int(v)) for u, v in edges]
    if weights is None:
        weights = [1.0] * len(edges)
    terms = [(0.5 * float(w), (u, v)) for (u, v), w in zip(edges, weights)]
    terms.append((-0.5 * float(sum(weights)), ()))
    return terms


def random_regular_graph(d: int, n: int, seed: int):
    """Uniformly paired random d-regular simple graph (configuration model with
    rejection of self-loops and multi-edges).  Returns a sorted edge list."""
    if (d * n) % 2 or d >= n:
        raise ValueError("need d*n even and d < n")
    rng = np.random.default_rng(seed)
    for _ in range(10000):
        stubs = np.repeat(np.arange(n), d)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        e = {tuple(sorted(map(int, p))) for p in pairs}
        if len(e) != len(pairs):
            continue
        return sorted(e)
    raise RuntimeError("failed to draw a simple regular graph")


def erdos_renyi_graph(n: int, prob: float, seed: int, wmin: int = 1, wmax: int = 10):
    """G(n, prob) with integer edge weights uniform in {wmin..wmax}."""
    rng = np.random.default_rng(seed)
    edges, weights = [], []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < prob:
                edges.append((i, j))
                weights.append(int(rng.integers(wmin, wmax + 1)))
    return edges, weights


def random_terms(n: int, num_terms: int, seed: int, max_order: int = 4,
                 integer: bool = True, wmax: int = 5):
    """Random spin polynomial with terms of order 0..max_order (repeated
    indices allowed, to exercise cancellation ``s_i^2 = 1``)."""
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(num_terms):
        order = int(rng.integers(0, max_order + 1))
        idx = tuple(int(v) for v in rng.integers(0, n, size=order))
        if integer:
            w = float(rng.integers(-wmax, wmax + 1))
        else:
            w = float(rng.uniform(-wmax, wmax))
        terms.append((w, idx))
    return terms


def terms_to_csr(terms):
    """Flatten ``[(w, idx), ...]`` to ``(w[L] f64, ptr[L+1] i64, idx[nnz] i32)``."""
    w = np.array([float(t[0]) for t in terms], dtype=np.float64)
    ptr = np.zeros(len(terms) + 1, dtype=np.int64)
    flat = []
    for k, (_, idx) in enumerate(terms):
        flat.extend(int(i) for i in idx)
        ptr[k + 1] = len(flat)
    return w, ptr, np.array(flat, dtype=np.int32)


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------

def linear_ramp(p: int, seed: int, noise: float = 0.0):
    """Linear-ramp schedule ``gamma_l = dg (l - 1/2)/p``,
    ``beta_l = db (1 - (l - 1/2)/p)``, with ``(dg, db) ~ U(0.1, 1.0)^2`` drawn
    from ``default_rng(seed)``; optional N(0, noise) perturbation."""
    rng = np.random.default_rng(seed)
    dg, db = rng.uniform(0.1, 1.0, size=2)
    l = np.arange(1, p + 1, dtype=np.float64)
    gamma = dg * (l - 0.5) / p
    beta = db * (1.0 - (l - 0.5) / p)
    if noise:
        gamma = gamma + rng.normal(0.0, noise, size=p)
        beta = beta + rng.normal(0.0, noise, size=p)
    return gamma, beta


def uniform_angles(p: int, seed: int, batch: int | None = None):
    """gamma, beta ~ U(0, pi); shape (p,) or (batch, p)."""
    rng = np.random.default_rng(seed)
    shape = (p,) if batch is None else (batch, p)
    gamma = rng.uniform(0.0, np.pi, size=shape)
    beta = rng.uniform(0.0, np.pi, size=shape)
    return gamma, beta


# ---------------------------------------------------------------------------
# Named workloads (sizes of the paper's experiments)
# ---------------------------------------------------------------------------

def C1():
    """MaxCut, random 3-regular graph, n=12, unit weights, p=1, complex128."""
    n = 12
    edges = random_regular_graph(3, n, seed=0)
    gamma, beta = uniform_angles(1, seed=1)
    return dict(name="maxcut3reg_n12_p1_c128", n=n, p=1, dtype="complex128",
                edges=edges, terms=maxcut_terms(edges), gamma=gamma, beta=beta)


def C2A():
    """LABS n=26, p=10, linear ramp, complex128."""
    n, p = 26, 10
    gamma, beta = linear_ramp(p, seed=2)
    return dict(name="labs_n26_p10_c128", n=n, p=p, dtype="complex128",
                terms=labs_terms(n), gamma=gamma, beta=beta)


def C2B():
    """LABS n=31, p=10, linear ramp, complex64."""
    n, p = 31, 10
    gamma, beta = linear_ramp(p, seed=3)
    return dict(name="labs_n31_p10_c64", n=n, p=p, dtype="complex64",
                terms=labs_terms(n), gamma=gamma, beta=beta)


def C3(batch: int = 512):
    """Weighted MaxCut on G(22, 0.3), integer weights U{1..10}, p=6, many
    (gamma, beta) sets ~ U(0, pi), complex64."""
    n, p = 22, 6
    edges, weights = erdos_renyi_graph(n, 0.3, seed=4)
    gamma, beta = uniform_angles(p, seed=5, batch=batch)
    return dict(name="maxcut_er22_p6_c64", n=n, p=p, dtype="complex64",
                edges=edges, weights=weights, terms=maxcut_terms(edges, weights),
                gamma=gamma, beta=beta)


def C4():
    """LABS n=24, p=20, ramp plus N(0, 0.05) noise, complex128 (gradient)."""
    n, p = 24, 20
    gamma, beta = linear_ramp(p, seed=6, noise=0.05)
    return dict(name="labs_n24_p20_c128", n=n, p=p, dtype="complex128",
                terms=labs_terms(n), gamma=gamma, beta=beta)
