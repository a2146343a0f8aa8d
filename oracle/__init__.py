"""FP64 CPU oracle for the QAOA hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it, and
it shares no code with the GPU path: the arithmetic lives in ``oracle.c``
(plain C, double precision, written from the paper's definitions), built with
gcc into ``liboracle.so`` and called here through ctypes.

Functions and the passages they follow:
  diag_terms      Eq. (1): spin polynomial, term by term
  diag_labs       Section 2, LABS: sum_k C_k^2 (direct autocorrelation form)
  diag_labs_at    the same at selected basis states (sampled checks)
  diag_maxcut     Section 2, MaxCut: minus the (weighted) cut
  evolve          Algorithm 3 with Section 3.2's gate exp(-i beta X) per qubit
  expectation     Section 3.1: E = sum |psi|^2 c (compensated), plus sum |psi|^2
  grad            dE/dgamma, dE/dbeta by the adjoint method (reverse Algorithm 3)
All functions are pinned by tests against closed forms, library routines,
brute force and invariants (see tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (IEEE double, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_diag_terms.argtypes = [ctypes.c_int, i64, P, P, P, P]
    lib.oracle_diag_labs.argtypes = [ctypes.c_int, P]
    lib.oracle_diag_labs_at.argtypes = [ctypes.c_int, i64, P, P]
    lib.oracle_diag_maxcut.argtypes = [ctypes.c_int, i64, P, P, P]
    lib.oracle_plus_state.argtypes = [ctypes.c_int, P]
    lib.oracle_apply_phase.argtypes = [ctypes.c_int, P, ctypes.c_double, P]
    lib.oracle_apply_rx.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, P]
    lib.oracle_apply_mixer.argtypes = [ctypes.c_int, ctypes.c_double, P]
    lib.oracle_qaoa_evolve.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P]
    lib.oracle_expectation.argtypes = [ctypes.c_int, P, P, P]
    lib.oracle_qaoa_grad.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    lib.oracle_apply_xy.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, P]
    lib.oracle_xy_edges.argtypes = [ctypes.c_int, ctypes.c_int, P]
    lib.oracle_xy_edges.restype = ctypes.c_int
    lib.oracle_apply_xy_mixer.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, P]
    lib.oracle_dicke_state.argtypes = [ctypes.c_int, ctypes.c_int, P]
    lib.oracle_qaoa_evolve_xy.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    """Threads for the parallel loops (results do not depend on it)."""
    _load().oracle_set_num_threads(int(t))


def diag_terms(n: int, terms) -> np.ndarray:
    """Cost vector from Eq. (1) terms ``[(w, idx), ...]`` (0-based), float64[2^n]."""
    w = np.ascontiguousarray([float(t[0]) for t in terms], dtype=np.float64)
    ptr = np.zeros(len(terms) + 1, dtype=np.int64)
    flat = []
    for k, (_, idx) in enumerate(terms):
        for i in idx:
            if not 0 <= int(i) < n:
                raise ValueError(f"term index {i} out of range for n={n}")
            flat.append(int(i))
        ptr[k + 1] = len(flat)
    idx = np.ascontiguousarray(flat if flat else [0], dtype=np.int32)
    c = np.empty(1 << n, dtype=np.float64)
    _load().oracle_diag_terms(n, len(terms), _ptr(w), _ptr(ptr), _ptr(idx), _ptr(c))
    return c


def diag_labs(n: int) -> np.ndarray:
    """LABS cost sum_k C_k^2 for every basis state, int64[2^n]."""
    c = np.empty(1 << n, dtype=np.int64)
    _load().oracle_diag_labs(n, _ptr(c))
    return c


def diag_labs_at(n: int, xs) -> np.ndarray:
    """LABS cost at the given basis states only, int64."""
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    out = np.empty(len(xs), dtype=np.int64)
    _load().oracle_diag_labs_at(n, len(xs), _ptr(xs), _ptr(out))
    return out


def diag_maxcut(n: int, edges, weights=None) -> np.ndarray:
    """Minus the weighted cut for every basis state, float64[2^n]."""
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    if weights is None:
        weights = np.ones(len(e))
    w = np.ascontiguousarray(weights, dtype=np.float64)
    c = np.empty(1 << n, dtype=np.float64)
    _load().oracle_diag_maxcut(n, len(e), _ptr(e), _ptr(w), _ptr(c))
    return c


def evolve(n: int, c, gamma, beta, psi0=None) -> np.ndarray:
    """QAOA state (Algorithm 3).  ``psi0=None`` starts from |+>^n.
    Returns complex128[2^n]."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    g = np.ascontiguousarray(np.atleast_1d(gamma), dtype=np.float64)
    b = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
    if g.shape != b.shape or c.shape != (1 << n,):
        raise ValueError("shape mismatch")
    psi = np.empty(1 << n, dtype=np.complex128)
    if psi0 is not None:
        psi[:] = psi0
    _load().oracle_qaoa_evolve(n, len(g), _ptr(c), _ptr(g), _ptr(b),
                               1 if psi0 is None else 0, _ptr(psi.view(np.float64)))
    return psi


def evolve_inplace(n: int, c: np.ndarray, gamma, beta, psi: np.ndarray, init: bool) -> None:
    """Algorithm 3 on ``psi`` (complex128[2^n], C-contiguous) in place, without
    the copies ``evolve`` makes; ``init`` starts from |+>^n.  For states too
    large to hold twice in host memory."""
    g = np.ascontiguousarray(np.atleast_1d(gamma), dtype=np.float64)
    b = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
    if (g.shape != b.shape or c.dtype != np.float64 or c.shape != (1 << n,) or psi.dtype != np.complex128
            or psi.shape != (1 << n,)):
        raise ValueError("shape or dtype mismatch")
    _load().oracle_qaoa_evolve(n, len(g), _ptr(c), _ptr(g), _ptr(b), 1 if init else 0,
                               _ptr(psi.view(np.float64)))


def apply_phase(n: int, c, gamma: float, psi: np.ndarray) -> np.ndarray:
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    _load().oracle_apply_phase(n, _ptr(np.ascontiguousarray(c, dtype=np.float64)),
                               float(gamma), _ptr(out.view(np.float64)))
    return out


def apply_mixer(n: int, beta: float, psi: np.ndarray) -> np.ndarray:
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    _load().oracle_apply_mixer(n, float(beta), _ptr(out.view(np.float64)))
    return out


def expectation(n: int, psi, c):
    """(E, sum |psi|^2) with compensated FP64 summation."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(2, dtype=np.float64)
    _load().oracle_expectation(n, _ptr(psi.view(np.float64)), _ptr(c), _ptr(out))
    return float(out[0]), float(out[1])


def qaoa_expectation(n: int, c, gamma, beta) -> float:
    """Convenience: E after p layers from |+>^n."""
    return expectation(n, evolve(n, c, gamma, beta), c)[0]


def apply_rx(n: int, q: int, beta: float, psi: np.ndarray) -> np.ndarray:
    """One mixer gate exp(-i beta X_q) on a copy of psi."""
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    _load().oracle_apply_rx(n, int(q), float(beta), _ptr(out.view(np.float64)))
    return out


def grad(n: int, c, gamma, beta):
    """(E, dE/dgamma[p], dE/dbeta[p]) from |+>^n, adjoint method, FP64."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    g = np.ascontiguousarray(np.atleast_1d(gamma), dtype=np.float64)
    b = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
    p = len(g)
    out = np.zeros(1 + 2 * p, dtype=np.float64)
    work = np.empty(4 << n, dtype=np.float64)
    _load().oracle_qaoa_grad(n, p, _ptr(c), _ptr(g), _ptr(b), _ptr(out), _ptr(work))
    return float(out[0]), out[1:1 + p].copy(), out[1 + p:].copy()


XY_RING, XY_COMPLETE = 1, 2


def xy_edges(n: int, kind: int) -> list:
    """Edges of one XY mixer layer in application order (ring: even, odd, wrap;
    complete: lexicographic)."""
    e = np.zeros(2 * n * n + 2, dtype=np.int32)
    m = _load().oracle_xy_edges(n, kind, _ptr(e))
    return [(int(e[2 * i]), int(e[2 * i + 1])) for i in range(m)]


def apply_xy(n: int, i: int, j: int, beta: float, psi: np.ndarray) -> np.ndarray:
    """exp(-i beta (X_i X_j + Y_i Y_j)/2) on a copy of psi."""
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    _load().oracle_apply_xy(n, int(i), int(j), float(beta), _ptr(out.view(np.float64)))
    return out


def apply_xy_mixer(n: int, kind: int, beta: float, psi: np.ndarray) -> np.ndarray:
    out = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    _load().oracle_apply_xy_mixer(n, int(kind), float(beta), _ptr(out.view(np.float64)))
    return out


def dicke_state(n: int, k: int) -> np.ndarray:
    out = np.empty(1 << n, dtype=np.complex128)
    _load().oracle_dicke_state(n, int(k), _ptr(out.view(np.float64)))
    return out


def evolve_xy(n: int, c, gamma, beta, kind: int, init: str = "plus", k: int = 0, psi0=None) -> np.ndarray:
    """QAOA state with an XY mixer; init "plus" (|+>^n), "dicke" (|D^n_k>) or
    "given" (psi0)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    g = np.ascontiguousarray(np.atleast_1d(gamma), dtype=np.float64)
    b = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
    if g.shape != b.shape or c.shape != (1 << n,):
        raise ValueError("shape mismatch")
    psi = np.zeros(1 << n, dtype=np.complex128)
    code = {"given": 0, "plus": 1, "dicke": 2}[init]
    if code == 0:
        psi[:] = psi0
    _load().oracle_qaoa_evolve_xy(n, len(g), _ptr(c), _ptr(g), _ptr(b), int(kind), code, int(k),
                                  _ptr(psi.view(np.float64)))
    return psi
