"""Python face of the request loop (qaoa_server_* in include/qaoa.h).

    srv = QAOAServer(arena_bytes=8 << 30, num_streams=4, max_in_flight=16)
    pid = srv.add_problem(n, terms)                   # cost vector stays resident
    t = srv.submit(pid, gamma, beta, gradient=False)  # returns a ticket at once
    result, latency_s = srv.wait(t)                   # (E, norm) or (E, dgamma, dbeta)

Marshalling only: admission, scheduling and execution run in the library.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib

_lib.lib.qaoa_server_create.restype = ctypes.c_int
_lib.lib.qaoa_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
_lib.lib.qaoa_server_destroy.restype = ctypes.c_int
_lib.lib.qaoa_server_destroy.argtypes = [ctypes.c_void_p]
_lib.lib.qaoa_server_add_problem.restype = ctypes.c_int
_lib.lib.qaoa_server_add_problem.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int)]
_lib.lib.qaoa_server_submit.restype = ctypes.c_int
_lib.lib.qaoa_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
_lib.lib.qaoa_server_wait.restype = ctypes.c_int
_lib.lib.qaoa_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_double)]
_lib.lib.qaoa_server_reset_stats.restype = ctypes.c_int
_lib.lib.qaoa_server_reset_stats.argtypes = [ctypes.c_void_p]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("in_flight", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64), ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("mean_s", ctypes.c_double), ("max_s", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("requests_per_s", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib.lib.qaoa_server_stats_get.restype = ctypes.c_int
_lib.lib.qaoa_server_stats_get.argtypes = [ctypes.c_void_p, ctypes.POINTER(ServerStats)]

_STATE = {"complex64": _lib.QAOA_C64, "complex128": _lib.QAOA_C128}


class QAOAServer:
    def __init__(self, arena_bytes: int, num_streams: int = 4, max_in_flight: int = 16):
        h = ctypes.c_void_p()
        _lib.check(_lib.lib.qaoa_server_create(int(arena_bytes), int(num_streams), int(max_in_flight),
                                               ctypes.byref(h)))
        self._h = h
        self._p = {}

    def close(self):
        if self._h:
            _lib.check(_lib.lib.qaoa_server_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_problem(self, n: int, terms, diag_dtype: str = "i32") -> int:
        w = np.ascontiguousarray([float(t[0]) for t in terms], dtype=np.float64)
        ptr = np.zeros(len(terms) + 1, dtype=np.int64)
        flat = []
        for k, (_, idx) in enumerate(terms):
            flat.extend(int(i) for i in idx)
            ptr[k + 1] = len(flat)
        idx = np.ascontiguousarray(flat if flat else [0], dtype=np.int32)
        pid = ctypes.c_int(-1)
        _lib.check(_lib.lib.qaoa_server_add_problem(self._h, n, len(terms), w.ctypes.data, ptr.ctypes.data,
                                                    idx.ctypes.data if flat else None, _lib.DIAG_NAMES[diag_dtype],
                                                    ctypes.byref(pid)))
        self._p[pid.value] = n
        return pid.value

    def submit(self, problem: int, gamma, beta, gradient: bool = False, dtype: str = "complex64") -> int:
        g = np.ascontiguousarray(np.atleast_1d(gamma), dtype=np.float64)
        b = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
        if g.shape != b.shape:
            raise ValueError("gamma and beta differ in length")
        t = ctypes.c_int64(0)
        _lib.check(_lib.lib.qaoa_server_submit(self._h, int(problem), 1 if gradient else 0, _STATE[dtype], len(g),
                                               g.ctypes.data, b.ctypes.data, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, max_p: int = 256):
        out = np.zeros(1 + 2 * max_p, dtype=np.float64)
        lat = ctypes.c_double(0.0)
        _lib.check(_lib.lib.qaoa_server_wait(self._h, int(ticket), out.ctypes.data, len(out), ctypes.byref(lat)))
        return out, lat.value

    def stats(self) -> dict:
        st = ServerStats()
        _lib.check(_lib.lib.qaoa_server_stats_get(self._h, ctypes.byref(st)))
        return st.as_dict()

    def reset_stats(self) -> None:
        _lib.check(_lib.lib.qaoa_server_reset_stats(self._h))
