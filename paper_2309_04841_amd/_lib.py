"""ctypes binding of libqaoa.so (include/qaoa.h).

Argument marshalling only: torch tensors supply device pointers and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  If the library is not built the import of this module fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqaoa.so")

QAOA_OK, QAOA_ERR_INVALID, QAOA_ERR_RANGE, QAOA_ERR_NOMEM, QAOA_ERR_DEVICE, QAOA_ERR_UNSUPPORTED = range(6)
QAOA_C64, QAOA_C128 = 0, 1
QAOA_DIAG_F64, QAOA_DIAG_I32, QAOA_DIAG_U16 = 0, 1, 2
QAOA_OP_PRECOMPUTE, QAOA_OP_EVOLVE, QAOA_OP_EXPECTATION, QAOA_OP_GRAD = range(4)
QAOA_MAX_QUBITS = 34
QAOA_NOALLOC_SCRATCH_BYTES = 9 << 20

EXPORTS = ("qaoa_version", "qaoa_last_error", "qaoa_workspace_bytes", "qaoa_precompute_diag",
           "qaoa_evolve", "qaoa_expectation", "qaoa_grad", "qaoa_plan_describe", "qaoa_evolve_batch",
           "qaoa_batch_workspace_bytes", "qaoa_grad_workspace_bytes", "qaoa_server_create",
           "qaoa_server_destroy", "qaoa_server_add_problem", "qaoa_server_submit", "qaoa_server_wait",
           "qaoa_server_stats_get", "qaoa_server_reset_stats", "qaoa_schedule_describe", "qaoa_set_tuning",
           "qaoa_get_tuning", "qaoa_evolve_xy", "qaoa_xy_workspace_bytes", "qaoa_xy_plan_describe",
           "qaoa_evolve_noalloc")

_STATUS_NAMES = {0: "QAOA_OK", 1: "QAOA_ERR_INVALID", 2: "QAOA_ERR_RANGE", 3: "QAOA_ERR_NOMEM",
                 4: "QAOA_ERR_DEVICE", 5: "QAOA_ERR_UNSUPPORTED"}


class QaoaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2309_04841_amd/build.py` "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I, I64, SZ = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    lib.qaoa_version.restype = ctypes.c_char_p
    lib.qaoa_version.argtypes = []
    lib.qaoa_last_error.restype = ctypes.c_char_p
    lib.qaoa_last_error.argtypes = []
    lib.qaoa_workspace_bytes.restype = I
    lib.qaoa_workspace_bytes.argtypes = [I, I, I, I, ctypes.POINTER(SZ)]
    lib.qaoa_precompute_diag.restype = I
    lib.qaoa_precompute_diag.argtypes = [I, I64, P, P, P, I, P, SZ, ctypes.POINTER(D), P, SZ, P]
    lib.qaoa_evolve.restype = I
    lib.qaoa_evolve.argtypes = [I, I, P, P, P, I, D, SZ, P, I, SZ, I, P, P, SZ, P]
    lib.qaoa_evolve_noalloc.restype = I
    lib.qaoa_evolve_noalloc.argtypes = [I, I, P, P, P, I, D, SZ, P, I, SZ, I, P, P]
    lib.qaoa_expectation.restype = I
    lib.qaoa_expectation.argtypes = [I, P, I, SZ, P, I, D, SZ, P, P, SZ, P]
    lib.qaoa_grad.restype = I
    lib.qaoa_grad.argtypes = [I, I, P, P, P, I, D, SZ, P, P, I, SZ, P, P, SZ, P]
    lib.qaoa_plan_describe.restype = I
    lib.qaoa_plan_describe.argtypes = [I, I, I, I, P, I]
    lib.qaoa_set_tuning.restype = I
    lib.qaoa_set_tuning.argtypes = [I, I]
    lib.qaoa_get_tuning.restype = I
    lib.qaoa_get_tuning.argtypes = [I, ctypes.POINTER(I)]
    lib.qaoa_schedule_describe.restype = I
    lib.qaoa_schedule_describe.argtypes = [I, I, I, I, I, I, P, I]
    lib.qaoa_grad_workspace_bytes.restype = I
    lib.qaoa_grad_workspace_bytes.argtypes = [I, I, I, I, ctypes.POINTER(SZ)]
    lib.qaoa_evolve_batch.restype = I
    lib.qaoa_evolve_batch.argtypes = [I, I, I, P, P, P, I, D, SZ, P, I, SZ, I, P, I, P, SZ, P]
    lib.qaoa_batch_workspace_bytes.restype = I
    lib.qaoa_batch_workspace_bytes.argtypes = [I, I, I, I, I, ctypes.POINTER(SZ)]
    lib.qaoa_evolve_xy.restype = I
    lib.qaoa_evolve_xy.argtypes = [I, I, P, P, I, P, I, D, SZ, P, I, SZ, I, I, P, P, SZ, P]
    lib.qaoa_xy_workspace_bytes.restype = I
    lib.qaoa_xy_workspace_bytes.argtypes = [I, I, I, ctypes.POINTER(SZ)]
    lib.qaoa_xy_plan_describe.restype = I
    lib.qaoa_xy_plan_describe.argtypes = [I, I, I, P, I]
    return lib


lib = _load()


def check(status: int) -> None:
    if status != QAOA_OK:
        raise QaoaError(status, lib.qaoa_last_error().decode())


def version() -> str:
    return lib.qaoa_version().decode()


# --------------------------------------------------------------------------
# dtype helpers
# --------------------------------------------------------------------------
_STATE_DT = {torch.complex64: QAOA_C64, torch.complex128: QAOA_C128}
_DIAG_DT = {torch.float64: QAOA_DIAG_F64, torch.int32: QAOA_DIAG_I32, torch.uint16: QAOA_DIAG_U16}
_DIAG_TORCH = {QAOA_DIAG_F64: torch.float64, QAOA_DIAG_I32: torch.int32, QAOA_DIAG_U16: torch.uint16}
DIAG_NAMES = {"f64": QAOA_DIAG_F64, "i32": QAOA_DIAG_I32, "u16": QAOA_DIAG_U16}


def state_dtype_code(t: torch.Tensor) -> int:
    try:
        return _STATE_DT[t.dtype]
    except KeyError:
        raise TypeError(f"state must be complex64 or complex128, got {t.dtype}") from None


def diag_dtype_code(t: torch.Tensor) -> int:
    try:
        return _DIAG_DT[t.dtype]
    except KeyError:
        raise TypeError(f"cost vector must be float64, int32 or uint16, got {t.dtype}") from None


def _dev_ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _f64(values) -> ctypes.Array:
    vals = [float(v) for v in values]
    return (ctypes.c_double * max(1, len(vals)))(*vals)


PLAN_EVOLVE, PLAN_ADJOINT, PLAN_TRANSFORM = 0, 1, 2


def plan_describe(n: int, state_dtype: int = QAOA_C128, elem_bytes: int = 0, kind: int | None = None) -> dict:
    """The sweep plan as a dict: {'eb', 'single', 'wide', 'sweeps': [{'tb','R','hA','qA','qB','act_lo','w_store','chunks'}]}.
    kind: PLAN_EVOLVE (default), PLAN_ADJOINT, or PLAN_TRANSFORM (elem_bytes)."""
    if kind is None:
        kind = PLAN_TRANSFORM if state_dtype < 0 else PLAN_EVOLVE
    need = lib.qaoa_plan_describe(kind, n, state_dtype, elem_bytes, None, 0)
    if need < 0:
        check(-need)
    buf = (ctypes.c_int * need)()
    lib.qaoa_plan_describe(kind, n, state_dtype, elem_bytes, buf, need)
    v = list(buf)
    ns, eb, single, wide = v[0], v[1], v[2], v[3]
    i = 4
    sweeps = []
    for _ in range(ns):
        tb, R, hA, qA, qB, act_lo, ws, nc = v[i:i + 8]
        i += 8
        chunks = [tuple(v[i + 3 * c:i + 3 * c + 3]) for c in range(nc)]
        i += 3 * nc
        sweeps.append(dict(tb=tb, R=R, hA=hA, qA=qA, qB=qB, act_lo=act_lo, w_store=ws, chunks=chunks))
    return dict(eb=eb, single=bool(single), wide=bool(wide), sweeps=sweeps)


F_INIT, F_PHASE, F_EXPV, F_FUSE = 1, 2, 4, 8

MIXER_X, MIXER_XY_RING, MIXER_XY_COMPLETE = 0, 1, 2
INIT_GIVEN, INIT_PLUS, INIT_DICKE = 0, 1, 2
MIXER_NAMES = {"x": MIXER_X, "xy_ring": MIXER_XY_RING, "xy_complete": MIXER_XY_COMPLETE}


def xy_plan_describe(n: int, mixer: int, state_dtype: int = QAOA_C128) -> dict:
    """The XY sweep plan: {'eb', 'single', 'sweeps': [{'tb','R','hA','qA','qB','gates': [(i, j), ...]}]}
    with gates as tile-bit pairs, in the order they are applied."""
    need = lib.qaoa_xy_plan_describe(n, mixer, state_dtype, None, 0)
    if need < 0:
        check(-need)
    buf = (ctypes.c_int * need)()
    lib.qaoa_xy_plan_describe(n, mixer, state_dtype, buf, need)
    v = list(buf)
    ns, eb, single = v[0], v[1], v[2]
    i = 3
    sweeps = []
    for _ in range(ns):
        tb, R, hA, qA, qB, ng = v[i:i + 6]
        i += 6
        gates = [(v[i + 2 * e], v[i + 2 * e + 1]) for e in range(ng)]
        i += 2 * ng
        sweeps.append(dict(tb=tb, R=R, hA=hA, qA=qA, qB=qB, gates=gates))
    return dict(eb=eb, single=bool(single), sweeps=sweeps)


TUNE_WIDE_TILES, TUNE_FUSE_LAYERS = 0, 1


def set_tuning(knob: int, value: int) -> None:
    check(lib.qaoa_set_tuning(knob, int(value)))


def get_tuning(knob: int) -> int:
    v = ctypes.c_int(0)
    check(lib.qaoa_get_tuning(knob, ctypes.byref(v)))
    return int(v.value)


class tuning:
    """Context manager: `with tuning(wide_tiles=0, fuse_layers=0): ...` restores the previous values."""

    def __init__(self, wide_tiles: int | None = None, fuse_layers: int | None = None):
        self._want = {TUNE_WIDE_TILES: wide_tiles, TUNE_FUSE_LAYERS: fuse_layers}
        self._saved = {}

    def __enter__(self):
        for k, v in self._want.items():
            if v is not None:
                self._saved[k] = get_tuning(k)
                set_tuning(k, v)
        return self

    def __exit__(self, *exc):
        for k, v in self._saved.items():
            set_tuning(k, v)
        return False


A_FIRST, A_PHASE, A_FUSE = 1, 2, 8
SCHED_EVOLVE, SCHED_ADJOINT = 0, 1


def schedule_describe(n: int, p: int, state_dtype: int = QAOA_C128, init: bool = True, reduce: bool = True,
                      kind: int = SCHED_EVOLVE) -> list:
    """Launch order of one evaluation (kind SCHED_EVOLVE) or of the gradient's
    reverse pass (SCHED_ADJOINT): [(sweep, layer, flags)], empty for one-tile states."""
    need = lib.qaoa_schedule_describe(kind, n, p, state_dtype, int(init), int(reduce), None, 0)
    if need < 0:
        check(-need)
    buf = (ctypes.c_int * max(need, 1))()
    lib.qaoa_schedule_describe(kind, n, p, state_dtype, int(init), int(reduce), buf, need)
    v = list(buf)[:need]
    return [tuple(v[i:i + 3]) for i in range(0, need, 3)]


def workspace_bytes(op: int, n: int, state_dtype: int = QAOA_C128, diag_dtype: int = QAOA_DIAG_I32) -> int:
    out = ctypes.c_size_t(0)
    check(lib.qaoa_workspace_bytes(op, n, state_dtype, diag_dtype, ctypes.byref(out)))
    return int(out.value)


def alloc_workspace(op: int, n: int, state_dtype: int, diag_dtype: int, device) -> torch.Tensor:
    nb = workspace_bytes(op, n, state_dtype, diag_dtype)
    return torch.empty(max(nb, 16), dtype=torch.uint8, device=device)


# --------------------------------------------------------------------------
# entry points (same names as the C ABI)
# --------------------------------------------------------------------------
def qaoa_precompute_diag(n: int, terms, diag_dtype: str | int = "i32", device="cuda",
                         work: torch.Tensor | None = None):
    """Cost vector for Eq. (1) terms ``[(w, idx), ...]``; returns ``(diag, offset)``
    with ``c = diag + offset``."""
    code = DIAG_NAMES[diag_dtype] if isinstance(diag_dtype, str) else int(diag_dtype)
    w = [float(t[0]) for t in terms]
    ptr = [0]
    flat = []
    for _, idx in terms:
        flat.extend(int(i) for i in idx)
        ptr.append(len(flat))
    w_arr = _f64(w)
    ptr_arr = (ctypes.c_int64 * len(ptr))(*ptr)
    idx_arr = (ctypes.c_int32 * max(1, len(flat)))(*flat) if flat else None
    diag = torch.empty(1 << n, dtype=_DIAG_TORCH[code], device=device)
    if work is None:
        work = alloc_workspace(QAOA_OP_PRECOMPUTE, n, QAOA_C128, code, diag.device)
    off = ctypes.c_double(0.0)
    check(lib.qaoa_precompute_diag(n, len(terms), w_arr, ptr_arr, idx_arr, code, _dev_ptr(diag), _nbytes(diag),
                                   ctypes.byref(off), _dev_ptr(work), _nbytes(work), _stream(diag.device)))
    return diag, float(off.value)


def qaoa_evolve(n: int, gamma, beta, diag: torch.Tensor, state: torch.Tensor, init: bool = True,
                diag_offset: float = 0.0, out: torch.Tensor | None = None,
                work: torch.Tensor | None = None) -> None:
    """Algorithm 3 in place on ``state``; if ``out`` (float64[2], device) is given
    it receives (E, sum |psi|^2)."""
    p = len(gamma)
    if len(beta) != p:
        raise ValueError("gamma and beta differ in length")
    sdt, ddt = state_dtype_code(state), diag_dtype_code(diag)
    if work is None and (p > 0 or out is not None):
        work = alloc_workspace(QAOA_OP_EVOLVE, n, sdt, ddt, state.device)
    check(lib.qaoa_evolve(n, p, _f64(gamma), _f64(beta), _dev_ptr(diag), ddt, float(diag_offset), _nbytes(diag),
                          _dev_ptr(state), sdt, _nbytes(state), 1 if init else 0, _dev_ptr(out),
                          _dev_ptr(work), 0 if work is None else _nbytes(work), _stream(state.device)))


def qaoa_evolve_noalloc(n: int, gamma, beta, diag: torch.Tensor, state: torch.Tensor, init: bool = True,
                        diag_offset: float = 0.0, out: torch.Tensor | None = None) -> None:
    """qaoa_evolve without a workspace: the library's static per-GPU scratch
    serves instead (complex64 up to n=32, complex128 up to n=31); calls that
    overlap on one GPU race."""
    p = len(gamma)
    if len(beta) != p:
        raise ValueError("gamma and beta differ in length")
    sdt, ddt = state_dtype_code(state), diag_dtype_code(diag)
    check(lib.qaoa_evolve_noalloc(n, p, _f64(gamma), _f64(beta), _dev_ptr(diag), ddt, float(diag_offset),
                                  _nbytes(diag), _dev_ptr(state), sdt, _nbytes(state), 1 if init else 0,
                                  _dev_ptr(out), _stream(state.device)))


def qaoa_expectation(n: int, state: torch.Tensor, diag: torch.Tensor, diag_offset: float = 0.0,
                     out: torch.Tensor | None = None, work: torch.Tensor | None = None) -> torch.Tensor:
    """(E, sum |psi|^2) as a float64[2] device tensor."""
    sdt, ddt = state_dtype_code(state), diag_dtype_code(diag)
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=state.device)
    if work is None:
        work = alloc_workspace(QAOA_OP_EXPECTATION, n, sdt, ddt, state.device)
    check(lib.qaoa_expectation(n, _dev_ptr(state), sdt, _nbytes(state), _dev_ptr(diag), ddt, float(diag_offset),
                               _nbytes(diag), _dev_ptr(out), _dev_ptr(work), _nbytes(work), _stream(state.device)))
    return out


def grad_workspace_bytes(n: int, p: int, state_dtype: int, diag_dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check(lib.qaoa_grad_workspace_bytes(n, p, state_dtype, diag_dtype, ctypes.byref(out)))
    return int(out.value)


def qaoa_grad(n: int, gamma, beta, diag: torch.Tensor, state: torch.Tensor, adj: torch.Tensor,
              diag_offset: float = 0.0, out: torch.Tensor | None = None,
              work: torch.Tensor | None = None) -> torch.Tensor:
    """(E, dE/dgamma[p], dE/dbeta[p]) as a float64[1 + 2p] device tensor.
    ``state`` and ``adj`` are two scratch states (overwritten)."""
    p = len(gamma)
    if len(beta) != p:
        raise ValueError("gamma and beta differ in length")
    sdt, ddt = state_dtype_code(state), diag_dtype_code(diag)
    if adj.dtype != state.dtype or adj.numel() != state.numel():
        raise ValueError("adj must match state")
    if out is None:
        out = torch.empty(1 + 2 * p, dtype=torch.float64, device=state.device)
    if work is None:
        work = torch.empty(max(16, grad_workspace_bytes(n, p, sdt, ddt)), dtype=torch.uint8, device=state.device)
    check(lib.qaoa_grad(n, p, _f64(gamma), _f64(beta), _dev_ptr(diag), ddt, float(diag_offset), _nbytes(diag),
                        _dev_ptr(state), _dev_ptr(adj), sdt, _nbytes(state), _dev_ptr(out), _dev_ptr(work),
                        _nbytes(work), _stream(state.device)))
    return out


def xy_workspace_bytes(n: int, mixer: int, state_dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check(lib.qaoa_xy_workspace_bytes(n, mixer, state_dtype, ctypes.byref(out)))
    return int(out.value)


def qaoa_evolve_xy(n: int, gamma, beta, diag: torch.Tensor, state: torch.Tensor, mixer: int | str = MIXER_XY_RING,
                   init: int = INIT_PLUS, k: int = 0, diag_offset: float = 0.0, out: torch.Tensor | None = None,
                   work: torch.Tensor | None = None) -> None:
    """p layers of phase and XY mixer (ring or complete graph) in place on ``state``,
    which starts as |+>^n (INIT_PLUS), the Dicke state of weight k (INIT_DICKE), or
    as given (INIT_GIVEN); ``out`` (float64[2], device) receives (E, sum |psi|^2)."""
    p = len(gamma)
    if len(beta) != p:
        raise ValueError("gamma and beta differ in length")
    code = MIXER_NAMES[mixer] if isinstance(mixer, str) else int(mixer)
    sdt, ddt = state_dtype_code(state), diag_dtype_code(diag)
    if work is None:
        work = torch.empty(max(16, xy_workspace_bytes(n, code, sdt)), dtype=torch.uint8, device=state.device)
    check(lib.qaoa_evolve_xy(n, p, _f64(gamma), _f64(beta), code, _dev_ptr(diag), ddt, float(diag_offset),
                             _nbytes(diag), _dev_ptr(state), sdt, _nbytes(state), int(init), int(k), _dev_ptr(out),
                             _dev_ptr(work), _nbytes(work), _stream(state.device)))


def batch_workspace_bytes(n: int, p: int, batch: int, state_dtype: int, diag_dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check(lib.qaoa_batch_workspace_bytes(n, p, batch, state_dtype, diag_dtype, ctypes.byref(out)))
    return int(out.value)


def qaoa_evolve_batch(n: int, gamma: torch.Tensor, beta: torch.Tensor, diag: torch.Tensor, states: torch.Tensor,
                      init: bool = True, diag_offset: float = 0.0, out: torch.Tensor | None = None,
                      sets_per_pass: int = 0, work: torch.Tensor | None = None) -> None:
    """``batch`` evaluations: gamma, beta are float64 device tensors [batch, p];
    states is [batch, 2^n] complex; out (float64 [batch, 2]) receives (E, norm)."""
    if gamma.dtype != torch.float64 or beta.dtype != torch.float64 or gamma.shape != beta.shape or gamma.dim() != 2:
        raise ValueError("gamma and beta must be float64 tensors of shape [batch, p]")
    batch, p = gamma.shape
    if states.dim() != 2 or states.shape[0] != batch or states.shape[1] != 1 << n:
        raise ValueError("states must have shape [batch, 2^n]")
    sdt, ddt = state_dtype_code(states), diag_dtype_code(diag)
    if out is not None and (out.dtype != torch.float64 or out.numel() < 2 * batch):
        raise ValueError("out must be float64 with 2 * batch elements")
    if work is None:
        work = torch.empty(max(16, batch_workspace_bytes(n, p, batch, sdt, ddt)), dtype=torch.uint8,
                           device=states.device)
    check(lib.qaoa_evolve_batch(n, p, batch, _dev_ptr(gamma.contiguous()) if p else None,
                                _dev_ptr(beta.contiguous()) if p else None, _dev_ptr(diag), ddt, float(diag_offset),
                                _nbytes(diag), _dev_ptr(states), sdt, _nbytes(states), 1 if init else 0,
                                _dev_ptr(out), int(sets_per_pass), _dev_ptr(work), _nbytes(work),
                                _stream(states.device)))
