"""Host-side parts of bench.py: the one-GPU contract and the algorithmic byte
counts its roofline uses (checked against closed forms written out here)."""
import os
import subprocess
import sys

import bench
from paper_2309_04841_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_sweep_bytes_closed_form():
    # per evaluation: L launches, the first writes only, every launch moves the
    # state (S bytes per element each way), the p + 1 launches that apply a
    # phase or reduce E read the cost vector: B = [(2L - 1) S + (p + 1) D] 2^n
    for n, p, sdt, S, D in ((26, 10, _lib.QAOA_C128, 16, 2), (31, 10, _lib.QAOA_C64, 8, 2), (20, 3, _lib.QAOA_C128, 16, 4)):
        sched = _lib.schedule_describe(n, p, sdt)
        L = len(sched)
        assert sum(bench._sweep_bytes(sched, n, S, D)) == ((2 * L - 1) * S + (p + 1) * D) * (1 << n)
    # LABS n=26 p=10 complex128 uint16: 11 launches, 24.0 GB
    sched = _lib.schedule_describe(26, 10, _lib.QAOA_C128)
    assert len(sched) == 11
    assert abs(sum(bench._sweep_bytes(sched, 26, 16, 2)) - 24.0e9) < 0.1e9


def test_xy_sweep_bytes_closed_form():
    # p layers of s sweeps: (2 p s - 1) state passes, p + 1 cost reads (one per
    # layer's phase, one for E) when s > 1
    n, p, s, S, D = 26, 10, 3, 16, 2
    assert sum(bench._xy_sweep_bytes(n, p, s, S, D)) == ((2 * p * s - 1) * S + (p + 1) * D) * (1 << n)


def test_adjoint_bytes_closed_form():
    # reverse pass: the first launch reads psi and c and writes psi and lambda;
    # every other moves both states both ways; launches that undo a phase read c
    n, p = 24, 20
    sched = _lib.schedule_describe(n, p, _lib.QAOA_C128, kind=_lib.SCHED_ADJOINT)
    per = bench._adjoint_bytes(sched, n, 16, 2)
    nphase = sum(1 for _, _, f in sched if f & (_lib.A_PHASE | _lib.A_FUSE))
    assert sum(per) == ((3 + 4 * (len(sched) - 1)) * 16 + (1 + nphase) * 2) * (1 << n)
    # every layer's phase is undone exactly once
    assert nphase == p
