"""QOKit-style simulator object over the C ABI (Section 4, Listing 1).

    sim = Simulator(n, terms=terms)            # precomputes the cost vector once
    costs = sim.get_cost_diagonal()
    result = sim.simulate_qaoa(gamma, beta)    # state stays on the GPU
    E = sim.get_expectation(result)

Only argument marshalling happens here; every step runs in libqaoa.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib

_STATE = {"complex64": torch.complex64, "complex128": torch.complex128,
          torch.complex64: torch.complex64, torch.complex128: torch.complex128}


class Simulator:
    """Transverse-field-mixer QAOA simulator for one problem (one cost vector)."""

    def __init__(self, n: int, terms=None, costs=None, dtype="complex128", diag_dtype: str = "i32",
                 device: str | torch.device = "cuda"):
        if (terms is None) == (costs is None):
            raise ValueError("give exactly one of terms= or costs=")
        if not 1 <= n <= _lib.QAOA_MAX_QUBITS:
            raise ValueError(f"n={n} out of range")
        self.n = int(n)
        self.device = torch.device(device)
        self.state_dtype = _STATE[dtype]
        if terms is not None:
            self.diag, self.offset = _lib.qaoa_precompute_diag(self.n, terms, diag_dtype, self.device)
        else:
            c = torch.as_tensor(np.asarray(costs) if not isinstance(costs, torch.Tensor) else costs)
            if c.numel() != 1 << self.n:
                raise ValueError("costs must have 2^n entries")
            self.diag = c.to(device=self.device, dtype=torch.float64).contiguous()
            self.offset = 0.0
        sdt = _lib.state_dtype_code(torch.empty(0, dtype=self.state_dtype))
        ddt = _lib.diag_dtype_code(self.diag)
        self._work = _lib.alloc_workspace(_lib.QAOA_OP_EVOLVE, self.n, sdt, ddt, self.device)
        self._out = torch.empty(2, dtype=torch.float64, device=self.device)

    # -- inputs ------------------------------------------------------------
    def get_cost_diagonal(self) -> np.ndarray:
        """The precomputed cost vector c as float64 on the host."""
        return self.diag.cpu().numpy().astype(np.float64) + self.offset

    # -- simulation --------------------------------------------------------
    def simulate_qaoa(self, gamma, beta, initial_state=None) -> torch.Tensor:
        """Evolve |+>^n (or ``initial_state``) through len(gamma) layers."""
        gamma = np.atleast_1d(np.asarray(gamma, dtype=np.float64))
        beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
        if initial_state is None:
            psi = torch.empty(1 << self.n, dtype=self.state_dtype, device=self.device)
            init = True
        else:
            psi = torch.as_tensor(initial_state).to(device=self.device, dtype=self.state_dtype).contiguous().clone()
            init = False
        _lib.qaoa_evolve(self.n, gamma, beta, self.diag, psi, init=init, diag_offset=self.offset, work=self._work)
        return psi

    # -- outputs -----------------------------------------------------------
    def get_expectation(self, result: torch.Tensor, costs=None) -> float:
        """E = sum |psi|^2 c with this problem's c, or with ``costs`` if given."""
        if costs is None:
            diag, off = self.diag, self.offset
        else:
            diag = torch.as_tensor(np.asarray(costs) if not isinstance(costs, torch.Tensor) else costs)
            diag, off = diag.to(device=self.device, dtype=torch.float64).contiguous(), 0.0
        out = _lib.qaoa_expectation(self.n, result, diag, off, out=self._out, work=self._work)
        return float(out[0].item())

    def get_norm(self, result: torch.Tensor) -> float:
        out = _lib.qaoa_expectation(self.n, result, self.diag, self.offset, out=self._out, work=self._work)
        return float(out[1].item())

    def get_gradient(self, gamma, beta):
        """(E, dE/dgamma, dE/dbeta) from |+>^n by the adjoint method on the GPU."""
        gamma = np.atleast_1d(np.asarray(gamma, dtype=np.float64))
        beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
        p = len(gamma)
        if getattr(self, "_grad_bufs", None) is None:
            self._grad_bufs = tuple(torch.empty(1 << self.n, dtype=self.state_dtype, device=self.device)
                                    for _ in range(2))
        psi, adj = self._grad_bufs
        out = _lib.qaoa_grad(self.n, gamma, beta, self.diag, psi, adj, diag_offset=self.offset)
        o = out.cpu().numpy()
        return float(o[0]), o[1:1 + p].copy(), o[1 + p:].copy()

    def get_statevector(self, result: torch.Tensor) -> np.ndarray:
        return result.cpu().numpy()

    def get_probabilities(self, result: torch.Tensor) -> np.ndarray:
        return np.abs(self.get_statevector(result)) ** 2
