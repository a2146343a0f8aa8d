"""QAOA state-vector simulation for AMD MI355X (gfx950).

Hot path of "Fast Simulation of High-Depth QAOA Circuits" (arXiv:2309.04841):
cost vector precomputed once from spin terms, p layers of phase and
transverse-field mixer applied by hand-written HIP kernels, and the objective
E = sum |psi|^2 c reduced in FP64.  The kernels sit behind the C ABI in
include/qaoa.h (libqaoa.so); this package is its thin Python binding.
"""
from ._lib import (QaoaError, qaoa_evolve, qaoa_evolve_batch, qaoa_evolve_noalloc, qaoa_evolve_xy, qaoa_expectation, qaoa_grad,
                   qaoa_precompute_diag, version, workspace_bytes)
from .autograd import QAOAObjective, qaoa_objective
from .server import QAOAServer
from .simulator import Simulator

__all__ = ["Simulator", "QAOAServer", "QaoaError", "qaoa_precompute_diag", "qaoa_evolve", "qaoa_evolve_batch", "qaoa_evolve_noalloc", "qaoa_evolve_xy",
           "qaoa_expectation", "qaoa_grad", "qaoa_objective", "QAOAObjective", "workspace_bytes", "version"]
