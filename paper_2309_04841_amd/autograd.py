"""torch.autograd binding of the adjoint gradient.

    E = qaoa_objective(gamma, beta, sim)     # gamma, beta: float64 tensors [p]
    E.backward()                             # gamma.grad, beta.grad from qaoa_grad

When any input requires a gradient, the forward pass calls qaoa_grad once
(forward evolution + reverse sweeps on the GPU) and keeps dE/dgamma, dE/dbeta
for backward; otherwise it runs the plain evaluation.
"""
from __future__ import annotations

import torch


class QAOAObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma: torch.Tensor, beta: torch.Tensor, sim) -> torch.Tensor:
        g = gamma.detach().to("cpu", torch.float64).numpy()
        b = beta.detach().to("cpu", torch.float64).numpy()
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            E, dg, db = sim.get_gradient(g, b)
            ctx.save_for_backward(torch.as_tensor(dg, dtype=gamma.dtype, device=gamma.device),
                                  torch.as_tensor(db, dtype=beta.dtype, device=beta.device))
        else:
            E = sim.get_expectation(sim.simulate_qaoa(g, b))
        return torch.tensor(E, dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        dg, db = ctx.saved_tensors
        return grad_out * dg, grad_out * db, None


def qaoa_objective(gamma: torch.Tensor, beta: torch.Tensor, sim) -> torch.Tensor:
    """Differentiable QAOA objective <gamma beta|C|gamma beta> of ``sim``'s problem."""
    return QAOAObjective.apply(gamma, beta, sim)
