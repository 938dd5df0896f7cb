"""torch.autograd wrapper of the adjoint gradient: the survival probability
F(T) as a differentiable function of the on-site fields.

The forward call sets the fields of the workspace's Hamiltonian and runs
qk_grad_return_prob, which returns F(T) and dF/dh in one pass; backward scales
the stored derivative by the incoming gradient.  All computation happens in
the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Krylov, qk_grad_return_prob, qk_ham_set_fields


class SurvivalProbability(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fields: torch.Tensor, k: Krylov, r0: int, T: float, n_steps: int, ckpt_every: int = 1):
        h = fields.detach().to("cpu", torch.float64).numpy()
        qk_ham_set_fields(k.H, h)
        F, g = qk_grad_return_prob(k, r0, T, n_steps, ckpt_every)
        ctx.save_for_backward(torch.from_numpy(np.ascontiguousarray(g)).to(fields.device, fields.dtype))
        return torch.tensor(F, dtype=fields.dtype, device=fields.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None, None, None


def survival_probability(fields: torch.Tensor, k: Krylov, r0: int, T: float, n_steps: int,
                         ckpt_every: int = 1) -> torch.Tensor:
    """F(T) = |<e_r0| exp(-iHT) |e_r0>|^2 with H's fields set to `fields` (length L);
    differentiable with respect to `fields`."""
    return SurvivalProbability.apply(fields, k, r0, T, n_steps, ckpt_every)
