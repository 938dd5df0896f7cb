"""torch.autograd wrapper of the adjoint gradient: the survival probability
F(T) (Sec. 4) as a differentiable function of the on-site fields of Eq. (1).

forward propagates e_r0 to T with the workspace's Krylov steps and returns
F(T) = |psi(T)[r0]|^2; nothing else is computed unless a gradient is asked
for.  backward runs the adjoint sweep (qk_grad_return_prob: forward states
kept as checkpoints, the costate taken backward as the conjugated forward
states, the in-step contractions) and scales dF/dh by the incoming gradient.  Both set the
workspace Hamiltonian's fields to the given ones for their duration and
restore the previous fields afterwards, so other users of the Hamiltonian
see no change.  All computation happens in the library's kernels.
"""
from __future__ import annotations

import contextlib

import numpy as np
import torch

from . import Krylov, qk_grad_return_prob, qk_ham_get_fields, qk_ham_set_fields, qk_ham_shape, qk_krylov_expm_step


@contextlib.contextmanager
def _fields_set(k: Krylov, h: np.ndarray):
    old = qk_ham_get_fields(k.H)
    qk_ham_set_fields(k.H, h)
    try:
        yield
    finally:
        qk_ham_set_fields(k.H, old)


class SurvivalProbability(torch.autograd.Function):
    @staticmethod
    def forward(ctx, fields: torch.Tensor, k: Krylov, r0: int, T: float, n_steps: int, ckpt_every: int = 1):
        h = np.ascontiguousarray(fields.detach().to("cpu", torch.float64).numpy())
        if h.shape != (k.H.L,):
            raise ValueError(f"fields must have shape ({k.H.L},)")
        with _fields_set(k, h):
            dtype = torch.complex128 if k.dtype == 0 else torch.complex64
            psi = torch.zeros(qk_ham_shape(k.H)[0], dtype=dtype, device="cuda")
            psi[r0] = 1.0
            for _ in range(n_steps):
                qk_krylov_expm_step(k, psi, T / n_steps)
            F = float(abs(psi[r0].item()) ** 2)
        ctx.k, ctx.r0, ctx.T, ctx.n_steps, ctx.ckpt_every, ctx.h = k, r0, T, n_steps, ckpt_every, h
        return torch.tensor(F, dtype=fields.dtype, device=fields.device)

    @staticmethod
    def backward(ctx, grad_out):
        with _fields_set(ctx.k, ctx.h):
            _, g = qk_grad_return_prob(ctx.k, ctx.r0, ctx.T, ctx.n_steps, ctx.ckpt_every)
        gt = torch.from_numpy(np.ascontiguousarray(g)).to(grad_out.device, grad_out.dtype)
        return grad_out * gt, None, None, None, None, None


def survival_probability(fields: torch.Tensor, k: Krylov, r0: int, T: float, n_steps: int,
                         ckpt_every: int = 1) -> torch.Tensor:
    """F(T) = |<e_r0| exp(-iHT) |e_r0>|^2 with H's fields set to `fields` (length L)
    for the call; differentiable with respect to `fields` (the adjoint runs in
    backward only)."""
    return SurvivalProbability.apply(fields, k, r0, T, n_steps, ckpt_every)
