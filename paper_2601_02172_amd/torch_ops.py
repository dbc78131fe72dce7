"""torch.autograd.Function over the solver: C_eff as a function of the Lame pairs.

Forward solves the six unit loads (``xfft_solve``); backward contracts the
incoming gradient with dC_eff/d(lambda_p, mu_p) from ``xfft_grad_lame`` (the
closed form that Galerkin orthogonality gives for the energy form of C_eff,
App. A of the paper).  torch only carries the (tiny) parameter and gradient
tensors; all field work runs in the HIP library.
"""

import numpy as np
import torch


class EffectiveStiffness(torch.autograd.Function):
    """C = EffectiveStiffness.apply(lame, problem): lame (nphase, 2) -> C_eff (6, 6)."""

    @staticmethod
    def forward(ctx, lame, problem):
        problem.set_lame(lame.detach().to("cpu", torch.float64).numpy())
        C, _ = problem.effective_stiffness()
        ctx.problem = problem
        return torch.as_tensor(C, dtype=lame.dtype, device=lame.device)

    @staticmethod
    def backward(ctx, grad_C):
        W = grad_C.detach().to("cpu", torch.float64).numpy()
        g, _ = ctx.problem.grad_lame(W)
        return torch.as_tensor(np.asarray(g), dtype=grad_C.dtype, device=grad_C.device), None


def effective_stiffness(lame, problem):
    """Differentiable C_eff(lame) for a set-up ``Problem``."""
    return EffectiveStiffness.apply(lame, problem)
