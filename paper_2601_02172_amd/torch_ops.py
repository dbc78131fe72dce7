"""torch.autograd.Function over the solver: C_eff as a function of the Lame pairs.

Forward solves the six unit loads (``xfft_solve``); backward contracts the
incoming gradient with dC_eff/d(lambda_p, mu_p) from ``xfft_grad_lame`` (the
closed form that Galerkin orthogonality gives for the energy form of C_eff,
App. A of the paper).  torch only carries the (tiny) parameter and gradient
tensors; all field work runs in the HIP library.

The gradient uses the unit-load solutions the problem holds.  Every graph node
records the moduli of its forward and the problem's solve generation; when
another solve has run on the problem since (a second forward, finite
differences), backward solves again at the recorded moduli before it takes the
gradient, so each node's gradient belongs to its own forward.
"""

import numpy as np
import torch


def _solve_unit_loads(problem):
    C, info = problem.effective_stiffness()
    if not info["converged"]:
        raise RuntimeError("xfft_solve did not reach the tolerance (res/|<sigma>| = "
                           f"{np.max(info['final_res']):.3e} after {int(np.max(info['iters']))} iterations)")
    return C


class EffectiveStiffness(torch.autograd.Function):
    """C = EffectiveStiffness.apply(lame, problem): lame (nphase, 2) -> C_eff (6, 6)."""

    @staticmethod
    def forward(ctx, lame, problem):
        lame64 = np.array(lame.detach().to("cpu", torch.float64).numpy(), dtype=np.float64)
        problem.set_lame(lame64)
        C = _solve_unit_loads(problem)
        ctx.problem = problem
        ctx.lame64 = lame64
        ctx.generation = problem.generation
        return torch.as_tensor(C, dtype=lame.dtype, device=lame.device)

    @staticmethod
    def backward(ctx, grad_C):
        p = ctx.problem
        if p.generation != ctx.generation:
            p.set_lame(ctx.lame64)
            _solve_unit_loads(p)
        W = grad_C.detach().to("cpu", torch.float64).numpy()
        g, _ = p.grad_lame(W)
        return torch.as_tensor(np.asarray(g), dtype=grad_C.dtype, device=grad_C.device), None


def effective_stiffness(lame, problem):
    """Differentiable C_eff(lame) for a set-up ``Problem``."""
    return EffectiveStiffness.apply(lame, problem)
