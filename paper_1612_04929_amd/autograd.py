"""torch.autograd bridge to the hand-written cost + exact-gradient kernels.

``QocCostGrad.apply(u, problem)`` runs one ``qoc_cost_grad_device`` call
on the tensor's device and current stream: the forward pass returns the
weighted cost C (differentiable), the fidelity cost C_fid and the per-step
penalties c_1..c_N (both non-differentiable); the backward pass scales the
gradient that the same call already produced (reverse accumulation of the
costates and the exact derivative of every step exponential, Sec. II.B and
Sec. III) by the incoming cotangent.  No work runs in torch beyond the
buffer allocation and that scaling.
"""
from __future__ import annotations

import torch

from .qoc import Problem


def _check_u(u: torch.Tensor, problem: Problem) -> None:
    if not isinstance(u, torch.Tensor):
        raise TypeError("u must be a torch.Tensor")
    if u.device.type != "cuda":
        raise ValueError("u must live on a GPU: the cost and gradient run only in the HIP kernels")
    if u.dtype != torch.float64:
        raise TypeError("u must be float64 (the C-ABI takes FP64 amplitudes)")
    if tuple(u.shape) != (problem.M, problem.N):
        raise ValueError(f"u has shape {tuple(u.shape)}, expected ({problem.M}, {problem.N})")


class QocCostGrad(torch.autograd.Function):
    """(C, C_fid, c) = QocCostGrad.apply(u, problem); dC/du in backward."""

    @staticmethod
    def forward(ctx, u, problem, check=False):
        _check_u(u, problem)
        uc = u.detach().contiguous()
        out = torch.empty(2 + problem.N, dtype=torch.float64, device=u.device)
        grad = torch.empty(max(1, problem.M * problem.N), dtype=torch.float64, device=u.device)
        stream = torch.cuda.current_stream(u.device).cuda_stream
        problem.cost_grad_device(uc.data_ptr(), out.data_ptr(), grad.data_ptr(), stream)
        if check:
            # synchronises: raises if the call ran with a clamped (p, n)
            problem.check_last()
        C, C_fid, c = out[0], out[1], out[2:]
        ctx.save_for_backward(grad)
        ctx.shape = (problem.M, problem.N)
        ctx.mark_non_differentiable(C_fid, c)
        return C, C_fid, c

    @staticmethod
    def backward(ctx, gC, gCfid, gc):
        (grad,) = ctx.saved_tensors
        M, N = ctx.shape
        g = grad[: M * N].view(M, N)
        return (gC * g if gC is not None else None), None, None


def cost(u: torch.Tensor, problem: Problem, check: bool = False):
    """Differentiable weighted cost C(u) (plus C_fid and c_1..c_N).  With
    check=True the call synchronises and raises if no (p, n) met the
    tolerance (QOC_WARN_NO_PAIR)."""
    return QocCostGrad.apply(u, problem, check)
