"""torch.autograd.Function around the C ABI: P(alpha, W) with the hand-written adjoint as backward.

forward() runs the forward sweep and the FP64 boundary reductions (qoc_objective);
backward() runs only the adjoint sweep (qoc_backward), which reuses the forward
sweep's end states held by the library, and scales dP/dalpha and dP/dW by the
incoming gradient.  The complex gradient follows PyTorch's convention for real
losses: grad W = dP/dRe W + i dP/dIm W.

The library keeps one forward state per System.  When the System has evaluated
other inputs since this node's forward (two graphs built on one System, a
finite-difference probe between forward and backward), backward() first re-runs
the forward sweep for the inputs saved with the node, so every graph receives the
adjoint of its own point.  backward() waits for the adjoint sweep and raises
QocError(QOC_ENOTCONV) when the implicit solve's contraction bound was exceeded.
"""
from __future__ import annotations

import torch

from . import qoc


def _load(system, alpha, W):
    system.set_controls(alpha.detach().contiguous())
    if system.M > 1:
        system.set_window_states(W.detach().contiguous())
    else:
        system.set_window_states(None)


class _PenaltyObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, W, system):
        if not alpha.is_cuda:
            raise ValueError("alpha must be a CUDA float64 tensor")
        _load(system, alpha, W)
        P = torch.empty(1, dtype=torch.float64, device=alpha.device)
        system.objective_into(P, None)
        ctx.system = system
        ctx.generation = system.generation
        ctx.has_W = system.M > 1
        ctx.save_for_backward(alpha.detach(), W.detach() if ctx.has_W else None)
        return P[0]

    @staticmethod
    def backward(ctx, grad_P):
        s = ctx.system
        if s.generation != ctx.generation:      # the System ran other inputs since this forward
            alpha, W = ctx.saved_tensors
            _load(s, alpha, W)
            s.objective_into(torch.empty(1, dtype=torch.float64, device=grad_P.device), None)
        ga = torch.empty(s.d, dtype=torch.float64, device=grad_P.device)
        gW = torch.empty((s.M - 1, s.E, s.N), dtype=torch.complex128, device=grad_P.device) if ctx.has_W else None
        s.backward_into(ga, gW)
        s.synchronize()                         # raises QOC_ENOTCONV on a bound violation
        ga = ga * grad_P
        if gW is not None:
            gW = gW * grad_P
        return ga, gW, None


def penalty_objective(alpha: torch.Tensor, W: torch.Tensor, system: "qoc.System") -> torch.Tensor:
    """P(alpha, W^1..W^{M-1}) as a differentiable scalar (alpha float64 [d], W complex128 [M-1, E, N])."""
    return _PenaltyObjective.apply(alpha, W, system)
