"""torch.autograd.Function over the library's objective and hand-written adjoint.

Two modes:
  "recompute"  forward runs mpbp_forward (no exit waves kept); backward runs
               mpbp_loss_grad, recomputing the exit waves;
  "fused"      forward runs mpbp_loss_grad once and keeps the three gradients
               (16 bytes per voxel) for backward.
The loss is the sum over the listed frames (eq. (4) restricted to a minibatch, as in
eq. (11)); its gradient with respect to u, chi and alpha is returned, scaled by the
incoming gradient.
"""
import torch


class MPBPLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, chi, alpha, plan, probe, y, frames=None, mode="recompute"):
        for name, t in (("u", u), ("chi", chi), ("alpha", alpha), ("y", y)):
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if probe.dtype != torch.complex64 or not probe.is_contiguous():
            raise ValueError("probe must be a contiguous complex64 CUDA tensor")
        if mode not in ("recompute", "fused"):
            raise ValueError("mode must be 'recompute' or 'fused'")
        loss = torch.zeros((), dtype=torch.float64, device=u.device)
        ctx.plan, ctx.frames, ctx.mode = plan, frames, mode
        if mode == "fused":
            gu, gc, ga = torch.empty_like(u), torch.empty_like(chi), torch.empty_like(alpha)
            plan.mpbp_loss_grad(u, chi, alpha, probe, y, gu, gc, ga, frames=frames, loss=loss)
            ctx.save_for_backward(gu, gc, ga)
        else:
            plan.mpbp_forward(u, chi, alpha, probe, y, frames=frames, loss=loss)
            ctx.save_for_backward(u, chi, alpha, probe, y)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        if ctx.mode == "fused":
            gu, gc, ga = ctx.saved_tensors
        else:
            u, chi, alpha, probe, y = ctx.saved_tensors
            gu, gc, ga = torch.empty_like(u), torch.empty_like(chi), torch.empty_like(alpha)
            ctx.plan.mpbp_loss_grad(u, chi, alpha, probe, y, gu, gc, ga, frames=ctx.frames)
        g = grad_loss.to(torch.float32)
        return gu * g, gc * g, ga * g, None, None, None, None, None
