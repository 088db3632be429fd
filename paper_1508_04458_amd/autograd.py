"""Differentiable I-divergence data term in the wavelet domain (eq. 1.3 with lambda = 0).

WamLoss.apply(c, d, i0, ctx) returns loss_b = I(d_b || I0 exp(-H Omega c_b)) (float64, [B])
for coefficients c [B, n, n] (Mallat layout, all coefficients free). The forward pass keeps
q_b = I0 exp(-H Omega c_b) (checkpoint); the backward pass is the hand-written adjoint
grad_b = g_b Omega^T H^T (d_b - q_b) on the GPU, computed from the checkpoint without
re-running the forward projection."""
import torch


class WamLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, c, d, i0, wctx):
        loss, q = wctx.loss(c.contiguous(), d.contiguous(), i0)
        fctx.save_for_backward(q, d)
        fctx.wctx = wctx
        return loss

    @staticmethod
    def backward(fctx, grad_loss):
        q, d = fctx.saved_tensors
        grad = fctx.wctx.loss_backward(q, d.contiguous(), grad_loss)
        return grad, None, None, None


def wam_loss(c, d, i0, wctx):
    return WamLoss.apply(c, d, i0, wctx)
