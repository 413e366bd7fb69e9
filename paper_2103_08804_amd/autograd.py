"""torch.autograd.Function around the fidelity-surrogate forward and its hand-written backward.

Forward: on a frozen sample set, R(s) = phi(s)/psi_{n+1}(s; a, b, W) and
tanh(theta) from crbm_local_estimators (Chebyshev mode), then
L = (1/n) sum_s |1 - R(s)|^2 from crbm_fidelity_grad (loss only).
Backward: crbm_fidelity_grad with the saved R and tanh(theta),
dL/dRe(alpha) + i dL/dIm(alpha) = (2/n) sum_s (1 - R) conj(R) conj(O(s)),
which is the gradient PyTorch expects for a real loss of complex leaves.
Both passes run in the HIP library; this module only moves tensors.
"""
from __future__ import annotations

import torch

from . import RBM, Plan, fidelity_grad, local_estimators


class FidelityLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b, W, plan: Plan, samples, psi_n: RBM, psi_nm1: RBM | None, cheb):
        n = samples.shape[0]
        fit = RBM(a.detach(), b.detach(), W.detach())
        R = torch.empty(n, dtype=torch.complex64, device=a.device)
        T = torch.empty(n, plan.M, dtype=torch.complex64, device=a.device)
        local_estimators(plan, fit, samples, psi_n=psi_n, psi_nm1=psi_nm1, cheb=cheb, R_out=R, tanh_out=T)
        loss = torch.empty(1, dtype=torch.float64, device=a.device)
        fidelity_grad(plan, fit, samples, T, R, None, loss)
        ctx.save_for_backward(samples, T, R)
        ctx.plan, ctx.fit = plan, fit
        return loss[0]

    @staticmethod
    def backward(ctx, g_loss):
        samples, T, R = ctx.saved_tensors
        plan = ctx.plan
        N, M = plan.N, plan.M
        grad = torch.empty(plan.P, dtype=torch.complex128, device=T.device)
        fidelity_grad(plan, ctx.fit, samples, T, R, grad, None)
        g = grad * g_loss
        return g[:N].to(torch.complex64), g[N:N + M].to(torch.complex64), \
            g[N + M:].view(N, M).to(torch.complex64), None, None, None, None, None


def fidelity_loss(fit: RBM, plan: Plan, samples, psi_n: RBM, psi_nm1: RBM | None, cheb):
    """L(fit) on frozen samples (float64 scalar); differentiable with respect to fit.a, fit.b, fit.W."""
    return FidelityLoss.apply(fit.a, fit.b, fit.W, plan, samples, psi_n, psi_nm1, cheb)
