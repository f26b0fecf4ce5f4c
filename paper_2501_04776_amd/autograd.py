"""torch.autograd Functions over the C-ABI (the computational graph of the
paper's Fig. 3 with the reverse pass written by hand)."""
from __future__ import annotations

import torch

from . import api


class IQPExpval(torch.autograd.Function):
    """(mean[l], stderr[l]) = IQPExpval.apply(theta, gens, ops, samples, n_qubits, precision).

    Differentiable in theta through mean; stderr carries no gradient (a
    non-zero gradient on it raises)."""

    @staticmethod
    def forward(ctx, theta, gens, ops, samples, n_qubits, precision="split_bf16"):
        circ = api.Circuit(n_qubits, gens, theta.detach())
        mean, se, ph = api.iqp_expval(circ, ops, samples, precision, stderr=True,
                                      phase_save=theta.requires_grad)
        ctx.save_for_backward(theta, gens, ops, samples, ph if ph is not None else
                              torch.empty(0, device=theta.device))
        ctx.n_qubits = n_qubits
        ctx.precision = precision
        ctx.mark_non_differentiable(se)
        return mean, se

    @staticmethod
    def backward(ctx, grad_mean, grad_se):
        theta, gens, ops, samples, ph = ctx.saved_tensors
        if grad_se is not None and bool((grad_se != 0).any()):
            raise RuntimeError("the standard error is not differentiable")
        circ = api.Circuit(ctx.n_qubits, gens, theta.detach())
        g = api.iqp_expval_grad(circ, ops, samples, grad_mean.to(torch.float64).contiguous(),
                                phase_save=ph if ph.numel() else None, precision=ctx.precision)
        return g.to(theta.dtype), None, None, None, None, None


class IQPMMDLoss(torch.autograd.Function):
    """loss = IQPMMDLoss.apply(theta, gens, ops, op_weight, samples, data, n_qubits,
    unbiased, precision). The gradient is computed with the loss and scaled by
    grad_output in backward."""

    @staticmethod
    def forward(ctx, theta, gens, ops, op_weight, samples, data, n_qubits, unbiased=True,
                precision="split_bf16"):
        circ = api.Circuit(n_qubits, gens, theta.detach())
        loss, g = api.iqp_mmd_loss_grad(circ, ops, op_weight, samples, data, unbiased,
                                        grad=theta.requires_grad, precision=precision)
        ctx.save_for_backward(g if g is not None else torch.empty(0, device=theta.device))
        ctx.theta_dtype = theta.dtype
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return ((g * grad_out).to(ctx.theta_dtype), None, None, None, None, None, None, None,
                None)


class IQPBitflipExpval(torch.autograd.Function):
    """mean[l] = IQPBitflipExpval.apply(theta, gens, ops, n_qubits): the exact
    expectation values of the stochastic bitflip version of the circuit
    (Prop. 3), differentiable in theta."""

    @staticmethod
    def forward(ctx, theta, gens, ops, n_qubits):
        circ = api.Circuit(n_qubits, gens, theta.detach())
        mean = api.iqp_bitflip_expval(circ, ops)
        ctx.save_for_backward(theta, gens, ops)
        ctx.n_qubits = n_qubits
        return mean

    @staticmethod
    def backward(ctx, grad_mean):
        theta, gens, ops = ctx.saved_tensors
        circ = api.Circuit(ctx.n_qubits, gens, theta.detach())
        g = api.iqp_bitflip_expval_grad(circ, ops, grad_mean.to(torch.float64).contiguous())
        return g.to(theta.dtype), None, None, None
