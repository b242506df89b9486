"""torch.autograd bindings of the convolutional coarse propagator, for
training it on trajectories of the fine propagator (Section 3.2,
Algorithm 1).  Argument marshalling only: forward and backward both run in
libpr's kernels (pr_coarse_apply, pr_cnn_backward).

CnnApply    one application G(u; W, b).
SchemeLoss  the scheme-residual loss of eq. loss_ACN of a pair (U_n, U_{n+1})
            with its gradient with respect to U_{n+1} (pr_scheme_loss).
CnnRollout  s successive applications u_{t+1} = G(u_t), returning every
            u_t (t = 1..s).  Only every `ckpt`-th state is kept; backward
            recomputes each segment of `ckpt` steps from its first state
            before running back through it (activation checkpointing across
            the rollout; inside one application the library recomputes the
            layers itself).
"""

from __future__ import annotations

import torch

from . import api


class CnnApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, W, B, net, problem):
        if W.data_ptr() != net.W.data_ptr() or B.data_ptr() != net.B.data_ptr():
            raise ValueError("W and B must be the network's own parameter buffers")
        out = api.pr_coarse_apply(problem, net, u.contiguous())
        ctx.save_for_backward(u)
        ctx.net, ctx.problem = net, problem
        return out

    @staticmethod
    def backward(ctx, gout):
        (u,) = ctx.saved_tensors
        du, dW, dB = api.pr_cnn_backward(ctx.problem, ctx.net, u.contiguous(), gout.contiguous())
        return du, dW, dB, None, None


def cnn_apply(net, problem, u):
    return CnnApply.apply(u, net.W, net.B, net, problem)


class CnnRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, W, B, net, problem, steps, ckpt):
        if W.data_ptr() != net.W.data_ptr() or B.data_ptr() != net.B.data_ptr():
            raise ValueError("W and B must be the network's own parameter buffers")
        outs = []
        keep = []
        u = u0.contiguous()
        for t in range(steps):
            if t % ckpt == 0:
                keep.append(u)
            u = api.pr_coarse_apply(problem, net, u)
            outs.append(u)
        ctx.save_for_backward(*keep)
        ctx.net, ctx.problem, ctx.steps, ctx.ckpt = net, problem, steps, ckpt
        return torch.stack(outs)

    @staticmethod
    def backward(ctx, gouts):
        keep = ctx.saved_tensors
        net, problem, steps, ckpt = ctx.net, ctx.problem, ctx.steps, ctx.ckpt
        dW = torch.zeros_like(net.W)
        dB = torch.zeros_like(net.B)
        d = torch.zeros_like(keep[0])
        for seg in reversed(range(0, steps, ckpt)):
            end = min(seg + ckpt, steps)
            inputs = [keep[seg // ckpt]]
            for _ in range(seg, end - 1):
                inputs.append(api.pr_coarse_apply(problem, net, inputs[-1]))
            for t in reversed(range(seg, end)):
                d = d + gouts[t]
                du, w, b = api.pr_cnn_backward(problem, net, inputs[t - seg], d.contiguous())
                dW += w
                dB += b
                d = du
        return d, dW, dB, None, None, None, None


def cnn_rollout(net, problem, u0, steps, ckpt=2):
    return CnnRollout.apply(u0, net.W, net.B, net, problem, steps, ckpt)


class SchemeLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u_n, u_np1, problem, dt):
        loss, grad, _ = api.pr_scheme_loss(problem, dt, u_n.detach().contiguous(),
                                           u_np1.detach().contiguous(), grad=True)
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return None, grad * gout, None, None


def scheme_loss(problem, u_n, u_np1, dt):
    """mean(r^2) of the Crank-Nicolson residual of (u_n, u_np1); differentiable
    in u_np1 (u_n is data)."""
    return SchemeLoss.apply(u_n, u_np1, problem, dt)
