"""torch.autograd.Function over the hand-written adjoint of the rollout.

loss = RolloutFn.apply(gains, x0, sim, n_steps, ckpt_every, w_omega) is the
tracking loss (1/n) sum_i sum_{t=1..T} |x_t - goal|^2 + w_omega |Omega_t|^2 of
the batch in ``sim`` started from x0 [13, n] with per-vehicle gains [10, n]
(rows 4..13 of the vehicle parameters).  Forward and backward each run one
HIP kernel (ag_rollout_forward / ag_rollout_adjoint); torch only holds the
tensors.
"""
import torch


class RolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gains, x0, sim, n_steps, ckpt_every, w_omega=0.01):
        if sim.vparams is None:
            raise ValueError("the simulator needs per-vehicle parameters to differentiate gains")
        with torch.no_grad():
            sim.vparams[4:14].copy_(gains.detach())
        x0c = x0.detach().contiguous()
        loss_i, _ = sim.rollout_forward(n_steps, ckpt_every, w_omega, x0=x0c)
        ctx.sim, ctx.args = sim, (n_steps, ckpt_every, w_omega)
        ctx.save_for_backward(x0c)
        return loss_i.double().sum().float() / sim.n

    @staticmethod
    def backward(ctx, grad_loss):
        (x0c,) = ctx.saved_tensors
        n_steps, ckpt_every, w_omega = ctx.args
        dg, dx = ctx.sim.rollout_adjoint(n_steps, ckpt_every, w_omega, seed_grad=float(grad_loss), x0=x0c)
        return dg, dx, None, None, None, None


def rollout_loss(sim, gains, x0, n_steps, ckpt_every, w_omega=0.01):
    return RolloutFn.apply(gains, x0, sim, n_steps, ckpt_every, w_omega)
