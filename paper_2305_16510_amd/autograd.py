"""torch.autograd.Function over the hand-written adjoint of the rollout.

loss = RolloutFn.apply(gains, x0, sim, n_steps, ckpt_every, w_omega) is the
tracking loss (1/n) sum_i sum_{t=1..T} |x_t - goal|^2 + w_omega |Omega_t|^2 of
the batch in ``sim`` started from x0 [13, n] with per-vehicle gains [10, n]
(the layout of rows 4..13 of the vehicle parameters).  The forward is one
call of ag_rollout_forward, which also forms the batch loss (fixed-order FP64
sum); the backward is one call of ag_rollout_adjoint, which reads the
upstream gradient on the device.  Torch only holds the tensors: each forward
keeps its own gains, starting state and checkpoint workspace for its
backward, so several losses may be formed on one simulator before any
backward runs.
"""
import torch


class RolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gains, x0, sim, n_steps, ckpt_every, w_omega=0.01):
        if sim.vparams is None:
            raise ValueError("the simulator needs per-vehicle parameters to differentiate gains")
        if gains.shape != (10, sim.n) or x0.shape != (13, sim.n):
            raise ValueError("gains [10, n] and x0 [13, n] expected")
        g = gains.detach().to(torch.float32).contiguous().clone()
        x = x0.detach().to(torch.float32).contiguous().clone()
        ws = sim.new_rollout_workspace(n_steps, ckpt_every)
        _, batch, _ = sim.rollout_forward(n_steps, ckpt_every, w_omega, x0=x, gains=g, ws=ws, want_loss_i=False)
        ctx.sim, ctx.ws, ctx.args = sim, ws, (n_steps, ckpt_every, w_omega)
        ctx.save_for_backward(g, x)
        return batch.reshape(())

    @staticmethod
    def backward(ctx, grad_loss):
        g, x = ctx.saved_tensors
        n_steps, ckpt_every, w_omega = ctx.args
        seed = grad_loss.detach().to(torch.float32).reshape(1).contiguous()
        dg, dx = ctx.sim.rollout_adjoint(n_steps, ckpt_every, w_omega, seed_grad=1.0, x0=x, gains=g, ws=ctx.ws,
                                         seed_dev=seed)
        return dg, dx, None, None, None, None


def rollout_loss(sim, gains, x0, n_steps, ckpt_every, w_omega=0.01):
    return RolloutFn.apply(gains, x0, sim, n_steps, ckpt_every, w_omega)
