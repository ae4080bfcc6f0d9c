"""Pins of the oracle's FP64 reverse-mode gradient of the tracking loss
against central finite differences and a directional (JVP/VJP) check."""
import numpy as np
import torch

import workloads
from oracle import step as ostep
from oracle.fleet import Fleet

F64 = torch.float64


def small_problem(n=6, seed=11, T=40):
    wl = workloads.c4_grad(n=n, seed=seed, steps=T)
    s0, mode, tgt = ostep.from_workload_arrays(wl.state0, wl.mode, wl.target)
    tgt[:, :3] = torch.randn(n, 3, generator=torch.Generator().manual_seed(seed), dtype=F64)
    fleet = Fleet.from_groups(wl.groups, n, wl.vparams)
    return s0, mode, tgt, fleet, wl


def test_autograd_matches_central_differences():
    s0, mode, tgt, fleet, wl = small_problem()
    T, w = 40, 0.01
    L, li, dg, ds = ostep.loss_and_grad(s0, mode, tgt, fleet, wl.dt, wl.g, T, w)
    fdg, fds, kg, ks = ostep.fd_grad(s0, mode, tgt, fleet, wl.dt, wl.g, T, w, h=1e-5)
    ok_g, ok_s = ~kg, ~ks
    assert ok_g.float().mean() > 0.5 and ok_s.float().mean() > 0.5
    sg = dg.abs().max(-1, keepdim=True).values
    ss = ds.abs().max(-1, keepdim=True).values
    eg = ((dg - fdg).abs() / torch.maximum(fdg.abs(), 1e-3 * sg))[ok_g]
    es = ((ds - fds).abs() / torch.maximum(fds.abs(), 1e-3 * ss))[ok_s]
    assert eg.max() < 1e-5, eg.max()
    assert es.max() < 1e-5, es.max()


def test_directional_derivative_matches_vjp():
    s0, mode, tgt, fleet, wl = small_problem(n=4, seed=12, T=30)
    T, w = 30, 0.01
    L, _, dg, ds = ostep.loss_and_grad(s0, mode, tgt, fleet, wl.dt, wl.g, T, w)
    g = torch.Generator().manual_seed(3)
    dG = torch.randn(dg.shape, generator=g, dtype=F64)
    dS = torch.randn(ds.shape, generator=g, dtype=F64)
    h = 1e-6

    def Lof(eps):
        fl = fleet.with_gains(fleet.gains + eps * dG)
        li, _ = ostep.per_vehicle_loss(s0 + eps * dS, mode, tgt, fl, wl.dt, wl.g, T, w)
        return li.sum() / s0.shape[0]

    with torch.no_grad():
        fd = (Lof(h) - Lof(-h)) / (2 * h)
    vjp = (dg * dG).sum() + (ds * dS).sum()
    assert abs(float(fd - vjp)) <= 1e-6 * abs(float(vjp)) + 1e-10


def test_loss_is_sum_over_post_step_states():
    """L counts post-step states t = 1..T only: a zero-step rollout has loss 0 and
    a one-step rollout equals the error of the stepped state."""
    s0, mode, tgt, fleet, wl = small_problem(n=3, seed=13, T=1)
    li0, _ = ostep.per_vehicle_loss(s0, mode, tgt, fleet, wl.dt, wl.g, 0, 0.01)
    assert torch.equal(li0, torch.zeros(3, dtype=F64))
    li1, s1 = ostep.per_vehicle_loss(s0, mode, tgt, fleet, wl.dt, wl.g, 1, 0.01)
    ref = ((s1[:, :3] - tgt[:, :3]) ** 2).sum(-1) + 0.01 * (s1[:, 10:] ** 2).sum(-1)
    assert torch.equal(li1, ref)
