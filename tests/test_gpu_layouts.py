"""Allocation of every rotor layout away from the default geometry.

Quad, hexa and octo groups with small and large arms and yaw-torque
coefficients (c_tau from 1e-3 to 0.3 m), mixed command modes: the commanded
and applied wrench of the GPU's quad butterflies and hexa / octo pair forms
stay within 1e-5 of the FP64 oracle (relative, floors m g and m g l; vehicles
with a raw rotor command within 1e-4 u_max of a clamp bound excluded), and
fused launches in mode order equal per-step launches bitwise.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from parity import need_gpu, oracle_inputs, to_vm64, wrench_errors, near_clamp
from test_gpu_order import mixed_commands

pytestmark = pytest.mark.gpu

LAYOUTS = [(4, 0.05, 1e-3), (4, 1.5, 0.3), (6, 0.05, 1e-3), (6, 1.5, 0.3), (8, 0.05, 1e-3), (8, 1.5, 0.3)]


def layout_fleet(count=700, seed=60):
    groups, first = [], 0
    for nr, arm, ctau in LAYOUTS:
        groups.append(workloads.Group(first, count, n_rotors=nr, arm=arm, c_tau=ctau, u_max=24.0 / nr))
        first += count
    rng = np.random.default_rng(seed)
    s0 = workloads.random_initial_state(rng, first)
    mode, tgt = mixed_commands(first, seed + 1, p=(0.3, 0.3, 0.3, 0.1, 0.0, 0.0))
    return workloads.Workload("layouts", first, 0.01, 30, groups, s0, mode, tgt, seed=seed)


def test_wrench_parity_across_layouts():
    need_gpu()
    from paper_2305_16510_amd.sim import Sim
    wl = layout_fleet()
    sim = Sim.from_workload(wl, outputs=True)
    sim.set_exec(kind=0, block=64, use_graph=0)
    _, mode, tgt, fleet = oracle_inputs(wl)
    worst = torch.zeros(4, dtype=torch.float64)
    excluded = 0
    for t in range(30):
        pre = to_vm64(sim.state)
        sim.step(1)
        if t % 5:
            continue
        _, info = oracle.step.step(pre, mode, tgt, fleet, wl.dt, wl.g)
        near = near_clamp(info, fleet)
        excluded += int(near.sum())
        errs = wrench_errors(to_vm64(sim.wrench), info, fleet, wl.g, near_kink=near)
        worst = torch.maximum(worst, torch.stack([e.max() for e in errs]))
    sim.close()
    print("layouts: max rel err f, M, f', M':", worst.tolist(), "excluded near a clamp:", excluded)
    assert worst.max() <= 1e-5


def test_fused_in_mode_order_equals_per_step_across_layouts():
    need_gpu()
    from paper_2305_16510_amd.sim import Sim
    wl = layout_fleet(count=5000, seed=61)
    out = []
    for kind in (1, 0):
        sim = Sim.from_workload(wl)
        if kind:
            sim.set_exec(kind=1, block=128, vpl=1, k=20, grid=0, use_graph=1)
        else:
            sim.set_exec(kind=0, block=128, use_graph=0)
        sim.step(60)
        sim.sync()
        out.append(sim.state.clone())
        sim.close()
    assert torch.equal(out[0], out[1])
