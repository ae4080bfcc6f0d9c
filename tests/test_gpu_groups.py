"""Uneven vehicle groups (quad, hexa and octo layouts; per-vehicle mass,
inertia, gains, arm and rotor limit) in one launch, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from parity import need_gpu, oracle_inputs, to_vm64, wrench_errors, near_clamp

pytestmark = pytest.mark.gpu
F64 = torch.float64


def make_sim(wl, **kw):
    from paper_2305_16510_amd.sim import Sim
    return Sim.from_workload(wl, **kw)


def test_uneven_groups_wrench_and_trajectory_parity():
    need_gpu()
    wl = workloads.c3_uneven(scale=0.006, seed=31)       # 48 groups, sizes ~3..800, ragged
    assert sorted(set(g.n_rotors for g in wl.groups)) == [4, 6, 8]
    sim = make_sim(wl, outputs=True)
    sim.set_exec(kind=0, block=128, use_graph=0)
    pres, ws = [], []
    for t in range(60):
        pres.append(sim.state.clone())
        sim.step(1)
        ws.append(sim.wrench.clone())
    sim.set_exec(kind=1, block=64, vpl=2, k=20, use_graph=1)
    sim.step(140)
    sim.sync()
    final = to_vm64(sim.state)
    sim.close()
    s0, mode, tgt, fleet = oracle_inputs(wl)
    worst = torch.zeros(4, dtype=F64)
    for t in range(0, 60, 6):
        pre = to_vm64(pres[t])
        _, info = oracle.step.step(pre, mode, tgt, fleet, wl.dt, wl.g)
        errs = wrench_errors(to_vm64(ws[t]), info, fleet, wl.g, near_kink=near_clamp(info, fleet))
        worst = torch.maximum(worst, torch.stack([e.max() for e in errs]))
    print("uneven groups: max rel err f, M, f', M':", worst.tolist())
    assert worst.max() <= 1e-5
    ref, _, _ = oracle.step.rollout(s0, mode, tgt, fleet, wl.dt, wl.g, 200)
    dx = (final[:, :3] - ref[:, :3]).norm(dim=-1)
    print("uneven groups: position error after 200 steps max %.3e p99 %.3e" % (dx.max(), dx.quantile(0.99)))
    assert dx.max() <= 1e-4


def test_group_alone_equals_group_in_batch():
    """A group simulated on its own (its own handle, rotor-count-specialised
    kernel) is bitwise identical to the same group inside the mixed batch."""
    need_gpu()
    wl = workloads.c3_uneven(scale=0.006, seed=32)
    sim = make_sim(wl)
    sim.set_exec(kind=1, block=128, vpl=1, k=25, use_graph=1)
    sim.step(100)
    sim.sync()
    full = sim.state.clone()
    sim.close()
    for gi in (0, 7, 23, 47):
        gr = wl.groups[gi]
        sl = slice(gr.first, gr.first + gr.count)
        alone = workloads.Workload("alone", gr.count, wl.dt, 100,
                                   [workloads.Group(0, gr.count, gr.n_rotors, gr.arm, gr.c_tau, gr.u_min,
                                                    gr.u_max, gr.mass, gr.inertia, gr.gains)],
                                   np.ascontiguousarray(wl.state0[:, sl]), wl.mode[sl].copy(),
                                   np.ascontiguousarray(wl.target[:, sl]),
                                   np.ascontiguousarray(wl.vparams[:, sl]), wl.g, wl.seed)
        s2 = make_sim(alone)
        s2.set_exec(kind=1, block=64, vpl=2, k=10, use_graph=1)
        s2.step(100)
        s2.sync()
        assert torch.equal(s2.state, full[:, sl]), gi
        s2.close()


def test_full_size_uneven_fleet_sampled_parity():
    """The full 48-group fleet (~1.1M vehicles) in the tuned fused launch,
    checked on sampled vehicles against the oracle run one by one."""
    need_gpu()
    wl = workloads.c3_uneven()
    sim = make_sim(wl, autotune_scratch=True)
    sim.autotune(32)
    sim.step(100)
    sim.sync()
    gpu = to_vm64(sim.state)
    sim.close()
    rng = np.random.default_rng(0)
    idx = np.sort(np.concatenate([rng.choice(wl.n, 200, replace=False),
                                  [g.first for g in wl.groups], [wl.n - 1]]))
    s0, mode, tgt, fleet = oracle_inputs(wl)
    it = torch.as_tensor(idx)
    ref, _, _ = oracle.step.rollout(s0[it], mode[it], tgt[it], fleet.select(it), wl.dt, wl.g, 100)
    dx = (gpu[it, :3] - ref[:, :3]).norm(dim=-1)
    print("full uneven fleet: %d vehicles, sampled position error max %.3e" % (wl.n, dx.max()))
    assert dx.max() <= 1e-4


def test_full_size_uneven_fleet_2000_steps_light_and_heavy():
    """The full 48-group fleet for the configuration's 2,000 steps in the
    tuned fused launch, against the oracle run one by one on sampled vehicles:
    random ones, the 20 lightest and 20 heaviest (mass 0.5 and 3 kg ends of the
    mass-scaled parameters), and the first vehicle of every group.  Closed-loop
    position control damps the FP32 rounding: positions agree within 1e-4 m
    and attitudes (rotation matrices) within 1e-4."""
    need_gpu()
    from parity import same_rotation_err
    wl = workloads.c3_uneven()
    sim = make_sim(wl, autotune_scratch=True)
    sim.autotune(512)
    sim.step(wl.steps)
    sim.sync()
    gpu = to_vm64(sim.state)
    sim.close()
    mass = wl.vparams[0].astype(np.float64)
    order = np.argsort(mass, kind="stable")
    rng = np.random.default_rng(1)
    idx = np.unique(np.concatenate([rng.choice(wl.n, 120, replace=False), order[:20], order[-20:],
                                    [g.first for g in wl.groups], [wl.n - 1]]))
    s0, mode, tgt, fleet = oracle_inputs(wl)
    it = torch.as_tensor(idx)
    ref, _, _ = oracle.step.rollout(s0[it], mode[it], tgt[it], fleet.select(it), wl.dt, wl.g, wl.steps)
    dx = (gpu[it, :3] - ref[:, :3]).norm(dim=-1)
    dR = same_rotation_err(gpu[it, 6:10], ref[:, 6:10])
    light, heavy = np.isin(idx, order[:20]), np.isin(idx, order[-20:])
    print("2,000 steps, %d sampled vehicles: position error max %.3e (lightest %.3e, heaviest %.3e), "
          "attitude max %.3e; masses %.3f..%.3f"
          % (len(idx), dx.max(), dx[light].max(), dx[heavy].max(), dR.max(), mass[order[0]], mass[order[-1]]))
    assert light.sum() == 20 and heavy.sum() == 20
    assert dx.max() <= 1e-4 and dR.max() <= 1e-4
