"""Fused launches in mode order against plain per-step launches, bitwise.

A fused call of 32 or more steps (one vehicle per lane) first lists the
vehicles of every group within each segment of 4,096 by command mode, so
that wavefronts hold one mode and run that mode's copy of the step loop.
Each lane then steps the vehicle the order assigns to it.  These tests check
that this changes no bit of any vehicle's trajectory:

* mixed modes including the wrench mode and invalid codes, over uneven
  groups that straddle segments, with a ragged last segment;
* segments cut by more groups than the order handles (listed in index order);
* modes rewritten between calls, through ag_set_targets and by writing the
  bound mode buffer directly;
* fleets of a single mode;
* calls shorter than the threshold (no order) mixed with longer ones.
"""
import numpy as np
import pytest
import torch

import workloads
from parity import need_gpu

pytestmark = pytest.mark.gpu

MODES = np.array([0, 1, 2, 3, -2, 9], np.int8)


def mixed_commands(n, seed, p=(0.3, 0.3, 0.3, 0.04, 0.03, 0.03)):
    """Per-vehicle modes drawn from MODES and finite commands for each."""
    rng = np.random.default_rng(seed)
    mode = rng.choice(MODES, size=n, p=p).astype(np.int8)
    tgt = np.zeros((4, n), np.float32)
    m1, m2, m3 = mode == 1, mode == 2, mode == 3
    tgt[:3, m1] = rng.uniform(-2, 2, (3, int(m1.sum())))
    tgt[0, m2] = rng.uniform(-0.3, 0.3, int(m2.sum()))
    tgt[1, m2] = rng.uniform(-0.3, 0.3, int(m2.sum()))
    tgt[2, m2] = rng.uniform(-1, 1, int(m2.sum()))
    tgt[3, m2] = rng.uniform(5, 15, int(m2.sum()))
    tgt[0, m3] = rng.uniform(5, 15, int(m3.sum()))
    tgt[1:, m3] = rng.uniform(-0.05, 0.05, (3, int(m3.sum())))
    return mode, tgt


def with_commands(wl, seed):
    mode, tgt = mixed_commands(wl.n, seed)
    wl.mode = mode
    wl.target = tgt
    return wl


def run_pair(wl, steps_fused, block=64, between=None):
    """Final states of the same call sequence under a fused policy and under
    per-step launches; `between(sim, j)` runs after call j."""
    from paper_2305_16510_amd.sim import Sim
    out = []
    for kind in (1, 0):
        sim = Sim.from_workload(wl)
        if kind == 1:
            sim.set_exec(kind=1, block=block, vpl=1, k=16, grid=0, use_graph=1)
        else:
            sim.set_exec(kind=0, block=block, use_graph=0)
        for j, n in enumerate(steps_fused):
            sim.step(n)
            if between:
                between(sim, j)
        sim.sync()
        out.append(sim.state.clone())
        sim.close()
    return out


def test_mixed_modes_uneven_groups_ragged():
    need_gpu()
    wl = with_commands(workloads.c3_uneven(scale=0.05, seed=41), seed=42)   # ~60k vehicles, 48 groups
    assert wl.n % 4096 != 0
    fused, plain = run_pair(wl, [48])
    assert torch.equal(fused, plain)
    assert torch.isfinite(fused).all()


def test_segments_with_many_groups():
    need_gpu()
    # log-uniform group sizes 1..4000: some segments hold more than 8 groups
    wl = with_commands(workloads.c3_uneven(n_groups=300, size_lo=1, size_hi=4000, seed=43), seed=44)
    starts = np.array([g.first for g in wl.groups])
    per_seg = np.bincount(starts // 4096)
    assert per_seg.max() > 8 and (per_seg[per_seg > 0] <= 7).any()
    fused, plain = run_pair(wl, [40])
    assert torch.equal(fused, plain)


@pytest.mark.parametrize("direct_write", [False, True])
def test_modes_rewritten_between_calls(direct_write):
    need_gpu()
    wl = with_commands(workloads.c1_parity(n=20_000, seed=45), seed=46)
    mode2, tgt2 = mixed_commands(wl.n, 47)

    def between(sim, j):
        if j != 0:
            return
        if direct_write:
            sim.mode.copy_(torch.from_numpy(mode2))
            sim.target.copy_(torch.from_numpy(tgt2))
            sim.set_targets(0, sim.n)          # re-derives the cached commands
        else:
            sim.set_targets(0, sim.n, mode=torch.from_numpy(mode2), target=torch.from_numpy(tgt2))

    fused, plain = run_pair(wl, [40, 5, 64], between=between)
    assert torch.equal(fused, plain)


@pytest.mark.parametrize("m", [0, 1, 2])
def test_single_mode_fleets(m):
    need_gpu()
    wl = with_commands(workloads.c1_parity(n=70_000, seed=48), seed=49)
    keep = wl.mode == m
    wl.mode[:] = m
    _, tgt = mixed_commands(wl.n, 50, p=(1, 0, 0, 0, 0, 0) if m == 0 else
                            ((0, 1, 0, 0, 0, 0) if m == 1 else (0, 0, 1, 0, 0, 0)))
    wl.target = np.where(keep[None, :], wl.target, tgt).astype(np.float32)
    fused, plain = run_pair(wl, [33, 31, 100], block=256)
    assert torch.equal(fused, plain)
