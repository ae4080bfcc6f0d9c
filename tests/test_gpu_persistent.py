"""Persistent fused launches (fewer blocks than tiles: each block strides over
the tiles) against plain per-step launches, bitwise: mixed command modes in
mode order, calls too short for the order, per-vehicle parameters over
uneven groups with all three rotor layouts, a single rotor class with
per-vehicle parameters, observers (wrench and rotor outputs, flags,
statistics), a ragged last tile and few tiles per block."""
import numpy as np
import pytest
import torch

import workloads
from parity import need_gpu

pytestmark = pytest.mark.gpu


def run(wl, policy, calls, **kw):
    from paper_2305_16510_amd.sim import Sim
    sim = Sim.from_workload(wl, **kw)
    sim.set_exec(**policy)
    for n in calls:
        sim.step(n)
    sim.sync()
    out = [sim.state.clone()]
    if sim.wrench is not None:
        out += [sim.wrench.clone(), sim.rotors.clone(), sim.flags.clone()]
    st = sim.stats() if kw.get("collect_stats") else None
    sim.close()
    return out, st


PLAIN = dict(kind=0, block=256, use_graph=0)


@pytest.mark.parametrize("block,grid,k", [(64, 8, 16), (256, 24, 40), (512, 13, 7), (128, 200, 64)])
def test_mixed_modes_in_mode_order(block, grid, k):
    need_gpu()
    wl = workloads.c2_scale(n=100_003, seed=71)
    ref, _ = run(wl, PLAIN, [45, 3])
    got, _ = run(wl, dict(kind=1, block=block, vpl=1, k=k, grid=grid, use_graph=1), [45, 3])
    assert torch.equal(got[0], ref[0])


def test_short_calls_without_order():
    need_gpu()
    wl = workloads.c2_scale(n=30_001, seed=72)
    ref, _ = run(wl, PLAIN, [5, 9, 2])
    got, _ = run(wl, dict(kind=1, block=64, vpl=1, k=4, grid=16, use_graph=1), [5, 9, 2])
    assert torch.equal(got[0], ref[0])


@pytest.mark.parametrize("grid", [16, 40])
def test_uneven_groups_with_per_vehicle_parameters(grid):
    need_gpu()
    wl = workloads.c3_uneven(scale=0.02, seed=73)         # 48 groups, ~20k vehicles, 4/6/8 rotors
    assert sorted(set(g.n_rotors for g in wl.groups)) == [4, 6, 8]
    ref, _ = run(wl, PLAIN, [33])
    got, _ = run(wl, dict(kind=1, block=128, vpl=1, k=11, grid=grid, use_graph=1), [33])
    assert torch.equal(got[0], ref[0])


def test_single_rotor_class_with_per_vehicle_parameters():
    need_gpu()
    wl = workloads.c4_grad(n=50_000, seed=74, steps=40)
    ref, _ = run(wl, PLAIN, [40])
    got, _ = run(wl, dict(kind=1, block=256, vpl=1, k=40, grid=32, use_graph=1), [40])
    assert torch.equal(got[0], ref[0])


def test_observers_and_statistics():
    need_gpu()
    wl = workloads.c2_scale(n=40_961, seed=75)
    ref, st_ref = run(wl, PLAIN, [20, 12], outputs=True, collect_stats=True)
    got, st = run(wl, dict(kind=1, block=256, vpl=1, k=8, grid=24, use_graph=1), [20, 12], outputs=True,
                  collect_stats=True)
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    for key in ("steps", "n_saturated", "n_nonfinite", "n_finite", "n_position"):
        assert st[key] == st_ref[key], key
    assert abs(st["pos_err_sum"] - st_ref["pos_err_sum"]) <= 1e-9 * abs(st_ref["pos_err_sum"])


def test_few_tiles_per_xcd():
    """79 tiles over 72 blocks: most blocks step one tile, seven step two."""
    need_gpu()
    wl = workloads.c2_scale(n=5_000, seed=76)             # 79 tiles of 64
    ref, _ = run(wl, PLAIN, [40])
    got, _ = run(wl, dict(kind=1, block=64, vpl=1, k=10, grid=72, use_graph=1), [40])
    assert torch.equal(got[0], ref[0])
