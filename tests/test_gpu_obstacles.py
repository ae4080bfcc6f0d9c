"""Obstacle pose randomisation at environment reset on the GPU against the
oracle: which rows change is bit-exact, poses within FP32 rounding."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import obstacles
from parity import need_gpu

pytestmark = pytest.mark.gpu

SLOTS = np.stack([
    obstacles.slot_row((0.1, 0.1, 0.0), (0.9, 0.9, 0.5), (-0.2, -0.2, -math.pi), (0.2, 0.2, math.pi)),
    obstacles.slot_row((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (0, 0, 0), (0, 0, 0), lock=(2, 5),
                       lock_val=(0, 0, 0.25, 0, 0, 1.0)),
    obstacles.slot_row((0.5, 0.2, 0.3), (0.5, 0.8, 0.7), (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0), lock=(0, 3),
                       lock_val=(0.75, 0, 0, 0.5, 0, 0)),
    obstacles.slot_row((0.2, 0.2, 0.2), (0.8, 0.8, 0.8), (-0.5, -0.5, -0.5), (0.5, 0.5, 0.5)),
])


@pytest.mark.parametrize("per_env_box", [False, True])
def test_obstacle_poses_match_oracle(per_env_box):
    need_gpu()
    from paper_2305_16510_amd.sim import Sim
    n = 4097
    wl = workloads.c1_parity(n=n, seed=70)
    wl.seed = 0x1234567890
    sim = Sim.from_workload(wl, index_base=11)
    rng = np.random.default_rng(71)
    lo = rng.uniform(-10, 0, (3, n)).astype(np.float32)
    hi = (lo + rng.uniform(1, 10, (3, n))).astype(np.float32)
    if not per_env_box:
        lo[:] = np.array([[-5.0], [-4.0], [0.0]], np.float32)
        hi[:] = np.array([[5.0], [4.0], [3.0]], np.float32)
    mask = (rng.random(n) < 0.3).astype(np.uint8)
    k = len(SLOTS)
    init = np.zeros((7, n * k), np.float32)
    init[3] = 1.0
    out = torch.as_tensor(init).cuda()
    if per_env_box:
        sim.randomize_obstacles(SLOTS, out, step=77, mask=torch.as_tensor(mask), env_lo=lo, env_hi=hi)
    else:
        sim.randomize_obstacles(SLOTS, out, step=77, mask=torch.as_tensor(mask), box_lo=(-5.0, -4.0, 0.0),
                                box_hi=(5.0, 4.0, 3.0))
    sim.sync()
    got = out.cpu().numpy().T.astype(np.float64)
    sim.close()
    ref = obstacles.randomize(lo.T, hi.T, SLOTS, mask.astype(bool), 77, wl.seed, np.arange(n) + 11,
                              init.T.astype(np.float64))
    changed = np.repeat(mask.astype(bool), k)
    assert np.array_equal(got[~changed], init.T[~changed])
    err = np.abs(got[changed] - ref[changed]).max()
    print("obstacle pose max abs err", err)
    assert err <= 4e-6
