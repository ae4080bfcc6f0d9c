"""Depth ray casting on the GPU against the FP64 oracle."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import workloads
from oracle import obstacles, raycast
from parity import need_gpu

pytestmark = pytest.mark.gpu


def scene(n, n_obs, seed):
    rng = np.random.default_rng(seed)
    shapes = np.zeros((n_obs, 8), np.float32)
    shapes[:, 0] = np.arange(n_obs) % 3
    shapes[:, 1] = rng.uniform(0.2, 0.8, n_obs)
    shapes[:, 2] = rng.uniform(0.2, 0.8, n_obs)
    shapes[:, 3] = rng.uniform(0.2, 0.8, n_obs)
    slots = np.stack([obstacles.slot_row((0.55, 0.05, 0.1), (0.95, 0.95, 0.9), (-1, -1, -math.pi), (1, 1, math.pi))
                      for _ in range(n_obs)])
    return shapes, slots


def compare(gpu, ref, maxd):
    """Per-pixel relative depth error.  Pixels off by more than 1e-4 may only
    sit at silhouettes (an oracle neighbour differs by more than 2%), where a
    grazing ray can hit in one precision and miss in the other.  Returns the
    largest error, the fraction of mismatched pixels and the number of
    mismatches away from silhouettes."""
    g = gpu.astype(np.float64)
    pad = np.pad(ref, ((0, 0), (1, 1), (1, 1)), mode="edge")
    nb = np.stack([pad[:, :-2, 1:-1], pad[:, 2:, 1:-1], pad[:, 1:-1, :-2], pad[:, 1:-1, 2:]])
    edge = (np.abs(nb - ref[None]) > 0.02 * ref[None]).any(0)
    err = np.abs(g - ref) / np.maximum(ref, 1e-6)
    mism = err > 1e-4
    return err[~edge].max(), mism.mean(), int((mism & ~edge).sum())


def render_case(n, n_obs, W, H, seed, floor=0.0):
    from paper_2305_16510_amd.sim import Sim
    wl = workloads.c1_parity(n=n, seed=seed)
    wl.state0[0:3] = np.array([[0.5], [5.0], [1.5]], np.float32) + wl.state0[0:3] * 0.2
    sim = Sim.from_workload(wl)
    shapes, slots = scene(n, n_obs, seed)
    obst = torch.zeros(7, n * n_obs, device="cuda")
    obst[3] = 1.0
    sim.randomize_obstacles(slots, obst, step=1, box_lo=(0.0, 0.0, 0.0), box_hi=(10.0, 10.0, 3.0))
    mount_q = Rotation.from_euler("y", 8, degrees=True).as_quat()[[3, 0, 1, 2]]
    depth = sim.render_depth(shapes, obst, W, H, 1.5, 10.0, floor_z=floor, mount_pos=(0.1, 0.0, 0.05),
                             mount_quat=tuple(mount_q))
    sim.sync()
    st = sim.state.cpu().numpy().T.astype(np.float64)
    ob = obst.cpu().numpy().T.astype(np.float64).reshape(n, n_obs, 7)
    d = depth.cpu().numpy()
    sim.close()
    return d, st, ob, shapes, mount_q


def test_depth_images_match_oracle():
    need_gpu()
    n, n_obs, W, H = 12, 15, 96, 54
    d, st, ob, shapes, mq = render_case(n, n_obs, W, H, 80)
    ref = raycast.render(st[:, 0:3], st[:, 6:10], np.array([0.1, 0.0, 0.05]), mq, shapes.astype(np.float64),
                         ob, 0.0, W, H, 1.5, 10.0)
    emax, mism, off_edge = compare(d, ref, 10.0)
    print("depth: max rel err off silhouettes %.2e, mismatched pixels %.3f%%, mismatches off silhouettes %d" %
          (emax, 100 * mism, off_edge))
    assert emax <= 1e-4 and mism < 0.005 and off_edge == 0
    assert ((ref < 10.0).mean() > 0.2) and ((ref == 10.0).mean() > 0.01)


def test_full_resolution_sampled_cameras():
    """2^10 vehicles with 270 x 480 depth cameras (the paper's camera
    benchmark shape); 4 sampled cameras checked against the oracle."""
    need_gpu()
    n, n_obs, W, H = 1024, 20, 480, 270
    d, st, ob, shapes, mq = render_case(n, n_obs, W, H, 81)
    idx = np.array([0, 333, 700, 1023])
    ref = raycast.render(st[idx, 0:3], st[idx, 6:10], np.array([0.1, 0.0, 0.05]), mq, shapes.astype(np.float64),
                         ob[idx], 0.0, W, H, 1.5, 10.0)
    emax, mism, off_edge = compare(d[idx], ref, 10.0)
    print("full res: max rel err off silhouettes %.2e, mismatched pixels %.3f%%" % (emax, 100 * mism))
    assert emax <= 1e-4 and mism < 0.005 and off_edge == 0


@pytest.mark.parametrize("maxd", [2.5, 10.0])
def test_tile_culling_short_range_and_inside_obstacles(maxd):
    """Cases aimed at the per-tile obstacle culling: a short max_depth (most
    obstacles lie beyond it and are culled by depth) and cameras inside an
    obstacle (vehicles 0 and 1 sit at the centre of one of their obstacles,
    so the tile cone starts inside a bounding sphere)."""
    need_gpu()
    from paper_2305_16510_amd.sim import Sim
    n, n_obs, W, H = 8, 20, 128, 64
    wl = workloads.c1_parity(n=n, seed=82)
    wl.state0[0:3] = np.array([[0.5], [5.0], [1.5]], np.float32) + wl.state0[0:3] * 0.2
    sim = Sim.from_workload(wl)
    shapes, slots = scene(n, n_obs, 82)
    obst = torch.zeros(7, n * n_obs, device="cuda")
    obst[3] = 1.0
    sim.randomize_obstacles(slots, obst, step=3, box_lo=(0.0, 0.0, 0.0), box_hi=(10.0, 10.0, 3.0))
    for i in (0, 1):
        sim.state[0:3, i] = obst[0:3, i * n_obs + 3 * i]
    mount_q = Rotation.from_euler("y", 8, degrees=True).as_quat()[[3, 0, 1, 2]]
    depth = sim.render_depth(shapes, obst, W, H, 1.5, maxd, floor_z=0.0, mount_pos=(0.1, 0.0, 0.05),
                             mount_quat=tuple(mount_q))
    sim.sync()
    st = sim.state.cpu().numpy().T.astype(np.float64)
    ob = obst.cpu().numpy().T.astype(np.float64).reshape(n, n_obs, 7)
    d = depth.cpu().numpy()
    sim.close()
    ref = raycast.render(st[:, 0:3], st[:, 6:10], np.array([0.1, 0.0, 0.05]), mount_q, shapes.astype(np.float64),
                         ob, 0.0, W, H, 1.5, maxd)
    emax, mism, off_edge = compare(d, ref, maxd)
    print("max_depth %.1f: max rel err off silhouettes %.2e, mismatched pixels %.3f%%, at max_depth %.1f%%" %
          (maxd, emax, 100 * mism, 100 * (ref == maxd).mean()))
    assert emax <= 1e-4 and mism < 0.005 and off_edge == 0
    assert (ref[0:2] < maxd).mean() > 0.5          # the cameras inside obstacles see their walls
