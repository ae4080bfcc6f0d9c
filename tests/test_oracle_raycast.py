"""Pins of the oracle's depth ray casting: closed forms (on-axis sphere,
planes perpendicular to the optical axis, camera inside a sphere), rigid-
motion invariance, and brute-force ray marching with point-in-solid tests."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import raycast as rc

I_Q = np.array([1.0, 0.0, 0.0, 0.0])


def shapes(*rows):
    out = np.zeros((len(rows), rc.SHAPE_DIM))
    for k, r in enumerate(rows):
        out[k, :len(r)] = r
    return out


def one(pos, quat, sh, obst, floor=float("nan"), W=31, H=21, hfov=1.2, maxd=50.0, mp=(0, 0, 0), mq=I_Q):
    return rc.render(np.array([pos], float), np.array([quat], float), np.array(mp, float), np.array(mq, float),
                     sh, np.array([obst], float), floor, W, H, hfov, maxd)[0]


def test_on_axis_sphere_and_miss():
    d = one((0, 0, 0), I_Q, shapes((rc.SPHERE, 0.7)), [[5.0, 0, 0, 1, 0, 0, 0]])
    assert abs(d[10, 15] - 4.3) < 1e-12                     # odd W, H: centre pixel on the axis
    assert d[0, 0] == 50.0                                   # corner ray misses
    assert (d <= 50.0).all()


def test_planes_perpendicular_to_the_axis_have_constant_depth():
    # camera pitched to look straight down from height 2.5 onto the floor
    down = Rotation.from_euler("y", 90, degrees=True).as_quat()[[3, 0, 1, 2]]
    d = one((1.0, -2.0, 2.5), down, shapes((rc.BOX, 0.1, 0.1, 0.1)), [[100, 100, 100, 1, 0, 0, 0]], floor=0.0)
    np.testing.assert_allclose(d, 2.5, rtol=1e-12)
    # a large box face at x = 3 (box centred at 4, half extent 1) and a cylinder cap
    d = one((0, 0, 0), I_Q, shapes((rc.BOX, 1.0, 10.0, 10.0)), [[4.0, 0, 0, 1, 0, 0, 0]])
    np.testing.assert_allclose(d, 3.0, rtol=1e-12)
    cyl_q = Rotation.from_euler("y", 90, degrees=True).as_quat()[[3, 0, 1, 2]]     # axis along world x
    d = one((0, 0, 0), I_Q, shapes((rc.CYLINDER, 10.0, 0.5)), [[6.0, 0, 0, *cyl_q]])
    np.testing.assert_allclose(d, 5.5, rtol=1e-12)


def test_camera_inside_sphere_sees_the_exit():
    W, H, hfov = 15, 11, 1.0
    d = one((0, 0, 0), I_Q, shapes((rc.SPHERE, 2.0)), [[0, 0, 0, 1, 0, 0, 0]], W=W, H=H, hfov=hfov)
    np.testing.assert_allclose(d, 2.0 * rc.camera_rays(W, H, hfov)[..., 0], rtol=1e-12)


def test_rigid_motion_invariance_and_mount():
    rng = np.random.default_rng(0)
    sh = shapes((rc.BOX, 0.5, 0.3, 0.8), (rc.SPHERE, 0.6), (rc.CYLINDER, 0.4, 0.9))
    obst = np.zeros((3, 7))
    obst[:, 0:3] = rng.uniform(2, 6, (3, 3)) * np.array([1, 0.3, 0.3])
    obst[:, 3:7] = Rotation.random(3, random_state=1).as_quat()[:, [3, 0, 1, 2]]
    pos = np.array([0.1, -0.2, 0.3])
    quat = Rotation.from_euler("ZYX", [0.15, -0.1, 0.2]).as_quat()[[3, 0, 1, 2]]
    mp, mq = (0.1, 0.0, -0.05), Rotation.from_euler("y", 10, degrees=True).as_quat()[[3, 0, 1, 2]]
    base = one(pos, quat, sh, obst, mp=mp, mq=mq)
    G = Rotation.random(random_state=3)
    c = np.array([3.0, -1.0, 2.0])
    Gq = G.as_quat()[[3, 0, 1, 2]]

    def qmul(a, b):
        return (Rotation.from_quat(a[[1, 2, 3, 0]]) * Rotation.from_quat(b[[1, 2, 3, 0]])).as_quat()[[3, 0, 1, 2]]
    obst2 = obst.copy()
    obst2[:, 0:3] = G.apply(obst[:, 0:3]) + c
    obst2[:, 3:7] = np.stack([qmul(Gq, q) for q in obst[:, 3:7]])
    moved = one(G.apply(pos) + c, qmul(Gq, quat), sh, obst2, mp=mp, mq=mq)
    np.testing.assert_allclose(moved, base, rtol=1e-9, atol=1e-9)
    assert (base < 50).any() and (base == 50).any()


def inside(p, typ, dims):
    if typ == rc.BOX:
        return np.all(np.abs(p) <= dims[:3], -1)
    if typ == rc.SPHERE:
        return (p * p).sum(-1) <= dims[0] ** 2
    return (p[..., 0] ** 2 + p[..., 1] ** 2 <= dims[0] ** 2) & (np.abs(p[..., 2]) <= dims[1])


def test_brute_force_ray_marching():
    """March each ray in steps of 1e-3 and take the first point inside any
    solid: the cast depth agrees within one step (rays near silhouettes,
    where the first crossing is shorter than a step, are skipped)."""
    rng = np.random.default_rng(5)
    sh = shapes((rc.BOX, 0.5, 0.3, 0.8), (rc.SPHERE, 0.6), (rc.CYLINDER, 0.4, 0.9), (rc.CYLINDER, 0.2, 0.3))
    obst = np.zeros((4, 7))
    obst[:, 0:3] = np.array([[3.0, 0.5, 0.2], [4.0, -0.6, -0.3], [2.5, -0.2, 0.6], [2.0, 0.4, -0.5]])
    obst[:, 3:7] = Rotation.random(4, random_state=6).as_quat()[:, [3, 0, 1, 2]]
    W, H, hfov, maxd = 17, 13, 1.3, 8.0
    d = one((0, 0, 0), I_Q, sh, obst, W=W, H=H, hfov=hfov, maxd=maxd)
    dirs = rc.camera_rays(W, H, hfov).reshape(-1, 3)
    step = 1e-3
    ts = np.arange(step, maxd / 0.5, step)
    checked = 0
    for idx in rng.choice(len(dirs), 60, replace=False):
        pts = ts[:, None] * dirs[idx]
        hit = np.zeros(len(ts), bool)
        for k in range(4):
            R = rc.quat_to_rot(obst[k, 3:7])
            loc = (pts - obst[k, :3]) @ R
            hit |= inside(loc, int(sh[k, 0]), sh[k, 1:])
        first = ts[np.argmax(hit)] if hit.any() else np.inf
        depth = first * dirs[idx, 0] if np.isfinite(first) and first * dirs[idx, 0] <= maxd else maxd
        ref = d.reshape(-1)[idx]
        if hit.any() and hit.sum() < 20:
            continue               # grazing ray
        assert abs(depth - ref) <= step + 1e-12, (idx, depth, ref)
        checked += 1
    assert checked > 40
