"""Depth images by ray casting against primitive obstacles, FP64 (oracle;
test infrastructure only).

The paper renders depth with its engine's camera (Sec. III, VI) and names
kernel-based ray casting as future work (Sec. I, VII).  Definition used here
(reading R31): a pinhole camera mounted on each vehicle (mount position and
attitude in the body frame), x forward, y left, z up; pixel (u, v) of a W x H
image (centres at u + 1/2, v + 1/2) looks along
d_c = normalize(1, -(u + 1/2 - W/2)/f, -(v + 1/2 - H/2)/f), f = (W/2)/tan(hfov/2).
The depth of a pixel is t * d_c.x for the smallest t > 0 at which the ray
enters an obstacle (box, sphere or capped cylinder in its own pose) or meets
the floor plane z = floor from above, or max_depth when there is no hit or
the depth exceeds max_depth.  A ray starting inside an obstacle reports the
exit point.

Obstacle shape rows (8 floats): type (0 box, 1 sphere, 2 cylinder along the
body z axis), then box half extents (hx, hy, hz) / sphere radius / cylinder
radius and half height.
"""
import math

import numpy as np

BOX, SPHERE, CYLINDER = 0, 1, 2
SHAPE_DIM = 8


def quat_to_rot(q):
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def camera_rays(W, H, hfov):
    """Unit ray directions in the camera frame, [H, W, 3]."""
    f = (W / 2) / math.tan(hfov / 2)
    u = np.arange(W) + 0.5
    v = np.arange(H) + 0.5
    U, V = np.meshgrid(u, v)
    d = np.stack([np.ones_like(U), -(U - W / 2) / f, -(V - H / 2) / f], -1)
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def _first_positive(t_in, t_out, hit):
    """Entry if it lies ahead, else exit if ahead (origin inside), else miss."""
    t = np.where(t_in > 0, t_in, np.where(t_out > 0, t_out, np.inf))
    return np.where(hit, t, np.inf)


def hit_box(o, d, h):
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t1 = (-h - o) * inv
        t2 = (h - o) * inv
    tn = np.max(np.minimum(t1, t2), -1)
    tf = np.min(np.maximum(t1, t2), -1)
    return _first_positive(tn, tf, tn <= tf)


def hit_sphere(o, d, r):
    b = (o * d).sum(-1)
    c = (o * o).sum(-1) - r * r
    disc = b * b - c
    s = np.sqrt(np.maximum(disc, 0.0))
    return _first_positive(-b - s, -b + s, disc >= 0)


def hit_cylinder(o, d, r, hh):
    a = d[..., 0] ** 2 + d[..., 1] ** 2
    b = o[..., 0] * d[..., 0] + o[..., 1] * d[..., 1]
    c = o[..., 0] ** 2 + o[..., 1] ** 2 - r * r
    disc = b * b - a * c
    s = np.sqrt(np.maximum(disc, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        # infinite cylinder interval (all t when the ray is parallel to the axis and inside)
        ts_in = np.where(a > 0, (-b - s) / a, np.where(c <= 0, -np.inf, np.inf))
        ts_out = np.where(a > 0, (-b + s) / a, np.where(c <= 0, np.inf, -np.inf))
        side_ok = (a > 0) & (disc >= 0) | (a == 0) & (c <= 0)
        t1 = (-hh - o[..., 2]) / d[..., 2]
        t2 = (hh - o[..., 2]) / d[..., 2]
    tz_in = np.where(d[..., 2] != 0, np.minimum(t1, t2), np.where(np.abs(o[..., 2]) <= hh, -np.inf, np.inf))
    tz_out = np.where(d[..., 2] != 0, np.maximum(t1, t2), np.where(np.abs(o[..., 2]) <= hh, np.inf, -np.inf))
    tn = np.maximum(ts_in, tz_in)
    tf = np.minimum(ts_out, tz_out)
    return _first_positive(tn, tf, side_ok & (tn <= tf))


def render(pos, quat, mount_p, mount_q, shapes, obst, floor_z, W, H, hfov, max_depth):
    """Depth images [n, H, W] for vehicles at (pos [n,3], quat [n,4]) with
    obstacles obst [n, n_obs, 7] (x, y, z, qw, qx, qy, qz) of the given shapes."""
    n = pos.shape[0]
    dc = camera_rays(W, H, hfov)                                  # [H,W,3]
    Rb = quat_to_rot(np.asarray(quat, np.float64))                 # [n,3,3]
    Rm = quat_to_rot(np.asarray(mount_q, np.float64))
    Rwc = Rb @ Rm
    org = pos + np.einsum("nij,j->ni", Rb, np.asarray(mount_p, np.float64))
    dw = np.einsum("nij,hwj->nhwi", Rwc, dc)                       # [n,H,W,3]
    o = np.broadcast_to(org[:, None, None, :], dw.shape)
    t = np.full(dw.shape[:-1], np.inf)
    if floor_z is not None and not math.isnan(floor_z):
        with np.errstate(divide="ignore", invalid="ignore"):
            tp = (floor_z - o[..., 2]) / dw[..., 2]
        t = np.minimum(t, np.where((dw[..., 2] < 0) & (o[..., 2] > floor_z) & (tp > 0), tp, np.inf))
    for k in range(shapes.shape[0]):
        typ = int(shapes[k, 0])
        c = obst[:, k, 0:3]
        R = quat_to_rot(obst[:, k, 3:7])
        ol = np.einsum("nji,nhwj->nhwi", R, o - c[:, None, None, :])
        dl = np.einsum("nji,nhwj->nhwi", R, dw)
        if typ == BOX:
            tk = hit_box(ol, dl, shapes[k, 1:4])
        elif typ == SPHERE:
            tk = hit_sphere(ol, dl, shapes[k, 1])
        else:
            tk = hit_cylinder(ol, dl, shapes[k, 1], shapes[k, 2])
        t = np.minimum(t, tk)
    depth = t * dc[None, :, :, 0]
    return np.where(np.isfinite(depth) & (depth <= max_depth), depth, max_depth)
