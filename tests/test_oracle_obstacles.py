"""Pins of the oracle's obstacle pose randomisation (Sec. V): attitudes
against scipy's Z-Y-X Euler conversion, bounds, locked dimensions, masks,
sharding invariance."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import obstacles

SLOTS = np.stack([
    obstacles.slot_row((0.1, 0.1, 0.0), (0.9, 0.9, 0.5), (-0.2, -0.2, -math.pi), (0.2, 0.2, math.pi)),
    obstacles.slot_row((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (0, 0, 0), (0, 0, 0), lock=(2, 5), lock_val=(0, 0, 0.25, 0, 0, 1.0)),
    obstacles.slot_row((0.5, 0.2, 0.3), (0.5, 0.8, 0.7), (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0), lock=(0, 3), lock_val=(0.75, 0, 0, 0.5, 0, 0)),
])


def setup(n_env=500, seed=3):
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-10, 0, (n_env, 3))
    hi = lo + rng.uniform(1, 10, (n_env, 3))
    st = np.zeros((n_env * len(SLOTS), 7))
    st[:, 3] = 1.0
    return lo, hi, st


def test_attitudes_match_scipy_zyx_and_bounds_hold():
    lo, hi, st = setup()
    n_env = lo.shape[0]
    out = obstacles.randomize(lo, hi, SLOTS, np.ones(n_env, bool), 17, 99, np.arange(n_env), st)
    u = np.stack([obstacles.uniforms(np.arange(n_env), 17, k, 99) for k in range(len(SLOTS))], 1)
    for k, row in enumerate(SLOTS.astype(np.float64)):
        rows = np.arange(n_env) * len(SLOTS) + k
        ang = row[6:9] + (row[9:12] - row[6:9]) * u[:, k, 3:6]
        bits = int(row[12])
        for d in range(3):
            if bits >> (3 + d) & 1:
                ang[:, d] = row[16 + d]
        ref = Rotation.from_euler("ZYX", ang[:, ::-1]).as_quat()[:, [3, 0, 1, 2]]
        got = out[rows, 3:7]
        sign = np.sign((ref * got).sum(-1, keepdims=True))
        np.testing.assert_allclose(got * sign, ref, atol=1e-14)
        flo = lo + (hi - lo) * row[0:3]
        fhi = lo + (hi - lo) * row[3:6]
        for d in range(3):
            if not bits >> d & 1:
                assert np.all(out[rows, d] >= np.minimum(flo, fhi)[:, d] - 1e-12)
                assert np.all(out[rows, d] <= np.maximum(flo, fhi)[:, d] + 1e-12)
            else:
                np.testing.assert_array_equal(out[rows, d], lo[:, d] + (hi[:, d] - lo[:, d]) * row[13 + d])


def test_locked_yaw_and_unmasked_environments():
    lo, hi, st = setup(200)
    mask = np.zeros(200, bool)
    mask[::3] = True
    out = obstacles.randomize(lo, hi, SLOTS, mask, 5, 7, np.arange(200), st)
    keep = np.repeat(~mask, len(SLOTS))
    np.testing.assert_array_equal(out[keep], st[keep])
    rows = np.flatnonzero(mask) * len(SLOTS) + 1             # slot 1: yaw locked at 1 rad, no tilt
    yaw = Rotation.from_quat(out[rows][:, [4, 5, 6, 3]]).as_euler("ZYX")[:, 0]
    np.testing.assert_allclose(yaw, 1.0, atol=1e-14)


def test_draws_depend_on_global_index_only():
    lo, hi, st = setup(300)
    full = obstacles.randomize(lo, hi, SLOTS, np.ones(300, bool), 9, 5, np.arange(300), st)
    part = obstacles.randomize(lo[100:], hi[100:], SLOTS, np.ones(200, bool), 9, 5, np.arange(100, 300),
                               st[100 * len(SLOTS):])
    np.testing.assert_array_equal(full[100 * len(SLOTS):], part)
    u = obstacles.uniforms(np.arange(20000), 3, 0, 1)
    assert abs(u.mean() - 0.5) < 0.01 and u.min() >= 0 and u.max() < 1
