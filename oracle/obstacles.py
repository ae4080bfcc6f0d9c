"""Obstacle pose randomisation at environment reset, FP64 (oracle; test
infrastructure only).

Sec. V of the paper: when an environment is reset, every obstacle in it gets
a random position and orientation; position bounds are fractions of the
environment's bounds, orientation bounds are Euler angles, and chosen
dimensions can be locked to a constant.  Reading (R30): per obstacle slot k
a class row gives

  frac_lo[3], frac_hi[3]   position as a fraction of the env box per axis
  eul_lo[3],  eul_hi[3]    roll, pitch, yaw bounds [rad]
  lock (6 bits)            x, y, z, roll, pitch, yaw held at lock_val
  lock_val[6]              fraction (positions) or angle (orientation)

position_a = lo_a + (hi_a - lo_a) * (flo_a + (fhi_a - flo_a) u_a), attitude
q = qz(yaw) (x) qy(pitch) (x) qx(roll) (the Z-Y-X order of eq. (1)).
Uniforms: Philox4x32-10 with key = seed, counters (e, lo32(t), k, TAG | j),
j = 0, 1 -> 8 words, u = (w >> 8) 2^-24; words 0-2 position, 3-5 angles.
Only environments in the reset mask are redrawn.
"""
import math

import numpy as np

from .philox import philox4x32_10
from .reset import key_of

TAG_OBST = 0x4F420000
SLOT_DIM = 20          # frac_lo 3, frac_hi 3, eul_lo 3, eul_hi 3, lock 1, lock_val 6, pad 1


def slot_row(frac_lo, frac_hi, eul_lo, eul_hi, lock=(), lock_val=(0.0,) * 6):
    """Pack one slot's class parameters; lock is a list of dimension indices."""
    bits = 0
    for d in lock:
        bits |= 1 << d
    return np.array(list(frac_lo) + list(frac_hi) + list(eul_lo) + list(eul_hi) + [float(bits)]
                    + list(lock_val) + [0.0], np.float32)


def uniforms(env_idx, t, k, seed):
    e = np.asarray(env_idx, np.uint64)
    words = []
    for j in range(2):
        ctr = np.stack([e, np.full_like(e, t & 0xFFFFFFFF), np.full_like(e, k),
                        np.full_like(e, TAG_OBST | j)], -1)
        words.append(philox4x32_10(ctr, key_of(seed)))
    w = np.concatenate(words, -1)
    return (w >> 8).astype(np.float64) * 2.0 ** -24


def randomize(env_lo, env_hi, slots, env_mask, t, seed, global_env_idx, obst_state):
    """env_lo, env_hi: [n_env, 3]; slots: [n_obs, SLOT_DIM]; env_mask: bool [n_env];
    obst_state: [n_env * n_obs, 7] FP64 (x, y, z, qw, qx, qy, qz), updated copy returned."""
    out = np.array(obst_state, np.float64, copy=True)
    slots = np.asarray(slots, np.float64)
    n_obs = slots.shape[0]
    envs = np.flatnonzero(env_mask)
    if len(envs) == 0:
        return out
    lo = np.asarray(env_lo, np.float64)[envs]
    hi = np.asarray(env_hi, np.float64)[envs]
    for k in range(n_obs):
        row = slots[k]
        flo, fhi, elo, ehi = row[0:3], row[3:6], row[6:9], row[9:12]
        bits = int(row[12])
        lval = row[13:19]
        u = uniforms(np.asarray(global_env_idx)[envs], t, k, seed)
        frac = flo + (fhi - flo) * u[:, 0:3]
        ang = elo + (ehi - elo) * u[:, 3:6]
        for d in range(3):
            if bits >> d & 1:
                frac[:, d] = lval[d]
            if bits >> (3 + d) & 1:
                ang[:, d] = lval[3 + d]
        pos = lo + (hi - lo) * frac
        r, p, y = ang[:, 0] / 2, ang[:, 1] / 2, ang[:, 2] / 2
        cr, sr, cp, sp, cy, sy = np.cos(r), np.sin(r), np.cos(p), np.sin(p), np.cos(y), np.sin(y)
        # qz(yaw) (x) qy(pitch) (x) qx(roll), written out
        qw = cy * cp * cr + sy * sp * sr
        qx = cy * cp * sr - sy * sp * cr
        qy = cy * sp * cr + sy * cp * sr
        qz = sy * cp * cr - cy * sp * sr
        rows = envs * n_obs + k
        out[rows, 0:3] = pos
        out[rows, 3:7] = np.stack([qw, qx, qy, qz], -1)
    return out
