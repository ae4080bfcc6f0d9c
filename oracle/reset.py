"""Counter-based reset of vehicles (oracle; test infrastructure only).

The paper re-samples obstacle poses when environments are reset (Sec. V) and
exposes Gym-style resets (Sec. III).  For vehicles this is a reading (R22,
R24): at global step t, vehicle i (global index) is reset iff the Philox
word selected below is below floor(p * 2^32); a reset vehicle gets a fresh
state drawn like the initial states, and a position-mode vehicle also a fresh
goal (yaw command 0).  Indices of reset vehicles are reported in ascending
order.

Stream layout (key = (seed_lo, seed_hi)):
  mask  : counter (i, lo32(t//4), hi32(t//4), TAG_MASK), word t mod 4
  draws : counter (i, lo32(t), hi32(t), TAG_DRAW | j), j = 0..3 -> 16 words
          u_k = (w_k >> 8) 2^-24
          words 0-2 position, 3-5 goal, 6 tilt-axis angle, 7 tilt, 8 yaw,
          (9,10) (11,12) (13,14) Box-Muller pairs -> 3 velocity + 3 rate normals
"""
import math

import numpy as np
import torch

from .philox import philox4x32_10

TAG_MASK = 0x4D41534B
TAG_DRAW = 0x44520000
TILT_MAX = math.pi / 6
VEL_SIGMA = 0.5
RATE_SIGMA = 0.2


def threshold(p):
    return int(min(max(math.floor(p * 4294967296.0), 0), 4294967296))


def key_of(seed):
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], np.uint64)


def mask(global_idx, t, seed, p):
    """Reset mask (bool [n]) for vehicles with global indices ``global_idx`` at step t."""
    i = np.asarray(global_idx, np.uint64)
    tb = t // 4
    ctr = np.stack([i, np.full_like(i, tb & 0xFFFFFFFF), np.full_like(i, tb >> 32),
                    np.full_like(i, TAG_MASK)], -1)
    w = philox4x32_10(ctr, key_of(seed))[:, t % 4]
    return w.astype(np.uint64) < np.uint64(threshold(p))


def draw_words(global_idx, t, seed):
    i = np.asarray(global_idx, np.uint64)
    out = []
    for j in range(4):
        ctr = np.stack([i, np.full_like(i, t & 0xFFFFFFFF), np.full_like(i, t >> 32),
                        np.full_like(i, TAG_DRAW | j)], -1)
        out.append(philox4x32_10(ctr, key_of(seed)))
    return np.concatenate(out, -1)          # [n, 16]


def box_muller(ua, ub):
    """Two independent standard normals from two independent uniforms on
    [0, 1) (Box and Muller, 1958): radius sqrt(-2 ln(1 - ua)), angle 2 pi ub.
    (1 - ua lies in (0, 1], so the logarithm is finite.)"""
    r = np.sqrt(-2.0 * np.log(1.0 - ua))
    return r * np.cos(2 * math.pi * ub), r * np.sin(2 * math.pi * ub)


def state_from_uniforms(u, lo, hi):
    """Fresh (state [n,13], goal [n,3]) in FP64 from 16 uniforms per vehicle
    (u [n,16], the word layout of the module docstring)."""
    u = np.asarray(u, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    x = lo + (hi - lo) * u[:, 0:3]
    goal = lo + (hi - lo) * u[:, 3:6]
    beta = -math.pi + 2 * math.pi * u[:, 6]
    tau = TILT_MAX * u[:, 7]
    psi = -math.pi + 2 * math.pi * u[:, 8]
    # q = qz(psi) (x) q_axis((cos beta, sin beta, 0), tau)
    a0, a3 = np.cos(psi / 2), np.sin(psi / 2)
    b0 = np.cos(tau / 2)
    b1 = np.sin(tau / 2) * np.cos(beta)
    b2 = np.sin(tau / 2) * np.sin(beta)
    q = np.stack([a0 * b0, a0 * b1 - a3 * b2, a0 * b2 + a3 * b1, a3 * b0], -1)
    normals = []
    for a, b in ((9, 10), (11, 12), (13, 14)):
        normals += list(box_muller(u[:, a], u[:, b]))
    n = np.stack(normals, -1)
    v = VEL_SIGMA * n[:, 0:3]
    W = RATE_SIGMA * n[:, 3:6]
    s = np.concatenate([x, v, q, W], -1)
    return torch.as_tensor(s), torch.as_tensor(goal)


def uniforms(global_idx, t, seed):
    """The 16 uniforms u_k = (w_k >> 8) 2^-24 of each vehicle's redraw."""
    w = draw_words(global_idx, t, seed)
    return (w >> 8).astype(np.float64) * 2.0 ** -24


def redraw(global_idx, t, seed, lo, hi):
    """Fresh (state [n,13], goal [n,3]) in FP64 for the given vehicles."""
    return state_from_uniforms(uniforms(global_idx, t, seed), lo, hi)


def apply(state, mode, target, global_idx, t, seed, p, lo, hi, explicit_mask=None):
    """Reset step: returns (state, target, mask, ascending indices).  state
    [n,13] and target [n,4] are FP64 tensors (copied, not modified)."""
    m = mask(global_idx, t, seed, p) if explicit_mask is None else np.asarray(explicit_mask, bool)
    idx = np.flatnonzero(m)
    state = state.clone()
    target = target.clone()
    if len(idx):
        s_new, goal = redraw(np.asarray(global_idx)[idx], t, seed, lo, hi)
        state[idx] = s_new.to(state.dtype)
        pos = torch.as_tensor(np.asarray(mode)[idx] == 0)
        tg = target[idx]
        tg[pos, :3] = goal[pos].to(tg.dtype)
        tg[pos, 3] = 0.0
        target[idx] = tg
    return state, target, m, idx.astype(np.int32)
