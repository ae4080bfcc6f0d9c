"""Rotor allocation in FP64 (oracle; test infrastructure only).

The paper applies f and M to the rigid body directly (end of Sec. IV-B) and
faults simulators that ignore the rotor's reaction torque (Sec. II).  The
allocation here is a reading (R12): n rotors at angles
alpha_i = pi/n + 2 pi i / n in the body x-y plane at arm length l, spin
signs s_i = (-1)^i, rotor i producing thrust u_i along +b3 and yaw torque
s_i c_tau u_i.  Column i of the allocation matrix A is
(1, l sin alpha_i, -l cos alpha_i, s_i c_tau)^T.  Rotor thrusts are the
min-norm solution u = A^+ (f, M), clamped elementwise to [u_min, u_max];
the wrench applied to the body is A u.
"""
import math

import torch


def layout(n_rotors):
    """Rotor angles and spin signs of the symmetric n-rotor layout."""
    i = torch.arange(n_rotors, dtype=torch.float64)
    alpha = math.pi / n_rotors + 2 * math.pi * i / n_rotors
    spin = torch.where(i.to(torch.int64) % 2 == 0, 1.0, -1.0).to(torch.float64)
    return alpha, spin


def allocation_matrix(n_rotors, arm, c_tau):
    """A [N,4,n] for per-vehicle arm [N] and c_tau [N]."""
    alpha, spin = layout(n_rotors)
    N = arm.shape[0]
    ones = torch.ones(N, n_rotors, dtype=torch.float64)
    return torch.stack([
        ones,
        arm[:, None] * torch.sin(alpha)[None, :],
        -arm[:, None] * torch.cos(alpha)[None, :],
        c_tau[:, None] * spin[None, :],
    ], 1)


def tables(fleet):
    """Per rotor count: (vehicle indices, A [n_i,4,nr], A^+ [n_i,nr,4]).
    A^+ is the Moore-Penrose pseudo-inverse (a library primitive)."""
    out = []
    for nr in sorted(set(int(k) for k in fleet.n_rotors.tolist())):
        idx = (fleet.n_rotors == nr).nonzero().squeeze(-1)
        A = allocation_matrix(nr, fleet.arm[idx], fleet.c_tau[idx])
        out.append((nr, idx, A, torch.linalg.pinv(A)))
    return out


def allocate(f, M, fleet, tabs=None):
    """Clamped min-norm allocation for every vehicle.

    Returns (u [N,8] zero-padded, f_applied [N], M_applied [N,3], u_raw [N,8])."""
    N = f.shape[0]
    if tabs is None:
        tabs = tables(fleet)
    u_all = torch.zeros(N, 8, dtype=torch.float64)
    raw_all = torch.zeros(N, 8, dtype=torch.float64)
    f_app = torch.zeros(N, dtype=torch.float64)
    M_app = torch.zeros(N, 3, dtype=torch.float64)
    w = torch.cat([f.unsqueeze(-1), M], -1)
    for nr, idx, A, A_pinv in tabs:
        raw = (A_pinv @ w[idx].unsqueeze(-1)).squeeze(-1)
        # torch.clamp passes the gradient where u_min <= raw <= u_max (inclusive, R20).
        u = torch.clamp(raw, fleet.u_min[idx, None], fleet.u_max[idx, None])
        wa = (A @ u.unsqueeze(-1)).squeeze(-1)
        u_all[idx, :nr] = u
        raw_all[idx, :nr] = raw
        f_app[idx] = wa[:, 0]
        M_app[idx] = wa[:, 1:]
    return u_all, f_app, M_app, raw_all


def clamp_distance(raw, fleet):
    """Per vehicle, the distance of the raw rotor command closest to a clamp
    bound (u_min or u_max), over that vehicle's rotors, relative to u_max."""
    N = raw.shape[0]
    d = torch.full((N,), float("inf"), dtype=raw.dtype)
    for nr in sorted(set(int(k) for k in fleet.n_rotors.tolist())):
        idx = (fleet.n_rotors == nr).nonzero().squeeze(-1)
        r = raw[idx, :nr]
        lo = (r - fleet.u_min[idx, None]).abs()
        hi = (r - fleet.u_max[idx, None]).abs()
        d[idx] = torch.minimum(lo, hi).min(-1).values / fleet.u_max[idx]
    return d


def saturated_count(raw, fleet):
    """Number of rotors per vehicle whose raw command lies strictly outside
    [u_min, u_max] (the clamp is inclusive, R20)."""
    N = raw.shape[0]
    cnt = torch.zeros(N, dtype=torch.int64)
    for nr in sorted(set(int(k) for k in fleet.n_rotors.tolist())):
        idx = (fleet.n_rotors == nr).nonzero().squeeze(-1)
        r = raw[idx, :nr]
        out = (r < fleet.u_min[idx, None]) | (r > fleet.u_max[idx, None])
        cnt[idx] = out.sum(-1)
    return cnt
