"""Full geometric tracking law on SE(3) in FP64 (oracle; test infrastructure only).

The paper adapts the controller of Lee et al. (its reference on geometric
control) and drops the feed-forward term of the moment (Sec. IV-A, after
eq. (5)).  This module is the undropped law, used by the trajectory-tracking
mode (mode 4):

  e_x = x - x_d,  e_v = v - v_d
  F   = m ( -kx e_x - kv e_v + a_d + g e3 )               (z-up, reading R1/R2)
  f   = F . R e3
  b3c = F / |F|,  b1d = (cos psi_d, sin psi_d, 0)
  b2c = b3c x b1d / |b3c x b1d|,  b1c = b2c x b3c,  R_d = [b1c b2c b3c]
  e_R = 1/2 (R_d^T R - R^T R_d)^vee,  e_Omega = Omega - R^T R_d Omega_d
  M   = -kR e_R - kW e_Omega + Omega x J Omega
        - J ( hat(Omega) R^T R_d Omega_d - R^T R_d dOmega_d )

Trajectory row layout per vehicle (16 values): x_d(3), v_d(3), a_d(3),
psi_d, Omega_d(3), dOmega_d(3).  When b3c is parallel to b1d the heading is
undefined; b1d is then replaced by e1 (and by e2 if b3c is parallel to e1).
"""
import torch

from .controller import gain_vectors, attitude_errors
from .so3 import mv, quat_to_rot

MODE_TRACK = 4


def _unit_cross(a, b):
    c = torch.cross(a, b, dim=-1)
    return c, torch.linalg.vector_norm(c, dim=-1, keepdim=True)


def desired_frame(F, psi_d):
    """R_d = [b1c b2c b3c] from the force direction and the heading."""
    b3 = F / torch.linalg.vector_norm(F, dim=-1, keepdim=True)
    z = torch.zeros_like(psi_d)
    b1d = torch.stack([torch.cos(psi_d), torch.sin(psi_d), z], -1)
    c, nc = _unit_cross(b3, b1d)
    e1 = torch.zeros_like(b3)
    e1[:, 0] = 1.0
    e2 = torch.zeros_like(b3)
    e2[:, 1] = 1.0
    c1, n1 = _unit_cross(b3, e1)
    c2, n2 = _unit_cross(b3, e2)
    c = torch.where(nc > 0, c, torch.where(n1 > 0, c1, c2))
    nc = torch.where(nc > 0, nc, torch.where(n1 > 0, n1, n2))
    b2 = c / nc
    b1 = torch.cross(b2, b3, dim=-1)
    return torch.stack([b1, b2, b3], -1)


def lee_tracking(x, v, q, Omega, traj, fleet, g):
    R = quat_to_rot(q)
    kx, kv, kR, kW = gain_vectors(fleet.gains)
    m = fleet.m.unsqueeze(-1)
    e3 = torch.zeros_like(x)
    e3[:, 2] = 1.0
    e_x = x - traj[:, 0:3]
    e_v = v - traj[:, 3:6]
    F = m * (-kx * e_x - kv * e_v + traj[:, 6:9] + g * e3)
    f = (F * R[:, :, 2]).sum(-1)
    R_d = desired_frame(F, traj[:, 9])
    Omega_d = traj[:, 10:13]
    dOmega_d = traj[:, 13:16]
    e_R, e_W = attitude_errors(R, R_d, Omega, Omega_d)
    RtRd = R.transpose(-1, -2) @ R_d
    J = fleet.J
    ff = J * (torch.cross(Omega, mv(RtRd, Omega_d), dim=-1) - mv(RtRd, dOmega_d))
    M = -kR * e_R - kW * e_W + torch.cross(Omega, J * Omega, dim=-1) - ff
    return {"f": f, "M": M, "R": R, "R_d": R_d, "e_R": e_R, "e_W": e_W, "F": F}
