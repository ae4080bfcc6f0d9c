"""Rigid-body dynamics in FP64 (oracle; test infrastructure only).

The paper hands f and M to its physics engine (Sec. I, end of Sec. IV-B).
The integrator here is a reading (R15): semi-implicit Euler on the
Newton-Euler equations of a rigid body with thrust +f' b3 and gravity -g e3:

  v+     = v + dt ((f'/m) R e3 - g e3)
  x+     = x + dt v+
  Omega+ = Omega + dt J^-1 (M' - Omega x J Omega)
  q+     = normalize(q + dt/2 q (x) (0, Omega+))

Controller quantities are evaluated at the pre-step state; the quaternion
update uses the post-step body rate.
"""
import torch

from .so3 import quat_to_rot, quat_mul


def integrate(x, v, q, Omega, f_app, M_app, fleet, dt, g):
    R = quat_to_rot(q)
    b3 = R[:, :, 2]
    e3 = torch.zeros_like(x)
    e3[:, 2] = 1.0
    m = fleet.m.unsqueeze(-1)
    acc = (f_app.unsqueeze(-1) / m) * b3 - g * e3
    v_n = v + dt * acc
    x_n = x + dt * v_n
    J = fleet.J
    Omega_n = Omega + dt * (M_app - torch.cross(Omega, J * Omega, dim=-1)) / J
    zero = torch.zeros_like(Omega_n[:, :1])
    q_t = q + 0.5 * dt * quat_mul(q, torch.cat([zero, Omega_n], -1))
    q_n = q_t / torch.linalg.vector_norm(q_t, dim=-1, keepdim=True)
    return x_n, v_n, q_n, Omega_n
