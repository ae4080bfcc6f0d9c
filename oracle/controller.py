"""Parallel SE(3) geometric controller in FP64 (oracle; test infrastructure only).

Follows Sec. IV of the paper (after Lee et al., 2011) equation by equation:

* attitude mode (Sec. IV-A): commands (phi_d, theta_d, psidot_d, f);
  R_d by eq. (1), Omega_d by eq. (2), e_R by eq. (3), e_Omega by eq. (4),
  moment M by eq. (5) (Lee's feed-forward term dropped, as the paper states);
* velocity mode (Sec. IV-B): command (v_d in the vehicle frame V, psidot_d);
  a_d by eq. (6), thrust f by eq. (7), tilt angles by eqs. (8)-(9), then the
  attitude controller;
* position mode (named in Sec. I and the abstract, no equations given):
  a = kx (x_d - x) - kv v in E, then the same force -> tilt -> attitude
  machinery, referenced to the commanded yaw psi_d with zero yaw rate;
* wrench mode (a test mode): (f, M) given directly.

Readings (numbered as in the package docstring): z-up inertial frame, gravity
-g e3, thrust +f b3 (R1); eq. (7) read as F = m (a_d + g e3) (R2) and eqs.
(8)-(9) evaluated on that gravity-compensated F expressed in V (R3); f is the
projection of F on the current b3 expressed in V (R4); yaw is the Z-Y-X yaw
(R7); theta_d = 0 when F_x = F_z = 0 and phi_d = 0 when F = 0 (R14);
unknown mode codes command a zero wrench (R28).
"""
import torch

from .so3 import quat_to_rot, rot_x, rot_y, rot_z, vee, yaw_of, mv

MODE_POSITION, MODE_VELOCITY, MODE_ATTITUDE, MODE_WRENCH = 0, 1, 2, 3


def _e3(like):
    e = torch.zeros(like.shape[0], 3, dtype=like.dtype)
    e[:, 2] = 1.0
    return e


def gain_vectors(gains):
    """Split the 10-gain layout into diagonal gain vectors kx, kv, kR, kW."""
    kx = torch.stack([gains[:, 0], gains[:, 0], gains[:, 1]], -1)
    kv = torch.stack([gains[:, 2], gains[:, 2], gains[:, 3]], -1)
    return kx, kv, gains[:, 4:7], gains[:, 7:10]


def position_accel(kx, kv, x_d, x, v):
    """Position mode (reading R8): a = kx o (x_d - x) - kv o v in the inertial
    frame, with kx = (kx_xy, kx_xy, kx_z) and kv = (kv_xy, kv_xy, kv_z)."""
    return kx * (x_d - x) - kv * v


def velocity_accel(kv, v_d, v_V):
    """Eq. (6): a_d = kv o (v_d - v), both in the vehicle frame V (R10)."""
    return kv * (v_d - v_V)


def tilt_from_force(F_V):
    """Eqs. (8)-(9) on the gravity-compensated force in V:
    phi_d = atan2(-F_y, sqrt(F_x^2 + F_z^2)), theta_d = atan2(F_x, F_z)."""
    Fx, Fy, Fz = F_V[:, 0], F_V[:, 1], F_V[:, 2]
    h = torch.sqrt(Fx * Fx + Fz * Fz)
    phi = torch.atan2(-Fy, h)
    theta = torch.atan2(Fx, Fz)
    theta = torch.where(h == 0, torch.zeros_like(theta), theta)
    phi = torch.where((h == 0) & (Fy == 0), torch.zeros_like(phi), phi)
    return phi, theta


def desired_rotation(psi_ref, theta_d, phi_d):
    """Eq. (1): R_d = R_z(psi) R_y(theta_d) R_x(phi_d)."""
    return rot_z(psi_ref) @ rot_y(theta_d) @ rot_x(phi_d)


def desired_rate(phi_d, theta_d, psidot_d):
    """Eq. (2): Omega_d = E(phi_d, theta_d) (0, 0, psidot_d)^T."""
    o, z = torch.ones_like(phi_d), torch.zeros_like(phi_d)
    E = torch.stack([
        torch.stack([o, z, -torch.sin(theta_d)], -1),
        torch.stack([z, torch.cos(phi_d), torch.sin(phi_d) * torch.cos(theta_d)], -1),
        torch.stack([z, -torch.sin(phi_d), torch.cos(phi_d) * torch.cos(theta_d)], -1),
    ], -2)
    return mv(E, torch.stack([z, z, psidot_d], -1))


def attitude_errors(R, R_d, Omega, Omega_d):
    """Eqs. (3)-(4): e_R = 1/2 (R_d^T R - R^T R_d)^vee, e_Omega = Omega - R^T R_d Omega_d."""
    Rt = R.transpose(-1, -2)
    e_R = 0.5 * vee(R_d.transpose(-1, -2) @ R - Rt @ R_d)
    e_W = Omega - mv(Rt @ R_d, Omega_d)
    return e_R, e_W


def moment(e_R, e_W, Omega, J, kR, kW):
    """Eq. (5): M = -kR e_R - kW e_Omega + Omega x J Omega."""
    return -kR * e_R - kW * e_W + torch.cross(Omega, J * Omega, dim=-1)


def control(x, v, q, Omega, mode, target, fleet, g, traj=None):
    """One controller evaluation for every vehicle.

    x, v, Omega: [N,3]; q: [N,4] (w,x,y,z); mode: [N] integer; target: [N,4]
    (the mode's 4-float command union); traj: optional [N,16] trajectory
    rows of the tracking mode 4 (``oracle.lee``); returns dict with the
    commanded thrust ``f`` [N] and moment ``M`` [N,3] plus intermediates.
    """
    mode = mode.to(torch.int64)
    R = quat_to_rot(q)
    psi = yaw_of(R)
    e3 = _e3(x)
    b3 = R[:, :, 2]
    kx, kv, kR, kW = gain_vectors(fleet.gains)
    m = fleet.m.unsqueeze(-1)
    zero = torch.zeros_like(psi)

    # Position mode: a = kx (x_d - x) - kv v in E; F = m (a + g e3);
    # referenced to the commanded yaw psi_d with zero yaw rate.
    psi_d = target[:, 3]
    a_E = position_accel(kx, kv, target[:, :3], x, v)
    F_E = m * (a_E + g * e3)
    RzT_d = rot_z(psi_d).transpose(-1, -2)
    F_V0 = mv(RzT_d, F_E)
    f0 = (F_E * b3).sum(-1)

    # Velocity mode: v expressed in V, eq. (6), eq. (7) read as a force.
    RzT = rot_z(psi).transpose(-1, -2)
    v_V = mv(RzT, v)
    a_d = velocity_accel(kv, target[:, :3], v_V)
    F_V1 = m * (a_d + g * e3)
    b3_V = mv(RzT, b3)
    f1 = (F_V1 * b3_V).sum(-1)

    is0 = (mode == MODE_POSITION)
    is1 = (mode == MODE_VELOCITY)
    is2 = (mode == MODE_ATTITUDE)
    is3 = (mode == MODE_WRENCH)
    F_V = torch.where(is0.unsqueeze(-1), F_V0, F_V1)
    phi_F, theta_F = tilt_from_force(F_V)                      # eqs. (8)-(9)

    phi_d = torch.where(is2, target[:, 0], phi_F)
    theta_d = torch.where(is2, target[:, 1], theta_F)
    psidot_d = torch.where(is1, target[:, 3], torch.where(is2, target[:, 2], zero))
    psi_ref = torch.where(is0, psi_d, psi)
    f = torch.where(is0, f0, torch.where(is1, f1, target[:, 3]))

    R_d = desired_rotation(psi_ref, theta_d, phi_d)            # eq. (1)
    Omega_d = desired_rate(phi_d, theta_d, psidot_d)           # eq. (2)
    e_R, e_W = attitude_errors(R, R_d, Omega, Omega_d)         # eqs. (3)-(4)
    M = moment(e_R, e_W, Omega, fleet.J, kR, kW)               # eq. (5)

    f = torch.where(is3, target[:, 0], f)
    M = torch.where(is3.unsqueeze(-1), target[:, 1:4], M)
    known = is0 | is1 | is2 | is3
    if traj is not None:
        from .lee import MODE_TRACK, lee_tracking
        is4 = mode == MODE_TRACK
        lt = lee_tracking(x, v, q, Omega, traj, fleet, g)
        f = torch.where(is4, lt["f"], f)
        M = torch.where(is4.unsqueeze(-1), lt["M"], M)
        R_d = torch.where(is4[:, None, None], lt["R_d"], R_d)
        known = known | is4
    f = torch.where(known, f, zero)
    M = torch.where(known.unsqueeze(-1), M, torch.zeros_like(M))
    return {"f": f, "M": M, "R": R, "R_d": R_d, "Omega_d": Omega_d, "e_R": e_R,
            "e_W": e_W, "phi_d": phi_d, "theta_d": theta_d, "psi": psi,
            "psi_ref": psi_ref, "psidot_d": psidot_d, "F_V": F_V}
