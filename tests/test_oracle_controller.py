"""Pins of the oracle's controller (Sec. IV, eqs. (1)-(9)) against closed
forms and identities that the equations fix."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import controller, so3
from oracle.fleet import Fleet
from workloads import Group, QUAD_GAINS

F64 = torch.float64
G = 9.81


def quad_fleet(n):
    return Fleet.from_groups([Group(0, n)], n)


def rgen(seed):
    return torch.Generator().manual_seed(seed)


def quat_of(R):
    q = Rotation.from_matrix(R.numpy()).as_quat()      # x, y, z, w
    return torch.as_tensor(q[:, [3, 0, 1, 2]])


def run(x, v, R, W, mode, tgt, fleet=None):
    n = x.shape[0]
    fleet = fleet or quad_fleet(n)
    return controller.control(x, v, quat_of(R), W, torch.full((n,), mode), tgt, fleet, G)


def test_desired_rotation_aligns_b3_with_force():
    """Eqs. (1), (8), (9): R_d e3 = R_z(psi) F_V / |F_V| for every F_V != 0."""
    g = rgen(1)
    F = torch.randn(400, 3, generator=g, dtype=F64) * 5
    psi = (torch.rand(400, generator=g, dtype=F64) * 2 - 1) * math.pi
    phi, theta = controller.tilt_from_force(F)
    Rd = controller.desired_rotation(psi, theta, phi)
    expect = so3.mv(so3.rot_z(psi), F / F.norm(dim=-1, keepdim=True))
    assert (Rd[:, :, 2] - expect).abs().max() < 1e-14


def test_level_attitude_when_force_is_vertical():
    F = torch.tensor([[0.0, 0.0, 9.81], [0.0, 0.0, 1e-3]], dtype=F64)
    phi, theta = controller.tilt_from_force(F)
    assert torch.equal(phi, torch.zeros(2, dtype=F64))
    assert torch.equal(theta, torch.zeros(2, dtype=F64))


def test_desired_rate_is_yaw_rate_about_desired_z():
    """Eq. (2): Omega_d = psidot_d R_d^T e3; = (0, 0, psidot_d) when level."""
    g = rgen(2)
    phi = (torch.rand(300, generator=g, dtype=F64) * 2 - 1) * 1.5
    theta = (torch.rand(300, generator=g, dtype=F64) * 2 - 1) * 3.0
    psi = (torch.rand(300, generator=g, dtype=F64) * 2 - 1) * 3.0
    rate = torch.randn(300, generator=g, dtype=F64)
    Wd = controller.desired_rate(phi, theta, rate)
    Rd = controller.desired_rotation(psi, theta, phi)
    assert (Wd - rate[:, None] * Rd[:, 2, :]).abs().max() < 1e-14
    z = torch.zeros(3, dtype=F64)
    r = torch.tensor([0.3, -1.0, 2.0], dtype=F64)
    assert torch.equal(controller.desired_rate(z, z, r),
                       torch.stack([z, z, r], -1))


def test_attitude_error_closed_form():
    """Eq. (3): for R = R_d Rot(n, a), e_R = sin(a) n; e_R = 0 iff a in {0, pi}."""
    g = rgen(3)
    n = torch.randn(300, 3, generator=g, dtype=F64)
    n = n / n.norm(dim=-1, keepdim=True)
    a = (torch.rand(300, generator=g, dtype=F64) * 2 - 1) * math.pi
    Rd = torch.as_tensor(Rotation.random(300, random_state=5).as_matrix())
    Rot = torch.as_tensor(Rotation.from_rotvec((n * a[:, None]).numpy()).as_matrix())
    R = Rd @ Rot
    e_R, _ = controller.attitude_errors(R, Rd, torch.zeros(300, 3, dtype=F64),
                                        torch.zeros(300, 3, dtype=F64))
    assert (e_R - torch.sin(a)[:, None] * n).abs().max() < 1e-14
    Rpi = Rd @ torch.as_tensor(Rotation.from_rotvec((n * math.pi).numpy()).as_matrix())
    e_pi, _ = controller.attitude_errors(Rpi, Rd, torch.zeros(300, 3, dtype=F64),
                                         torch.zeros(300, 3, dtype=F64))
    assert e_pi.abs().max() < 1e-14


def test_rate_error_reduces_to_yaw_rate_about_body():
    """Eqs. (1), (2), (4): e_Omega = Omega - psidot_d R^T e3 in attitude mode."""
    g = rgen(4)
    n = 300
    R = torch.as_tensor(Rotation.random(n, random_state=6).as_matrix())
    W = torch.randn(n, 3, generator=g, dtype=F64)
    tgt = torch.stack([(torch.rand(n, generator=g, dtype=F64) - 0.5),
                       (torch.rand(n, generator=g, dtype=F64) - 0.5),
                       torch.randn(n, generator=g, dtype=F64), torch.full((n,), 9.0, dtype=F64)], -1)
    z = torch.zeros(n, 3, dtype=F64)
    out = run(z, z, R, W, 2, tgt)
    expect = W - tgt[:, 2:3] * out["R"][:, 2, :]
    assert (out["e_W"] - expect).abs().max() < 1e-13


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_moment_for_pure_axis_error(axis):
    """Eq. (5): R = R_d Rot(b_axis, a), Omega = 0, no yaw rate ->
    M = -kR[axis] sin(a) b_axis (gyroscopic term vanishes)."""
    a = torch.tensor([0.3, -0.7, 1.2], dtype=F64)
    n = a.shape[0]
    rv = torch.zeros(n, 3, dtype=F64)
    rv[:, axis] = a
    psi = torch.tensor([0.4, -2.0, 3.0], dtype=F64)
    Rd = so3.rot_z(psi)
    R = Rd @ torch.as_tensor(Rotation.from_rotvec(rv.numpy()).as_matrix())
    z = torch.zeros(n, 3, dtype=F64)
    tgt = torch.zeros(n, 4, dtype=F64)
    tgt[:, 3] = 9.81
    if axis == 2:
        # a yaw error is measured against the current yaw in attitude mode; use position
        # mode with a commanded yaw instead (hover force, level desired attitude).
        tgt = torch.zeros(n, 4, dtype=F64)
        tgt[:, 3] = psi
        out = run(z, z, R, z, 0, tgt)
    else:
        out = run(z, z, R, z, 2, tgt)
    kR = torch.tensor(np.float32(QUAD_GAINS[4:7]), dtype=F64)   # the fleet holds FP32 gains
    expect = torch.zeros(n, 3, dtype=F64)
    expect[:, axis] = -kR[axis] * torch.sin(a)
    assert (out["M"] - expect).abs().max() < 1e-13


def test_hover_is_an_equilibrium_of_the_controller():
    """Position mode at the goal, level, with the commanded yaw and at rest:
    f = m g, M = 0, e_R = 0.  Velocity mode with v = v_d: same wrench."""
    n = 7
    psi_d = torch.linspace(-3.0, 3.0, n, dtype=F64)
    xg = torch.randn(n, 3, generator=rgen(5), dtype=F64)
    tgt = torch.cat([xg, psi_d[:, None]], -1)
    z = torch.zeros(n, 3, dtype=F64)
    out = run(xg, z, so3.rot_z(psi_d), z, 0, tgt)
    assert (out["f"] - G).abs().max() < 1e-14
    assert out["M"].abs().max() < 1e-14
    assert out["e_R"].abs().max() < 1e-15
    vd = torch.randn(n, 3, generator=rgen(6), dtype=F64)
    v = so3.mv(so3.rot_z(psi_d), vd)
    tgt1 = torch.cat([vd, torch.zeros(n, 1, dtype=F64)], -1)
    out1 = run(z, v, so3.rot_z(psi_d), z, 1, tgt1)
    assert (out1["f"] - G).abs().max() < 1e-13
    assert out1["M"].abs().max() < 1e-13


def test_velocity_mode_tilt_closed_form():
    """Eqs. (6)-(9): level vehicle at rest, v_d = (c, 0, 0) in V:
    theta_d = atan2(kv c, g), phi_d = 0, f = m g (projection on level b3)."""
    c = torch.tensor([9.81 / 2.0, -1.0, 0.25, 3.0], dtype=F64)
    n = c.shape[0]
    z = torch.zeros(n, 3, dtype=F64)
    psi = torch.tensor([0.0, 1.0, -2.5, 3.1], dtype=F64)
    tgt = torch.stack([c, torch.zeros_like(c), torch.zeros_like(c), torch.zeros_like(c)], -1)
    out = run(z, z, so3.rot_z(psi), z, 1, tgt)
    kv = QUAD_GAINS[2]
    assert (out["theta_d"] - torch.atan2(kv * c, torch.full_like(c, G))).abs().max() < 1e-14
    assert out["phi_d"].abs().max() < 1e-15
    assert (out["f"] - G).abs().max() < 1e-14
    assert torch.allclose(out["theta_d"][0], torch.tensor(math.pi / 4, dtype=F64), atol=1e-15)


def test_attitude_mode_on_target_gives_gyroscopic_moment_only():
    """Eqs. (3)-(5): R = R_d and Omega = Omega_d -> e_R = 0, e_Omega = 0, M = Omega x J Omega."""
    n = 50
    g = rgen(7)
    phi = (torch.rand(n, generator=g, dtype=F64) - 0.5)
    theta = (torch.rand(n, generator=g, dtype=F64) - 0.5)
    psi = (torch.rand(n, generator=g, dtype=F64) * 2 - 1) * 3
    rate = torch.randn(n, generator=g, dtype=F64)
    Rd = controller.desired_rotation(psi, theta, phi)
    Wd = controller.desired_rate(phi, theta, rate)
    tgt = torch.stack([phi, theta, rate, torch.full_like(phi, 12.0)], -1)
    z = torch.zeros(n, 3, dtype=F64)
    out = run(z, z, Rd, Wd, 2, tgt)
    J = torch.tensor(np.float32([0.007, 0.007, 0.012]), dtype=F64)
    assert out["e_R"].abs().max() < 1e-14
    assert out["e_W"].abs().max() < 1e-14
    assert (out["M"] - torch.cross(Wd, J * Wd, dim=-1)).abs().max() < 1e-14
    assert torch.equal(out["f"], tgt[:, 3])


def test_position_mode_yaw_equivariance_and_translation_invariance():
    """Rotating state and goal about e3 by b (and the yaw command by b)
    leaves the body-frame wrench unchanged; so does translating x and x_d."""
    n = 200
    g = rgen(8)
    x = torch.randn(n, 3, generator=g, dtype=F64)
    v = torch.randn(n, 3, generator=g, dtype=F64)
    W = torch.randn(n, 3, generator=g, dtype=F64) * 0.3
    R = torch.as_tensor(Rotation.random(n, random_state=9).as_matrix())
    xg = torch.randn(n, 3, generator=g, dtype=F64)
    psi_d = torch.rand(n, generator=g, dtype=F64)
    tgt = torch.cat([xg, psi_d[:, None]], -1)
    base = run(x, v, R, W, 0, tgt)
    b = torch.rand(n, generator=g, dtype=F64) * 2 - 1
    Rz = so3.rot_z(b)
    tgt_r = torch.cat([so3.mv(Rz, xg), (psi_d + b)[:, None]], -1)
    rot = run(so3.mv(Rz, x), so3.mv(Rz, v), Rz @ R, W, 0, tgt_r)
    assert (rot["f"] - base["f"]).abs().max() < 1e-12
    assert (rot["M"] - base["M"]).abs().max() < 1e-12
    c = torch.randn(1, 3, generator=g, dtype=F64) * 10
    tr = run(x + c, v, R, W, 0, torch.cat([xg + c, psi_d[:, None]], -1))
    assert (tr["f"] - base["f"]).abs().max() < 1e-12
    assert (tr["M"] - base["M"]).abs().max() < 1e-12


def test_wrench_mode_and_unknown_mode():
    n = 4
    z = torch.zeros(n, 3, dtype=F64)
    R = so3.rot_z(torch.zeros(n, dtype=F64))
    tgt = torch.tensor([[1.0, 0.1, -0.2, 0.3]] * n, dtype=F64)
    out = run(z, z, R, z, 3, tgt)
    assert torch.equal(out["f"], tgt[:, 0]) and torch.equal(out["M"], tgt[:, 1:])
    out7 = run(z, z, R, z, 7, tgt)
    assert torch.equal(out7["f"], torch.zeros(n, dtype=F64))
    assert torch.equal(out7["M"], torch.zeros(n, 3, dtype=F64))


# ---- split gains (kx_xy != kx_z, kv_xy != kv_z) and nonzero velocity ---------
# Every case below is level (b3 = e3) with zero body rate, so the commanded
# force is the only thing that moves; values are exact in FP32, so the fleet
# holds them unrounded.
SPLIT_GAINS = (1.5, 3.0, 2.5, 0.75, 1.6, 1.6, 0.6, 0.5, 0.5, 0.2)
SPLIT_MASS = 1.25


def split_fleet(n):
    from workloads import Group
    return Fleet.from_groups([Group(0, n, mass=SPLIT_MASS, gains=SPLIT_GAINS)], n)


def test_position_mode_vertical_velocity_is_damped_by_kv_z():
    """Eq. (6) read for position mode (R8): at the goal, level, v = (0, 0, c):
    a = -kv_z c e3, so F is vertical, f = m (g - kv_z c), the desired attitude
    is the commanded yaw frame and M = 0."""
    c = torch.tensor([2.0, -1.5, 0.5, 4.0], dtype=F64)
    n = c.shape[0]
    psi_d = torch.tensor([0.0, 0.7, -2.2, 3.0], dtype=F64)
    xg = torch.tensor([[1.0, -2.0, 0.5]] * n, dtype=F64)
    v = torch.zeros(n, 3, dtype=F64)
    v[:, 2] = c
    z = torch.zeros(n, 3, dtype=F64)
    out = run(xg, v, so3.rot_z(psi_d), z, 0, torch.cat([xg, psi_d[:, None]], -1), split_fleet(n))
    kv_z = SPLIT_GAINS[3]
    assert (out["f"] - SPLIT_MASS * (G - kv_z * c)).abs().max() < 1e-13
    assert out["M"].abs().max() < 1e-13
    assert out["phi_d"].abs().max() < 1e-15 and out["theta_d"].abs().max() < 1e-15


def test_position_mode_horizontal_velocity_tilts_against_it():
    """Position mode at the goal with v = R_z(psi_d) (c, 0, 0):
    F_V = m (-kv_xy c, 0, g), hence theta_d = atan2(-kv_xy c, g), phi_d = 0 and
    f = m g on a level body (eqs. (8)-(9))."""
    c = torch.tensor([1.0, -3.0, 0.25], dtype=F64)
    n = c.shape[0]
    psi_d = torch.tensor([0.3, -1.9, 2.6], dtype=F64)
    xg = torch.zeros(n, 3, dtype=F64)
    Rz = so3.rot_z(psi_d)
    v = so3.mv(Rz, torch.stack([c, torch.zeros_like(c), torch.zeros_like(c)], -1))
    z = torch.zeros(n, 3, dtype=F64)
    out = run(xg, v, Rz, z, 0, torch.cat([xg, psi_d[:, None]], -1), split_fleet(n))
    kv_xy = SPLIT_GAINS[2]
    assert (out["theta_d"] - torch.atan2(-kv_xy * c, torch.full_like(c, G))).abs().max() < 1e-14
    assert out["phi_d"].abs().max() < 1e-14
    assert (out["f"] - SPLIT_MASS * G).abs().max() < 1e-13


def test_position_mode_offset_uses_kx_xy_and_kx_z():
    """Position mode at rest, level, x = x_d - R_z(psi_d) (d_x, 0, d_z):
    F_V = m (kx_xy d_x, 0, g + kx_z d_z), so theta_d = atan2(kx_xy d_x, g + kx_z d_z),
    phi_d = 0, f = m (g + kx_z d_z)."""
    dx = torch.tensor([0.5, -1.0, 2.0], dtype=F64)
    dz = torch.tensor([1.0, -0.5, 0.25], dtype=F64)
    n = dx.shape[0]
    psi_d = torch.tensor([-0.4, 1.1, 2.9], dtype=F64)
    Rz = so3.rot_z(psi_d)
    xg = torch.tensor([[0.5, 1.5, -1.0]] * n, dtype=F64)
    x = xg - so3.mv(Rz, torch.stack([dx, torch.zeros_like(dx), dz], -1))
    z = torch.zeros(n, 3, dtype=F64)
    out = run(x, z, Rz, z, 0, torch.cat([xg, psi_d[:, None]], -1), split_fleet(n))
    kx_xy, kx_z = SPLIT_GAINS[0], SPLIT_GAINS[1]
    assert (out["theta_d"] - torch.atan2(kx_xy * dx, G + kx_z * dz)).abs().max() < 1e-14
    assert out["phi_d"].abs().max() < 1e-14
    assert (out["f"] - SPLIT_MASS * (G + kx_z * dz)).abs().max() < 1e-13


def test_velocity_mode_split_gains_at_nonzero_velocity():
    """Eqs. (6)-(9) with v_d = 0 and a level vehicle moving with
    v = R_z(psi) (c1, 0, c3): a_d = (-kv_xy c1, 0, -kv_z c3) in V, so
    theta_d = atan2(-kv_xy c1, g - kv_z c3), phi_d = 0, f = m (g - kv_z c3)."""
    c1 = torch.tensor([1.0, -2.0, 0.5], dtype=F64)
    c3 = torch.tensor([2.0, 1.0, -3.0], dtype=F64)
    n = c1.shape[0]
    psi = torch.tensor([0.2, -2.7, 1.4], dtype=F64)
    Rz = so3.rot_z(psi)
    v = so3.mv(Rz, torch.stack([c1, torch.zeros_like(c1), c3], -1))
    z = torch.zeros(n, 3, dtype=F64)
    out = run(z, v, Rz, z, 1, torch.zeros(n, 4, dtype=F64), split_fleet(n))
    kv_xy, kv_z = SPLIT_GAINS[2], SPLIT_GAINS[3]
    assert (out["theta_d"] - torch.atan2(-kv_xy * c1, G - kv_z * c3)).abs().max() < 1e-14
    assert out["phi_d"].abs().max() < 1e-14
    assert (out["f"] - SPLIT_MASS * (G - kv_z * c3)).abs().max() < 1e-13
