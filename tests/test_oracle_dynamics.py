"""Pins of the oracle's step and integrator: discrete closed forms (free
fall, torque-free axisymmetric body, pure roll error), the hover fixed
point, and invariances of whole trajectories."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import so3, step as ostep
from oracle.fleet import Fleet
from workloads import Group

F64 = torch.float64
G = 9.81


def state(x, v, q, W):
    return torch.cat([x, v, q, W], -1)


def test_free_fall_discrete_closed_form():
    """Wrench mode with f = 0, M = 0: v_n = v0 - n g dt e3,
    x_n = x0 + n dt v0 - g dt^2 n (n+1)/2 e3 (exact for the integrator);
    the continuous parabola is met within g dt t / 2."""
    n, dt, T = 16, 0.01, 300
    g = torch.Generator().manual_seed(0)
    x0 = torch.randn(n, 3, generator=g, dtype=F64)
    v0 = torch.randn(n, 3, generator=g, dtype=F64)
    q0 = torch.as_tensor(Rotation.random(n, random_state=1).as_quat()[:, [3, 0, 1, 2]])
    W0 = torch.zeros(n, 3, dtype=F64)
    fleet = Fleet.from_groups([Group(0, n)], n)
    mode = torch.full((n,), 3)
    tgt = torch.zeros(n, 4, dtype=F64)
    sT, _, _ = ostep.rollout(state(x0, v0, q0, W0), mode, tgt, fleet, dt, G, T)
    e3 = torch.tensor([0, 0, 1.0], dtype=F64)
    v_exact = v0 - T * G * dt * e3
    x_exact = x0 + T * dt * v0 - G * dt * dt * T * (T + 1) / 2 * e3
    assert (sT[:, 3:6] - v_exact).abs().max() < 1e-12
    assert (sT[:, 0:3] - x_exact).abs().max() < 1e-12
    t = T * dt
    x_cont = x0 + v0 * t - 0.5 * G * t * t * e3
    assert (sT[:, 0:3] - x_cont).abs().max() <= G * dt * t / 2 + 1e-12


def test_torque_free_axisymmetric_body():
    """J1 = J2, zero wrench: Omega_3 constant and, with lam = (J3-J1) Omega_3 / J1,
    (Omega_1 + i Omega_2)_n = (1 + i lam dt)^n (Omega_1 + i Omega_2)_0 for the
    explicit rate update; the continuous solution exp(i lam t) is approached O(dt)."""
    n, dt, T = 8, 0.001, 400
    g = torch.Generator().manual_seed(2)
    W0 = torch.randn(n, 3, generator=g, dtype=F64) * 3
    q0 = torch.as_tensor(Rotation.random(n, random_state=3).as_quat()[:, [3, 0, 1, 2]])
    J = (0.007, 0.007, 0.012)
    fleet = Fleet.from_groups([Group(0, n, inertia=J)], n)
    z = torch.zeros(n, 3, dtype=F64)
    sT, _, _ = ostep.rollout(state(z, z, q0, W0), torch.full((n,), 3), torch.zeros(n, 4, dtype=F64),
                             fleet, dt, G, T)
    J1, J3 = float(np.float32(J[0])), float(np.float32(J[2]))
    lam = (J3 - J1) * W0[:, 2].numpy() / J1
    w0 = W0[:, 0].numpy() + 1j * W0[:, 1].numpy()
    wT = sT[:, 10].numpy() + 1j * sT[:, 11].numpy()
    np.testing.assert_allclose(wT, (1 + 1j * lam * dt) ** T * w0, rtol=1e-12, atol=1e-12)
    assert (sT[:, 12] - W0[:, 2]).abs().max() < 1e-14
    cont = np.exp(1j * lam * T * dt) * w0
    assert np.abs(wT - cont).max() < 2 * np.abs(lam).max() ** 2 * T * dt * dt * np.abs(w0).max()
    assert (sT[:, 6:10].norm(dim=-1) - 1).abs().max() < 1e-14


def test_hover_is_a_fixed_point_of_the_step():
    n = 6
    psi = torch.linspace(-3, 3, n, dtype=F64)
    xg = torch.randn(n, 3, generator=torch.Generator().manual_seed(4), dtype=F64)
    q = torch.stack([torch.cos(psi / 2), 0 * psi, 0 * psi, torch.sin(psi / 2)], -1)
    z = torch.zeros(n, 3, dtype=F64)
    s = state(xg, z, q, z)
    fleet = Fleet.from_groups([Group(0, n)], n)
    tgt = torch.cat([xg, psi[:, None]], -1)
    s1, info = ostep.step(s, torch.zeros(n), tgt, fleet, 0.01, G)
    assert (s1 - s).abs().max() < 1e-15
    assert (info["u"][:, :4] - float(np.float32(1.0)) * G / 4).abs().max() < 1e-14


def test_pure_roll_error_one_step_recurrence():
    """Attitude mode, level command, R = R_z(psi) R_x(a), Omega = (w, 0, 0),
    f = m g (no saturation): gyroscopic terms cancel, so
    Omega_1+ = w + dt (-kR_x sin a - kW_x w) / J1 and Omega_2+ = Omega_3+ = 0."""
    a = torch.tensor([0.05, -0.2, 0.4], dtype=F64)
    w = torch.tensor([0.3, -0.1, 0.0], dtype=F64)
    psi = torch.tensor([0.5, -1.0, 2.0], dtype=F64)
    n, dt = 3, 0.01
    R = so3.rot_z(psi) @ so3.rot_x(a)
    q = torch.as_tensor(Rotation.from_matrix(R.numpy()).as_quat()[:, [3, 0, 1, 2]])
    z = torch.zeros(n, 3, dtype=F64)
    W = torch.stack([w, 0 * w, 0 * w], -1)
    fleet = Fleet.from_groups([Group(0, n)], n)
    tgt = torch.tensor([[0.0, 0.0, 0.0, G]] * n, dtype=F64)
    s1, info = ostep.step(state(z, z, q, W), torch.full((n,), 2), tgt, fleet, dt, G)
    kR, kW, J1 = fleet.gains[0, 4], fleet.gains[0, 7], fleet.J[0, 0]
    expect = w + dt * (-kR * torch.sin(a) - kW * w) / J1
    assert (s1[:, 10] - expect).abs().max() < 1e-12
    assert s1[:, 11:13].abs().max() < 1e-12


def _random_fleet_state(n, seed):
    g = torch.Generator().manual_seed(seed)
    x = torch.randn(n, 3, generator=g, dtype=F64)
    v = torch.randn(n, 3, generator=g, dtype=F64) * 0.5
    q = torch.as_tensor(Rotation.random(n, random_state=seed).as_quat()[:, [3, 0, 1, 2]])
    # keep tilts moderate so the trajectories stay smooth
    R = so3.quat_to_rot(q)
    psi = so3.yaw_of(R)
    q = torch.stack([torch.cos(psi / 2), 0 * psi, 0 * psi, torch.sin(psi / 2)], -1)
    W = torch.randn(n, 3, generator=g, dtype=F64) * 0.2
    return state(x, v, q, W), g


def test_trajectory_yaw_equivariance_and_translation_invariance():
    """Rotating the initial state and the goal (and the yaw command) about e3
    by b rotates the whole position-mode trajectory; translating x and x_d by
    c translates it."""
    n, T = 32, 60
    s0, g = _random_fleet_state(n, 5)
    xg = torch.randn(n, 3, generator=g, dtype=F64)
    psi_d = torch.rand(n, generator=g, dtype=F64)
    tgt = torch.cat([xg, psi_d[:, None]], -1)
    fleet = Fleet.from_groups([Group(0, n)], n)
    mode = torch.zeros(n)
    base, _, _ = ostep.rollout(s0, mode, tgt, fleet, 0.01, G, T)
    b = torch.rand(n, generator=g, dtype=F64) * 4 - 2
    Rz = so3.rot_z(b)
    qz = torch.stack([torch.cos(b / 2), 0 * b, 0 * b, torch.sin(b / 2)], -1)
    s0r = state(so3.mv(Rz, s0[:, 0:3]), so3.mv(Rz, s0[:, 3:6]), so3.quat_mul(qz, s0[:, 6:10]),
                s0[:, 10:13])
    tgtr = torch.cat([so3.mv(Rz, xg), (psi_d + b)[:, None]], -1)
    rot, _, _ = ostep.rollout(s0r, mode, tgtr, fleet, 0.01, G, T)
    assert (rot[:, 0:3] - so3.mv(Rz, base[:, 0:3])).abs().max() < 1e-11
    assert (rot[:, 3:6] - so3.mv(Rz, base[:, 3:6])).abs().max() < 1e-11
    assert (so3.quat_to_rot(rot[:, 6:10]) - Rz @ so3.quat_to_rot(base[:, 6:10])).abs().max() < 1e-11
    assert (rot[:, 10:13] - base[:, 10:13]).abs().max() < 1e-11
    c = torch.tensor([[3.0, -7.0, 11.0]], dtype=F64)
    tr, _, _ = ostep.rollout(state(s0[:, 0:3] + c, s0[:, 3:6], s0[:, 6:10], s0[:, 10:13]), mode,
                             torch.cat([xg + c, psi_d[:, None]], -1), fleet, 0.01, G, T)
    assert (tr[:, 0:3] - c - base[:, 0:3]).abs().max() < 1e-11
    assert (tr[:, 3:] - base[:, 3:]).abs().max() < 1e-11


def test_quaternion_update_constant_body_rate():
    """Omega = (0, 0, w) on a body with J1 = J2 stays constant; each step then
    right-multiplies q by the unit quaternion of (1, dt w/2 e3), a rotation
    by 2 atan(dt w / 2) about b3: R_n = R_0 Rot(e3, 2 n atan(dt w / 2))."""
    n, dt, T = 5, 0.01, 250
    w = torch.tensor([0.5, -2.0, 3.0, 7.0, -0.1], dtype=F64)
    q0 = torch.as_tensor(Rotation.random(n, random_state=8).as_quat()[:, [3, 0, 1, 2]])
    z = torch.zeros(n, 3, dtype=F64)
    W = torch.stack([0 * w, 0 * w, w], -1)
    fleet = Fleet.from_groups([Group(0, n)], n)
    sT, _, _ = ostep.rollout(state(z, z, q0, W), torch.full((n,), 3), torch.zeros(n, 4, dtype=F64),
                             fleet, dt, G, T)
    ang = 2 * T * torch.atan(dt * w / 2)
    expect = so3.quat_to_rot(q0) @ so3.rot_z(ang)
    assert (so3.quat_to_rot(sT[:, 6:10]) - expect).abs().max() < 1e-12
    assert torch.equal(sT[:, 10:13], W)
