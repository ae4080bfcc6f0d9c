"""Pins of the oracle's full geometric tracking law (mode 4): hover
equilibrium, the desired frame, agreement with the paper's Z-Y-X
construction where the two coincide, the restored feed-forward term in
closed form, and first-order convergence of closed-loop tracking of a
circle whose feed-forward is known exactly."""
import math

import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import controller, lee, so3, step as ostep
from oracle.fleet import Fleet
from workloads import Group

F64 = torch.float64
G = 9.81


def quat_of(R):
    return torch.as_tensor(Rotation.from_matrix(R.numpy()).as_quat()[:, [3, 0, 1, 2]])


def traj_rows(xd, vd, ad, psi, wd, dwd):
    return torch.cat([xd, vd, ad, psi[:, None], wd, dwd], -1)


def test_hover_equilibrium():
    n = 5
    psi = torch.linspace(-3, 3, n, dtype=F64)
    xd = torch.randn(n, 3, generator=torch.Generator().manual_seed(0), dtype=F64)
    z = torch.zeros(n, 3, dtype=F64)
    fleet = Fleet.from_groups([Group(0, n)], n)
    tr = traj_rows(xd, z, z, psi, z, z)
    out = lee.lee_tracking(xd, z, quat_of(so3.rot_z(psi)), z, tr, fleet, G)
    assert (out["f"] - G).abs().max() < 1e-14
    assert out["M"].abs().max() < 1e-14


def test_desired_frame_properties():
    g = torch.Generator().manual_seed(1)
    F = torch.randn(300, 3, generator=g, dtype=F64) * 5
    psi = (torch.rand(300, generator=g, dtype=F64) * 2 - 1) * math.pi
    Rd = lee.desired_frame(F, psi)
    I = torch.eye(3, dtype=F64)
    assert (Rd.transpose(-1, -2) @ Rd - I).abs().max() < 1e-14
    assert (torch.linalg.det(Rd) - 1).abs().max() < 1e-14
    assert (Rd[:, :, 2] - F / F.norm(dim=-1, keepdim=True)).abs().max() < 1e-15
    b1d = torch.stack([torch.cos(psi), torch.sin(psi), 0 * psi], -1)
    assert (Rd[:, :, 1] * b1d).sum(-1).abs().max() < 1e-14          # b2c is orthogonal to b1d
    assert ((Rd[:, :, 0] * b1d).sum(-1) >= 0).all()                 # b1c leans towards b1d


def test_matches_zyx_construction_for_pure_roll_or_pitch():
    """With no feed-forward, the tracking mode equals the position mode (eq. (1)
    with eqs. (8)-(9)) whenever the commanded tilt is a pure roll or a pure
    pitch in the heading frame."""
    n = 6
    g = torch.Generator().manual_seed(2)
    psi = (torch.rand(n, generator=g, dtype=F64) * 2 - 1) * math.pi
    d = torch.rand(n, generator=g, dtype=F64) * 2 - 1
    z = torch.zeros(n, 3, dtype=F64)
    R = torch.as_tensor(Rotation.random(n, random_state=3).as_matrix())
    W = torch.randn(n, 3, generator=g, dtype=F64) * 0.2
    fleet = Fleet.from_groups([Group(0, n)], n)
    for axis in (0, 1):          # offset along the heading (pitch) or across it (roll)
        off = torch.zeros(n, 3, dtype=F64)
        off[:, axis] = d
        xd = so3.mv(so3.rot_z(psi), off)
        tgt = torch.cat([xd, psi[:, None]], -1)
        c0 = controller.control(z, z, quat_of(R), W, torch.zeros(n), tgt, fleet, G)
        c4 = lee.lee_tracking(z, z, quat_of(R), W, traj_rows(xd, z, z, psi, z, z), fleet, G)
        assert (c0["R_d"] - c4["R_d"]).abs().max() < 1e-14
        assert (c0["M"] - c4["M"]).abs().max() < 1e-13
        assert (c0["f"] - c4["f"]).abs().max() < 1e-13


def test_feed_forward_term_closed_form():
    """On the desired attitude and rate: e_R = 0, e_Omega = 0 and
    M = Omega_d x J Omega_d + J dOmega_d (the term the paper drops)."""
    n = 40
    g = torch.Generator().manual_seed(4)
    xd = torch.randn(n, 3, generator=g, dtype=F64)
    vd = torch.randn(n, 3, generator=g, dtype=F64)
    ad = torch.randn(n, 3, generator=g, dtype=F64)
    psi = torch.rand(n, generator=g, dtype=F64) * 6 - 3
    wd = torch.randn(n, 3, generator=g, dtype=F64)
    dwd = torch.randn(n, 3, generator=g, dtype=F64)
    fleet = Fleet.from_groups([Group(0, n)], n)
    e3 = torch.tensor([0, 0, 1.0], dtype=F64)
    Rd = lee.desired_frame(fleet.m[:, None] * (ad + G * e3), psi)
    out = lee.lee_tracking(xd, vd, quat_of(Rd), wd, traj_rows(xd, vd, ad, psi, wd, dwd), fleet, G)
    J = fleet.J
    assert out["e_R"].abs().max() < 1e-14 and out["e_W"].abs().max() < 1e-13
    assert (out["M"] - (torch.cross(wd, J * wd, dim=-1) + J * dwd)).abs().max() < 1e-13


def circle_case(dt, T=2.0, r=1.0, w=1.0, h=2.0, psi0=0.3):
    n = 1
    fleet = Fleet.from_groups([Group(0, n)], n)
    m = float(fleet.m[0])
    e3 = np.array([0.0, 0.0, 1.0])

    def traj_at(t):
        c, s = math.cos(w * t), math.sin(w * t)
        xd = [r * c, r * s, h]
        vd = [-r * w * s, r * w * c, 0.0]
        ad = [-r * w * w * c, -r * w * w * s, 0.0]
        return xd, vd, ad, w * t + psi0

    xd, vd, ad, psi = traj_at(0.0)
    Rd0 = lee.desired_frame(torch.as_tensor((m * (np.array(ad) + G * e3))[None], dtype=F64),
                            torch.tensor([psi], dtype=F64))[0]
    wd = (Rd0.T @ torch.tensor([0.0, 0.0, w], dtype=F64))          # constant body rate, dOmega_d = 0

    def traj(k):
        xd, vd, ad, psi = traj_at(k * dt)
        return torch.tensor([xd + vd + ad + [psi] + wd.tolist() + [0.0, 0.0, 0.0]], dtype=F64)

    s0 = torch.tensor([xd + vd + quat_of(Rd0[None]).tolist()[0] + wd.tolist()], dtype=F64)
    steps = int(round(T / dt))
    s = s0
    tabs = ostep.allocation.tables(fleet)
    err = 0.0
    for k in range(steps):
        s, _ = ostep.step(s, torch.tensor([4]), torch.zeros(1, 4, dtype=F64), fleet, dt, G, tabs, traj(k))
        xk = traj_at((k + 1) * dt)[0]
        err = max(err, float((s[0, :3] - torch.tensor(xk, dtype=F64)).norm()))
    return err


def test_circle_tracking_converges_with_dt():
    e1 = circle_case(0.004)
    e2 = circle_case(0.002)
    print("circle tracking error", e1, e2)
    assert e2 < 5e-3
    assert 1.6 < e1 / e2 < 2.4
