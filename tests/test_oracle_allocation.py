"""Pins of the oracle's rotor allocation against the closed form that the
symmetric layouts fix and against an independent pseudo-inverse (NumPy)."""
import math

import numpy as np
import pytest
import torch

from oracle import allocation
from oracle.fleet import Fleet
from workloads import Group

F64 = torch.float64


@pytest.mark.parametrize("nr", [4, 6, 8])
def test_gram_matrix_is_diagonal(nr):
    l, ct = 0.13, 0.016
    A = allocation.allocation_matrix(nr, torch.tensor([l], dtype=F64), torch.tensor([ct], dtype=F64))[0]
    expect = torch.diag(torch.tensor([nr, l * l * nr / 2, l * l * nr / 2, ct * ct * nr], dtype=F64))
    assert (A @ A.T - expect).abs().max() < 1e-15


@pytest.mark.parametrize("nr", [4, 6, 8])
def test_pseudo_inverse_closed_form(nr):
    """u_i = f/n + 2 (Mx sin a_i - My cos a_i) / (n l) + s_i Mz / (n c_tau)."""
    l, ct = 0.21, 0.02
    fleet = Fleet.from_groups([Group(0, 50, n_rotors=nr, arm=l, c_tau=ct, u_min=-1e9, u_max=1e9)], 50)
    g = torch.Generator().manual_seed(nr)
    f = torch.rand(50, generator=g, dtype=F64) * 20
    M = torch.randn(50, 3, generator=g, dtype=F64)
    u, fa, Ma, raw = allocation.allocate(f, M, fleet)
    alpha = [math.pi / nr + 2 * math.pi * i / nr for i in range(nr)]
    l32, ct32 = float(np.float32(l)), float(np.float32(ct))
    for i, a in enumerate(alpha):
        s = 1.0 if i % 2 == 0 else -1.0
        ui = f / nr + 2 * (M[:, 0] * math.sin(a) - M[:, 1] * math.cos(a)) / (nr * l32) \
            + s * M[:, 2] / (nr * ct32)
        assert (raw[:, i] - ui).abs().max() < 1e-12
    # unclamped: applied wrench equals the command
    assert (fa - f).abs().max() < 1e-12 and (Ma - M).abs().max() < 1e-12
    A = allocation.allocation_matrix(nr, fleet.arm[:1], fleet.c_tau[:1])[0].numpy()
    np.testing.assert_allclose(torch.linalg.pinv(allocation.allocation_matrix(
        nr, fleet.arm[:1], fleet.c_tau[:1]))[0].numpy(), np.linalg.pinv(A), atol=1e-12)
    np.testing.assert_allclose(A @ np.linalg.pinv(A), np.eye(4), atol=1e-13)


def test_quad_pseudo_inverse_is_inverse():
    A = allocation.allocation_matrix(4, torch.tensor([0.13], dtype=F64), torch.tensor([0.016], dtype=F64))[0]
    assert (torch.linalg.pinv(A) - torch.linalg.inv(A)).abs().max() < 1e-12


def test_x_layout_geometry():
    """Quad X: rotors at 45, 135, 225, 315 deg with alternating spin."""
    alpha, spin = allocation.layout(4)
    np.testing.assert_allclose(np.degrees(alpha.numpy()), [45, 135, 225, 315])
    assert spin.tolist() == [1.0, -1.0, 1.0, -1.0]


def test_clamp_bounds_and_hover_split():
    fleet = Fleet.from_groups([Group(0, 3, n_rotors=6, u_min=0.0, u_max=2.0)], 3)
    f = torch.tensor([6.0, 50.0, -3.0], dtype=F64)
    M = torch.zeros(3, 3, dtype=F64)
    u, fa, Ma, raw = allocation.allocate(f, M, fleet)
    assert (u[0, :6] - 1.0).abs().max() < 1e-14                           # hover: f/n each
    assert torch.equal(u[1, :6], torch.full((6,), 2.0, dtype=F64))     # clamped at u_max
    assert torch.equal(u[2, :6], torch.zeros(6, dtype=F64))            # clamped at u_min
    assert torch.equal(u[:, 6:], torch.zeros(3, 2, dtype=F64))
    assert allocation.saturated_count(raw, fleet).tolist() == [0, 6, 6]


def test_clamp_distance_closed_form_and_rotor_columns():
    """Distance of the raw command nearest a clamp bound, relative to u_max:
    hover split of a 1 kg quad (u = g/4 in [0, 6]) gives min(g/4, 6 - g/4)/6;
    padding columns past a vehicle's rotor count do not count."""
    from oracle import Fleet
    import workloads
    groups = [workloads.Group(0, 1), workloads.Group(1, 1, n_rotors=6, u_max=5.0)]
    fleet = Fleet.from_groups(groups, 2, None)
    raw = torch.full((2, 8), -100.0, dtype=torch.float64)
    raw[0, :4] = 9.81 / 4
    raw[1, :6] = torch.tensor([1.0, 2.0, 4.8, 3.0, 2.5, 1.5], dtype=torch.float64)   # 0.2 below u_max
    d = allocation.clamp_distance(raw, fleet)
    assert abs(float(d[0]) - min(9.81 / 4, 6 - 9.81 / 4) / 6) < 1e-15
    assert abs(float(d[1]) - 0.2 / 5.0) < 1e-15


def test_clamp_margin_of_a_hovering_rollout():
    """A hovering quad is a fixed point: every step's raw commands are g/4."""
    import oracle
    import workloads
    from oracle import Fleet
    fleet = Fleet.from_groups([workloads.Group(0, 3)], 3, None)
    s0 = torch.zeros(3, 13, dtype=torch.float64)
    s0[:, 6] = 1.0
    s0[:, 0:3] = torch.tensor([[0.0, 0.0, 0.0], [1.0, -2.0, 3.0], [0.5, 0.5, -0.5]], dtype=torch.float64)
    tgt = torch.zeros(3, 4, dtype=torch.float64)
    tgt[:, 0:3] = s0[:, 0:3]
    m = oracle.step.clamp_margin(s0, torch.zeros(3, dtype=torch.int64), tgt, fleet, 0.01, 9.81, 30)
    assert (m - min(9.81 / 4, 6 - 9.81 / 4) / 6).abs().max() < 1e-12
