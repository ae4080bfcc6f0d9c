"""Pins of the oracle's SO(3) helpers against identities and an independent
library (scipy.spatial.transform)."""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import so3

F64 = torch.float64


def rand_quat(n, seed=0):
    g = torch.Generator().manual_seed(seed)
    q = torch.randn(n, 4, generator=g, dtype=F64)
    return q / q.norm(dim=-1, keepdim=True)


def test_hat_vee_inverse_and_cross():
    g = torch.Generator().manual_seed(1)
    a = torch.randn(64, 3, generator=g, dtype=F64)
    b = torch.randn(64, 3, generator=g, dtype=F64)
    assert torch.equal(so3.vee(so3.hat(a)), a)
    np.testing.assert_allclose(so3.mv(so3.hat(a), b).numpy(), np.cross(a.numpy(), b.numpy()),
                               atol=1e-15)
    S = so3.hat(a)
    assert torch.equal(S, -S.transpose(-1, -2))


def test_quat_to_rot_matches_scipy_and_is_orthonormal():
    q = rand_quat(256)
    R = so3.quat_to_rot(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]].numpy()).as_matrix()
    np.testing.assert_allclose(R.numpy(), ref, atol=2e-15)
    I = torch.eye(3, dtype=F64).expand(256, 3, 3)
    assert (R.transpose(-1, -2) @ R - I).abs().max() < 1e-14
    assert (torch.linalg.det(R) - 1).abs().max() < 1e-14


def test_quat_product_composes_rotations_and_sign_invariance():
    q, p = rand_quat(128, 2), rand_quat(128, 3)
    Rq, Rp = so3.quat_to_rot(q), so3.quat_to_rot(p)
    assert (so3.quat_to_rot(so3.quat_mul(q, p)) - Rq @ Rp).abs().max() < 1e-14
    assert torch.equal(so3.quat_to_rot(-q), Rq)
    # scipy composes the same way: Rotation(q) * Rotation(p)
    ref = (Rotation.from_quat(q[:, [1, 2, 3, 0]].numpy())
           * Rotation.from_quat(p[:, [1, 2, 3, 0]].numpy())).as_matrix()
    np.testing.assert_allclose((Rq @ Rp).numpy(), ref, atol=1e-14)


def test_elementary_rotations_match_scipy():
    a = torch.linspace(-3.0, 3.0, 25, dtype=F64)
    for axis, fn in (("x", so3.rot_x), ("y", so3.rot_y), ("z", so3.rot_z)):
        ref = Rotation.from_euler(axis, a.numpy()).as_matrix()
        np.testing.assert_allclose(fn(a).numpy(), ref, atol=1e-15)


def test_yaw_readout_recovers_zyx_yaw():
    g = torch.Generator().manual_seed(4)
    n = 500
    alpha = (torch.rand(n, generator=g, dtype=F64) * 2 - 1) * math.pi * 0.999
    beta = (torch.rand(n, generator=g, dtype=F64) * 2 - 1) * (math.pi / 2) * 0.99
    gamma = (torch.rand(n, generator=g, dtype=F64) * 2 - 1) * math.pi
    R = so3.rot_z(alpha) @ so3.rot_y(beta) @ so3.rot_x(gamma)
    psi = so3.yaw_of(R)
    assert (psi - alpha).abs().max() < 1e-12
    ref = Rotation.from_matrix(R.numpy()).as_euler("ZYX")[:, 0]
    np.testing.assert_allclose(psi.numpy(), ref, atol=1e-12)


def test_yaw_readout_degenerate_pitch_is_zero():
    R = so3.rot_y(torch.tensor([math.pi / 2], dtype=F64))
    R[:, 0, 0] = 0.0
    R[:, 1, 0] = 0.0
    assert so3.yaw_of(R).item() == 0.0
