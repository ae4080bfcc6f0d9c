"""SO(3) helpers in FP64 (oracle; test infrastructure only).

Conventions (Sec. IV symbol table): R maps body-frame coordinates to the
inertial frame E; quaternions are Hamilton, scalar first (w, x, y, z).
All functions are batched over a leading vehicle axis.
"""
import torch


def hat(w):
    """so(3) hat map: hat(w) @ b == cross(w, b).  w: [N,3] -> [N,3,3]."""
    z = torch.zeros_like(w[:, 0])
    return torch.stack([
        torch.stack([z, -w[:, 2], w[:, 1]], -1),
        torch.stack([w[:, 2], z, -w[:, 0]], -1),
        torch.stack([-w[:, 1], w[:, 0], z], -1),
    ], -2)


def vee(S):
    """Vee map so(3) -> R^3, the inverse of ``hat`` (used by eq. (3))."""
    return torch.stack([S[:, 2, 1], S[:, 0, 2], S[:, 1, 0]], -1)


def quat_to_rot(q):
    """Rotation matrix of a unit quaternion q = (w, x, y, z): [N,4] -> [N,3,3].

    Uses the unit-norm form (no division by |q|^2)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def quat_mul(a, b):
    """Hamilton product a (x) b, scalar first: [N,4] x [N,4] -> [N,4]."""
    aw, av = a[:, :1], a[:, 1:]
    bw, bv = b[:, :1], b[:, 1:]
    w = aw * bw - (av * bv).sum(-1, keepdim=True)
    v = aw * bv + bw * av + torch.cross(av, bv, dim=-1)
    return torch.cat([w, v], -1)


def rot_x(a):
    c, s, o, z = torch.cos(a), torch.sin(a), torch.ones_like(a), torch.zeros_like(a)
    return torch.stack([torch.stack([o, z, z], -1),
                        torch.stack([z, c, -s], -1),
                        torch.stack([z, s, c], -1)], -2)


def rot_y(a):
    c, s, o, z = torch.cos(a), torch.sin(a), torch.ones_like(a), torch.zeros_like(a)
    return torch.stack([torch.stack([c, z, s], -1),
                        torch.stack([z, o, z], -1),
                        torch.stack([-s, z, c], -1)], -2)


def rot_z(a):
    c, s, o, z = torch.cos(a), torch.sin(a), torch.ones_like(a), torch.zeros_like(a)
    return torch.stack([torch.stack([c, -s, z], -1),
                        torch.stack([s, c, z], -1),
                        torch.stack([z, z, o], -1)], -2)


def yaw_of(R):
    """Current yaw psi (symbol table of Sec. IV) read as the Z angle of a
    Z-Y-X Euler decomposition, matching the rotation order of eq. (1):
    psi = atan2(R[1,0], R[0,0]); psi = 0 when both entries vanish (pitch of
    +-90 deg), where the decomposition leaves yaw undefined."""
    r10, r00 = R[:, 1, 0], R[:, 0, 0]
    degenerate = (r10 == 0) & (r00 == 0)
    psi = torch.atan2(r10, r00)
    return torch.where(degenerate, torch.zeros_like(psi), psi)


def mv(A, b):
    """Batched matrix-vector product [N,3,3] x [N,3] -> [N,3]."""
    return (A @ b.unsqueeze(-1)).squeeze(-1)
