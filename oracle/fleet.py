"""Per-vehicle parameters in FP64 (oracle; test infrastructure only).

Every vehicle carries its own mass m, inertia J = diag(J1, J2, J3) (Sec. IV
symbol table), the ten controller gains in the order
(kx_xy, kx_z, kv_xy, kv_z, kR_x, kR_y, kR_z, kW_x, kW_y, kW_z), its rotor
count, arm length, yaw-torque coefficient and rotor thrust limits.

``from_groups`` expands contiguous vehicle groups (each with defaults) and an
optional per-vehicle override table with rows
(m, J1, J2, J3, 10 gains, arm, u_max).
"""
from dataclasses import dataclass

import numpy as np
import torch

F64 = torch.float64


@dataclass
class Fleet:
    m: torch.Tensor         # [N]
    J: torch.Tensor         # [N,3]
    gains: torch.Tensor     # [N,10]
    arm: torch.Tensor       # [N]
    c_tau: torch.Tensor     # [N]
    u_min: torch.Tensor     # [N]
    u_max: torch.Tensor     # [N]
    n_rotors: torch.Tensor  # [N] int64

    @property
    def n(self):
        return self.m.shape[0]

    def select(self, idx):
        return Fleet(*(getattr(self, f)[idx] for f in self.__dataclass_fields__))

    def with_gains(self, gains):
        return Fleet(self.m, self.J, gains, self.arm, self.c_tau, self.u_min, self.u_max,
                     self.n_rotors)

    @staticmethod
    def from_groups(groups, n, vparams=None):
        m = np.zeros(n)
        J = np.zeros((n, 3))
        gains = np.zeros((n, 10))
        arm = np.zeros(n)
        c_tau = np.zeros(n)
        u_min = np.zeros(n)
        u_max = np.zeros(n)
        nr = np.zeros(n, np.int64)
        covered = 0
        for gr in groups:
            sl = slice(gr.first, gr.first + gr.count)
            m[sl] = gr.mass
            J[sl] = np.asarray(gr.inertia, np.float32)
            gains[sl] = np.asarray(gr.gains, np.float32)
            arm[sl] = np.float32(gr.arm)
            c_tau[sl] = np.float32(gr.c_tau)
            u_min[sl] = np.float32(gr.u_min)
            u_max[sl] = np.float32(gr.u_max)
            nr[sl] = gr.n_rotors
            covered += gr.count
        if covered != n:
            raise ValueError("groups must cover all vehicles")
        # Group defaults reach the GPU as FP32; the oracle sees the same values.
        m = m.astype(np.float32).astype(np.float64)
        if vparams is not None:
            vp = np.asarray(vparams, np.float32).astype(np.float64)
            m = vp[0].copy()
            J = vp[1:4].T.copy()
            gains = vp[4:14].T.copy()
            arm = vp[14].copy()
            u_max = vp[15].copy()
        t = lambda a: torch.as_tensor(np.asarray(a, np.float64), dtype=F64)
        return Fleet(t(m), t(J), t(gains), t(arm), t(c_tau), t(u_min), t(u_max),
                     torch.as_tensor(nr))
