"""Helpers shared by the GPU parity tests: run the FP64 oracle on the same
inputs and measure the FP32 GPU results against it."""
import numpy as np
import pytest
import torch

import oracle

F64 = torch.float64


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def oracle_inputs(wl, state_soa=None, target_soa=None):
    s0, mode, tgt = oracle.step.from_workload_arrays(
        wl.state0 if state_soa is None else state_soa, wl.mode,
        wl.target if target_soa is None else target_soa)
    fleet = oracle.Fleet.from_groups(wl.groups, wl.n, wl.vparams)
    return s0, mode, tgt, fleet


def to_vm64(t):
    """Device SoA [R, n] tensor -> host vehicle-major FP64 [n, R]."""
    return t.detach().to("cpu", torch.float64).T.contiguous()


def wrench_errors(W_gpu, info, fleet, g, near_kink=None):
    """Relative errors of commanded and applied wrench with the scale floors
    m g (thrust) and m g l (moment).  W_gpu: host FP64 [n, 8]."""
    sf = fleet.m * g
    sM = fleet.m * g * fleet.arm
    ef = (W_gpu[:, 0] - info["f"]).abs() / torch.maximum(info["f"].abs(), sf)
    eM = (W_gpu[:, 1:4] - info["M"]).norm(dim=-1) / torch.maximum(info["M"].norm(dim=-1), sM)
    efa = (W_gpu[:, 4] - info["f_app"]).abs() / torch.maximum(info["f_app"].abs(), sf)
    eMa = (W_gpu[:, 5:8] - info["M_app"]).norm(dim=-1) / torch.maximum(info["M_app"].norm(dim=-1), sM)
    if near_kink is not None:
        efa = torch.where(near_kink, torch.zeros_like(efa), efa)
        eMa = torch.where(near_kink, torch.zeros_like(eMa), eMa)
    return ef, eM, efa, eMa


def near_clamp(info, fleet, rel=1e-4):
    """Vehicles with a raw rotor command within rel*u_max of a clamp bound:
    there FP32 and FP64 may legitimately take different clamp branches."""
    raw = info["u_raw"]
    tol = rel * fleet.u_max[:, None]
    near = ((raw - fleet.u_min[:, None]).abs() < tol) | ((raw - fleet.u_max[:, None]).abs() < tol)
    nr = fleet.n_rotors
    cols = torch.arange(8)[None, :] < nr[:, None]
    return (near & cols).any(-1)


def same_rotation_err(q_a, q_b):
    """max |R(q_a) - R(q_b)| per vehicle (q and -q are the same attitude)."""
    Ra = oracle.so3.quat_to_rot(q_a)
    Rb = oracle.so3.quat_to_rot(q_b)
    return (Ra - Rb).abs().flatten(1).max(-1).values
