"""One step of the batched multirotor method and rollouts in FP64 (oracle;
test infrastructure only).

A step is: controller (Sec. IV, eqs. (1)-(9)) -> clamped rotor allocation ->
rigid-body integration, all at the pre-step state.  State layout per vehicle
(13 values): x(3), v(3), q(4; w,x,y,z), Omega(3).

Tracking loss of the differentiation workload (reading R18):
  L = (1/N) sum_i sum_{t=1..T} ( |x_{i,t} - x_goal,i|^2 + w_Omega |Omega_{i,t}|^2 )
over post-step states, x_goal = the position-mode target.  Its FP64
reverse-mode gradient comes from torch autograd; central finite differences
are provided for pinning it.
"""
import numpy as np
import torch

from . import allocation
from .controller import control
from .dynamics import integrate

F64 = torch.float64


def split(state):
    return state[:, 0:3], state[:, 3:6], state[:, 6:10], state[:, 10:13]


def step(state, mode, target, fleet, dt, g, tabs=None, traj=None):
    """state [N,13], mode [N], target [N,4] -> (next state [N,13], info)."""
    x, v, q, W = split(state)
    c = control(x, v, q, W, mode, target, fleet, g, traj)
    u, f_app, M_app, raw = allocation.allocate(c["f"], c["M"], fleet, tabs)
    xn, vn, qn, Wn = integrate(x, v, q, W, f_app, M_app, fleet, dt, g)
    info = {"f": c["f"], "M": c["M"], "f_app": f_app, "M_app": M_app, "u": u, "u_raw": raw}
    return torch.cat([xn, vn, qn, Wn], -1), info


def rollout(state0, mode, target, fleet, dt, g, steps, keep_states=False, traj=None):
    """Run ``steps`` steps; returns (final state, list of states or None, saturated
    rotor-step count per vehicle)."""
    tabs = allocation.tables(fleet)
    s = state0
    states = [] if keep_states else None
    sat = torch.zeros(state0.shape[0], dtype=torch.int64)
    for k in range(steps):
        tr = traj(k) if callable(traj) else traj      # traj may be a function of the step
        s, info = step(s, mode, target, fleet, dt, g, tabs, tr)
        sat += allocation.saturated_count(info["u_raw"].detach(), fleet)
        if keep_states:
            states.append(s)
    return s, states, sat


def clamp_margin(state0, mode, target, fleet, dt, g, steps):
    """Per vehicle, the smallest distance over the steps of a rollout of a raw
    rotor command to a clamp bound, relative to u_max.  Where it is small the
    loss has a kink close to the trajectory (the clamp of reading R20), and an
    FP32 run of the same rollout may pass the other side of it."""
    tabs = allocation.tables(fleet)
    s = state0
    m = torch.full((state0.shape[0],), float("inf"), dtype=state0.dtype)
    with torch.no_grad():
        for _ in range(steps):
            s, info = step(s, mode, target, fleet, dt, g, tabs)
            m = torch.minimum(m, allocation.clamp_distance(info["u_raw"], fleet))
    return m


def per_vehicle_loss(state0, mode, target, fleet, dt, g, steps, w_omega):
    """l_i = sum_{t=1..T} |x_t - x_goal|^2 + w_Omega |Omega_t|^2 (per vehicle)."""
    tabs = allocation.tables(fleet)
    s = state0
    goal = target[:, 0:3]
    li = torch.zeros(state0.shape[0], dtype=state0.dtype)
    for _ in range(steps):
        s, _ = step(s, mode, target, fleet, dt, g, tabs)
        li = li + ((s[:, 0:3] - goal) ** 2).sum(-1) + w_omega * (s[:, 10:13] ** 2).sum(-1)
    return li, s


def loss_and_grad(state0, mode, target, fleet, dt, g, steps, w_omega, n_total=None):
    """L = (1/n_total) sum_i l_i and its FP64 reverse-mode gradient with respect to
    the per-vehicle gains [N,10] and initial states [N,13]."""
    n_total = n_total or state0.shape[0]
    gains = fleet.gains.clone().requires_grad_(True)
    s0 = state0.clone().requires_grad_(True)
    li, _ = per_vehicle_loss(s0, mode, target, fleet.with_gains(gains), dt, g, steps, w_omega)
    L = li.sum() / n_total
    dg, ds = torch.autograd.grad(L, (gains, s0))
    return L.detach(), li.detach(), dg, ds


def fd_grad(state0, mode, target, fleet, dt, g, steps, w_omega, h=1e-3, n_total=None):
    """Central finite differences of L with respect to every gain and state
    component.  Vehicles are independent, so component k is perturbed in all
    vehicles at once and read off per vehicle.  Also returns, per vehicle and
    component, whether the +h and -h runs crossed a clamp boundary."""
    n_total = n_total or state0.shape[0]
    tabs_fleet = fleet

    def run(s0, fl):
        li, _ = per_vehicle_loss(s0, mode, target, fl, dt, g, steps, w_omega)
        return li

    def sat_pattern(s0, fl):
        s = s0
        tabs = allocation.tables(fl)
        pats = []
        for _ in range(steps):
            s, info = step(s, mode, target, fl, dt, g, tabs)
            raw = info["u_raw"]
            pats.append((raw < fl.u_min[:, None]) | (raw > fl.u_max[:, None]))
        return torch.stack(pats, 1)

    N = state0.shape[0]
    dg = torch.zeros(N, 10, dtype=F64)
    ds = torch.zeros(N, 13, dtype=F64)
    kink_g = torch.zeros(N, 10, dtype=torch.bool)
    kink_s = torch.zeros(N, 13, dtype=torch.bool)
    with torch.no_grad():
        for k in range(10):
            gp = fleet.gains.clone(); gp[:, k] += h
            gm = fleet.gains.clone(); gm[:, k] -= h
            fp, fm = fleet.with_gains(gp), fleet.with_gains(gm)
            dg[:, k] = (run(state0, fp) - run(state0, fm)) / (2 * h) / n_total
            kink_g[:, k] = (sat_pattern(state0, fp) != sat_pattern(state0, fm)).flatten(1).any(-1)
        for k in range(13):
            sp = state0.clone(); sp[:, k] += h
            sm = state0.clone(); sm[:, k] -= h
            ds[:, k] = (run(sp, tabs_fleet) - run(sm, tabs_fleet)) / (2 * h) / n_total
            kink_s[:, k] = (sat_pattern(sp, fleet) != sat_pattern(sm, fleet)).flatten(1).any(-1)
    return dg, ds, kink_g, kink_s


def from_workload_arrays(state0_soa, mode, target_soa):
    """Upcast the FP32 structure-of-arrays inputs to vehicle-major FP64."""
    s = torch.as_tensor(np.ascontiguousarray(np.asarray(state0_soa, np.float32).T), dtype=F64)
    t = torch.as_tensor(np.ascontiguousarray(np.asarray(target_soa, np.float32).T), dtype=F64)
    return s, torch.as_tensor(np.asarray(mode, np.int64)), t
