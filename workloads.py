"""Seeded synthetic inputs for the batched multirotor step.

This module only draws input data (initial states, commands, vehicle
parameters, group layouts).  It holds none of the method's arithmetic: no
controller, allocation or dynamics.  Both the FP64 oracle (through the tests)
and the HIP path (through the tests and the benchmark) take their inputs from
here, so the two sides always see bit-identical FP32 inputs.

All draws use NumPy's ``Generator(Philox(seed))``.  Arrays handed out are the
ones the GPU receives: state as FP32 structure-of-arrays ``[13, N]`` in the
order x(3), v(3), q(4; w, x, y, z), Omega(3); targets as FP32 ``[4, N]``;
modes as int8 ``[N]``; optional per-vehicle parameters as FP32 ``[16, N]``.

Vehicle and workload constants come from the benchmark configurations of the
multirotor step (1,024 / 1,048,576 / 48 uneven groups / 65,536 / 4,194,304
vehicles); the paper's own benchmark scenario (Sec. VI: 2^17 robots, constant
attitude or velocity commands, 10 ms steps) is ``paper_context``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Per-vehicle parameter rows (vparams[16, N]).
VP_MASS, VP_J0 = 0, 1          # J occupies rows 1..3
VP_GAINS = 4                   # 10 gains occupy rows 4..13
VP_ARM, VP_UMAX = 14, 15
VPARAM_DIM = 16

# Gain layout: (kx_xy, kx_z, kv_xy, kv_z, kR_x, kR_y, kR_z, kW_x, kW_y, kW_z).
QUAD_GAINS = (2.0, 2.0, 2.0, 2.0, 1.6, 1.6, 0.6, 0.5, 0.5, 0.2)
QUAD_MASS = 1.0
QUAD_J = (0.007, 0.007, 0.012)
QUAD_ARM = 0.13
QUAD_CTAU = 0.016
QUAD_UMIN, QUAD_UMAX = 0.0, 6.0
G = 9.81


@dataclass
class Group:
    """A contiguous range of vehicles sharing a rotor layout and defaults."""
    first: int
    count: int
    n_rotors: int = 4
    arm: float = QUAD_ARM
    c_tau: float = QUAD_CTAU
    u_min: float = QUAD_UMIN
    u_max: float = QUAD_UMAX
    mass: float = QUAD_MASS
    inertia: tuple = QUAD_J
    gains: tuple = QUAD_GAINS


@dataclass
class Workload:
    name: str
    n: int
    dt: float
    steps: int
    groups: List[Group]
    state0: np.ndarray            # float32 [13, N]
    mode: np.ndarray              # int8 [N]
    target: np.ndarray            # float32 [4, N]
    vparams: Optional[np.ndarray] = None   # float32 [16, N] or None
    g: float = G
    seed: int = 0                 # key of the in-method counter-based RNG (resets)
    reset_prob: float = 0.0
    reset_lo: tuple = (-5.0, -5.0, -5.0)
    reset_hi: tuple = (5.0, 5.0, 5.0)
    meta: dict = field(default_factory=dict)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def random_initial_state(rng: np.random.Generator, n: int, pos_lo=-2.0, pos_hi=2.0,
                         vel_sigma=0.5, tilt_max=math.pi / 6, rate_sigma=0.2) -> np.ndarray:
    """Initial states: x ~ U[lo,hi]^3, v ~ N(0, vel_sigma^2)^3, attitude as a
    random horizontal tilt axis (angle beta ~ U[-pi,pi]) with tilt tau ~
    U[0, tilt_max] composed after a yaw psi0 ~ U[-pi,pi], Omega ~ N(0,
    rate_sigma^2)^3.  Returned as float32 [13, N]."""
    x = rng.uniform(pos_lo, pos_hi, size=(3, n))
    v = rng.normal(0.0, vel_sigma, size=(3, n))
    beta = rng.uniform(-math.pi, math.pi, size=n)
    tau = rng.uniform(0.0, tilt_max, size=n)
    psi0 = rng.uniform(-math.pi, math.pi, size=n)
    w = rng.normal(0.0, rate_sigma, size=(3, n))
    # q = qz(psi0) (x) q_axis((cos b, sin b, 0), tau), written out component-wise.
    a0, a3 = np.cos(psi0 / 2), np.sin(psi0 / 2)
    b0 = np.cos(tau / 2)
    b1 = np.sin(tau / 2) * np.cos(beta)
    b2 = np.sin(tau / 2) * np.sin(beta)
    q = np.stack([a0 * b0, a0 * b1 - a3 * b2, a0 * b2 + a3 * b1, a3 * b0])
    s = np.concatenate([x, v, q, w], axis=0)
    return s.astype(np.float32)


def _quad_groups(n: int) -> List[Group]:
    return [Group(first=0, count=n)]


def c1_parity(n: int = 1024, seed: int = 1, steps: int = 500) -> Workload:
    """1,024 X-quads, position mode to the origin with yaw 0, dt = 0.01 s."""
    rng = _rng(seed)
    s0 = random_initial_state(rng, n)
    tgt = np.zeros((4, n), np.float32)
    mode = np.zeros(n, np.int8)
    return Workload("c1_parity_1k_quads_position", n, 0.01, steps, _quad_groups(n),
                    s0, mode, tgt, seed=seed)


def c2_scale(n: int = 1_048_576, seed: int = 2, steps: int = 1000) -> Workload:
    """1M X-quads, mode uniform over {position, velocity, attitude}:
    position -> goal 0, yaw 0; velocity -> v_d ~ U[-2,2]^3 in the vehicle frame,
    yaw rate 0; attitude -> roll, pitch ~ U[-0.3,0.3] rad, yaw rate ~
    U[-1,1] rad/s, thrust ~ U[5,15] N."""
    rng = _rng(seed)
    s0 = random_initial_state(rng, n)
    mode = rng.integers(0, 3, size=n).astype(np.int8)
    tgt = np.zeros((4, n), np.float64)
    vd = rng.uniform(-2.0, 2.0, size=(3, n))
    att = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.3, 0.3, n),
                    rng.uniform(-1.0, 1.0, n), rng.uniform(5.0, 15.0, n)])
    m1, m2 = mode == 1, mode == 2
    tgt[:3, m1] = vd[:, m1]
    tgt[:, m2] = att[:, m2]
    return Workload("c2_scale_1M_quads_mixed_modes", n, 0.01, steps, _quad_groups(n),
                    s0, mode, tgt.astype(np.float32), seed=seed)


def c3_uneven(seed: int = 3, n_groups: int = 48, steps: int = 2000,
              size_lo: int = 512, size_hi: int = 131_072, scale: float = 1.0) -> Workload:
    """48 groups with log-uniform sizes in [512, 131072] (optionally scaled
    down by ``scale`` for quick tests), rotor count per group in {4, 6, 8},
    per-vehicle mass ~ U[0.5, 3] kg, inertia scaled by m^(5/3), arm by
    m^(1/3), rotor limit 24 m / n_rotors N, attitude gains scaled by m^(5/3),
    every gain jittered by a factor U[0.8, 1.2]; position mode to the origin."""
    rng = _rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(size_lo), math.log(size_hi), n_groups)))
    sizes = np.maximum(1, np.rint(sizes * scale)).astype(np.int64)
    rotors = rng.choice(np.array([4, 6, 8]), size=n_groups)
    n = int(sizes.sum())
    groups, first = [], 0
    for sz, nr in zip(sizes, rotors):
        groups.append(Group(first=first, count=int(sz), n_rotors=int(nr),
                            u_max=24.0 / float(nr)))
        first += int(sz)
    m = rng.uniform(0.5, 3.0, n)
    s53 = m ** (5.0 / 3.0)
    vp = np.zeros((VPARAM_DIM, n), np.float64)
    vp[VP_MASS] = m
    for k in range(3):
        vp[VP_J0 + k] = QUAD_J[k] * s53
    base = np.array(QUAD_GAINS)
    jit = rng.uniform(0.8, 1.2, size=(10, n))
    for k in range(10):
        scale_k = s53 if k >= 4 else 1.0
        vp[VP_GAINS + k] = base[k] * scale_k * jit[k]
    vp[VP_ARM] = QUAD_ARM * np.cbrt(m)
    nr_per_vehicle = np.repeat(rotors, sizes)
    vp[VP_UMAX] = 24.0 * m / nr_per_vehicle
    s0 = random_initial_state(rng, n)
    tgt = np.zeros((4, n), np.float32)
    mode = np.zeros(n, np.int8)
    return Workload("c3_uneven_48_groups", n, 0.01, steps, groups, s0, mode, tgt,
                    vparams=vp.astype(np.float32), seed=seed,
                    meta={"sizes": sizes.tolist(), "rotors": rotors.tolist()})


def c4_grad(n: int = 65_536, seed: int = 4, steps: int = 200) -> Workload:
    """65,536 quads, 200-step position rollout (differentiation workload);
    per-vehicle gains given explicitly (the C1 gains) so they can be
    differentiated."""
    rng = _rng(seed)
    s0 = random_initial_state(rng, n)
    vp = per_vehicle_defaults(n)
    tgt = np.zeros((4, n), np.float32)
    mode = np.zeros(n, np.int8)
    return Workload("c4_grad_64k_quads", n, 0.01, steps, _quad_groups(n), s0, mode, tgt,
                    vparams=vp, seed=seed, meta={"ckpt_every": 20})


def c5_large(n: int = 4_194_304, seed: int = 5, steps: int = 2000) -> Workload:
    """4M quads, position mode with goals ~ U[-5,5]^3, dt = 0.005 s, 1% of
    vehicles reset each step by the counter-based RNG."""
    rng = _rng(seed)
    s0 = random_initial_state(rng, n, pos_lo=-5.0, pos_hi=5.0)
    tgt = np.zeros((4, n), np.float32)
    tgt[:3] = rng.uniform(-5.0, 5.0, size=(3, n)).astype(np.float32)
    mode = np.zeros(n, np.int8)
    return Workload("c5_large_4M_quads_resets", n, 0.005, steps, _quad_groups(n), s0, mode,
                    tgt, seed=seed, reset_prob=0.01,
                    meta={"tune_subset": 262_144, "tune_steps": 100})


def paper_context(n: int = 131_072, seed: int = 6, steps: int = 1000) -> Workload:
    """The paper's benchmark shape (Sec. VI): 2^17 robots, no obstacles,
    constant attitude or velocity commands, 10 ms per step."""
    rng = _rng(seed)
    s0 = random_initial_state(rng, n)
    mode = rng.integers(1, 3, size=n).astype(np.int8)
    tgt = np.zeros((4, n), np.float64)
    vd = rng.uniform(-2.0, 2.0, size=(3, n))
    att = np.stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.3, 0.3, n),
                    rng.uniform(-1.0, 1.0, n), rng.uniform(5.0, 15.0, n)])
    m1, m2 = mode == 1, mode == 2
    tgt[:3, m1] = vd[:, m1]
    tgt[:, m2] = att[:, m2]
    return Workload("paper_context_131k_att_vel", n, 0.01, steps, _quad_groups(n), s0, mode,
                    tgt.astype(np.float32), seed=seed)


def per_vehicle_defaults(n: int, group: Optional[Group] = None) -> np.ndarray:
    """vparams [16, N] filled with one group's defaults."""
    gr = group or Group(0, n)
    vp = np.zeros((VPARAM_DIM, n), np.float32)
    vp[VP_MASS] = gr.mass
    vp[VP_J0:VP_J0 + 3] = np.asarray(gr.inertia, np.float32)[:, None]
    vp[VP_GAINS:VP_GAINS + 10] = np.asarray(gr.gains, np.float32)[:, None]
    vp[VP_ARM] = gr.arm
    vp[VP_UMAX] = gr.u_max
    return vp


def subset(wl: Workload, count: int, name: Optional[str] = None) -> Workload:
    """The first ``count`` vehicles of a workload (groups truncated)."""
    groups = []
    for gr in wl.groups:
        if gr.first >= count:
            break
        c = min(gr.count, count - gr.first)
        groups.append(Group(gr.first, c, gr.n_rotors, gr.arm, gr.c_tau, gr.u_min, gr.u_max,
                            gr.mass, gr.inertia, gr.gains))
    vp = None if wl.vparams is None else np.ascontiguousarray(wl.vparams[:, :count])
    return Workload(name or wl.name + f"_first{count}", count, wl.dt, wl.steps, groups,
                    np.ascontiguousarray(wl.state0[:, :count]), wl.mode[:count].copy(),
                    np.ascontiguousarray(wl.target[:, :count]), vp, wl.g, wl.seed,
                    wl.reset_prob, wl.reset_lo, wl.reset_hi, dict(wl.meta))
