"""FP64 CPU oracle of the batched multirotor step (test infrastructure only).

This package is the checker, not the product.  Only the test suite, the smoke
check of ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path: it is written from the paper
(Kulkarni, Forgaard, Alexis, "Aerial Gym -- Isaac Gym Simulator for Aerial
Robots", arXiv 2305.16510, Sec. IV, eqs. (1)-(9)) and from the published
definitions of the pieces the paper delegates to its physics engine.

Everything is plain ``torch.float64`` on the CPU, vectorised over vehicles,
written in the order and notation of the paper so that it can be read against
it.  Readings of silent or garbled passages (numbered; the modules cite
them as R1, R2, ...) are listed at the end of this docstring.

Modules
-------
so3          hat / vee, quaternion -> rotation, elementary rotations, yaw readout
controller   eqs. (1)-(9): attitude, velocity and position tracking modes
allocation   rotor layout, min-norm allocation, clamping
dynamics     rigid-body Newton-Euler and quaternion integration
step         one step, rollouts, tracking loss, FP64 reverse-mode gradient, FD
philox       Philox4x32-10 counter-based generator (Salmon et al., SC'11)
reset        counter-based reset masks, redraws (Box-Muller normals) and ascending compaction
stats        batch statistics
task         goal-reaching observation, reward and termination (imported on its own)
lee          full geometric tracking law with feed-forward (imported on its own)
obstacles    obstacle poses at environment reset (imported on its own)
raycast      depth images against primitive obstacles (imported on its own)

Every function is pinned by a CPU test against a closed form, an identity, a
hand-worked case or an independent implementation of a published definition,
and a planted mistake in it makes that pin fail (``tests/test_oracle_*.py``).

Parity status: the position-mode construction, the integrator, the rotor
layout and the mass scaling of uneven fleets are readings (no paper numbers
exist for them); they are pinned only by identities and closed forms, not by
values the paper prints ("parity unpinned" against the paper itself).

Readings
--------
The paper is silent, ambiguous or garbled on these points; the HIP path
implements the same readings independently.

R1  Frames: z-up inertial frame, gravity -g e3 (g = 9.81), thrust +f b3.  The
    symbol table's "along -b3" is Lee's z-down convention; eqs. (8)-(9) only
    give a level attitude at hover for z up.
R2  Eq. (7) adds an acceleration to a force; read F = m (a_d + g e3).  kx, kv
    are acceleration gains, kR, kW torque gains.
R3  Eqs. (8)-(9) are evaluated on the gravity-compensated F expressed in V
    (so R_d e3 = F/|F|), not on a_d.
R4  "b3 in V" (end of Sec. IV-B) is the current body b3 expressed in V; f is
    the projection of F on it and may be negative (then clamped).
R5  "e_R in R" is R^3.
R6  Angles are in radians (the symbol says degrees).
R7  Current yaw psi = atan2(R21, R11) (Z-Y-X, matching eq. (1)); 0 if both vanish.
R8  Position mode (named, no equations): a = kx (x_d - x) - kv v in E,
    F = m (a + g e3), expressed in R_z(psi_d), R_d = R_z(psi_d) R_y R_x,
    zero yaw rate, no acceleration feed-forward.
R9  Lee's feed-forward term -J(hat(Omega) R^T R_d Omega_d - R^T R_d dOmega_d) is
    dropped, as the paper says.
R10 Velocity commands are in the vehicle frame V.
R11 The yaw-rate command of velocity-mode vehicles is the 4th target value.
R12 Allocation: n rotors at alpha_i = pi/n + 2 pi i/n, arm l, spin (-1)^i,
    column i of A = (1, l sin a_i, -l cos a_i, s_i c_tau); u = clip(A^+ w).
R13 Eqs. (1)+(2) give Omega_d = psidot_d R_d^T e3, so eq. (4) is
    e_Omega = Omega - psidot_d R^T e3 (an identity used as a pin).
R14 Tilt degeneracies: theta_d = 0 when F_x = F_z = 0; phi_d = 0 when F = 0.
R15 Integrator: semi-implicit Euler (velocity, then position; rate, then
    quaternion with the new rate), controller at the pre-step state.
R16 Quaternions are Hamilton, scalar first; q and -q are the same attitude.
R17 Ten gains: (kx_xy, kx_z, kv_xy, kv_z, kR_x, kR_y, kR_z, kW_x, kW_y, kW_z).
R18 Loss: sum over post-step states t = 1..T, mean over vehicles; q0 is not
    normalised at entry; gradients are taken in ambient R^13.
R20 Clamp subgradient: d clip / du = 1 iff u_min <= u <= u_max (inclusive).
R22 Reset RNG: Philox4x32-10, key = seed, counters as in ``reset``.
R24 A reset redraws the state; a position-mode vehicle also gets a new goal
    (yaw command 0); other modes keep their command.
R26 Uneven fleets: arm l = 0.13 m^(1/3), rotor limit 24 m / n, kR and kW
    scaled by m^(5/3) before the +-20% jitter.
R28 Unknown mode codes command a zero wrench (then allocation and dynamics run).
"""
from . import so3, controller, allocation, dynamics, step, philox, reset, stats  # noqa: F401
from .fleet import Fleet  # noqa: F401
