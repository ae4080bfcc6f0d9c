"""Readings of passages the paper leaves silent, ambiguous or garbled
(oracle; test infrastructure only).  The HIP path implements the same
readings independently.

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
