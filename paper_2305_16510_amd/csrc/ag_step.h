// ag_step.h -- per-vehicle device math of the batched multirotor step (gfx950).
//
// One lane owns one vehicle; everything here is straight-line FP32 scalar
// code on registers (the 3x3 algebra is not a dense contraction, so no MFMA).
// The three command modes share one branch-free path with selects, so a
// wavefront holding a mix of modes never diverges; a caller whose wavefront
// holds one mode instantiates step_core with that mode (MS), which folds the
// selects and drops the work the mode does not need.
//
// The controller follows Sec. IV of Kulkarni et al. (arXiv 2305.16510) with
// these algebraic rewrites, each exact in real arithmetic:
//   * eqs. (8)-(9) are evaluated trig-free: with h = sqrt(F_x^2 + F_z^2) and
//     n = |F|, cos(theta_d) = F_z/h, sin(theta_d) = F_x/h, cos(phi_d) = h/n,
//     sin(phi_d) = -F_y/n (theta_d = 0 if h = 0, phi_d = 0 if n = 0);
//   * eq. (1) is never formed: e_R of eq. (3) needs only six entries of
//     R_d^T R = T^T (R_z(psi)^T R) with T = R_y(theta_d) R_x(phi_d);
//   * eqs. (1)+(2) give Omega_d = psidot_d R_d^T e3, hence eq. (4) becomes
//     e_Omega = Omega - psidot_d R^T e3;
//   * the x-y gains are equal, so the commanded force is formed in the
//     inertial frame and rotated into the reference yaw frame afterwards,
//     with the target terms as per-vehicle constants;
//   * dt, the mass, 1/J and the 1/2 of eq. (3) are folded into per-vehicle
//     constants, which a fused launch computes once (loop-invariant).
// Allocation uses a unit-arm table per rotor layout: u = clip(A1^+ (f, M_x/l,
// M_y/l, M_z)), applied wrench (sum u, l (A1 u)_1, l (A1 u)_2, (A1 u)_3);
// for the quad X layout both products are 4-point butterflies, for hexa and
// octo they run over opposite-rotor pairs.
// Integration is semi-implicit Euler with quaternion renormalisation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#ifndef AG_DEV
#define AG_DEV __device__ __forceinline__
#endif

namespace ag {

// ---- per-group table (floats), staged in LDS by every block ---------------
constexpr int GSTRIDE = 96;       // floats per group entry (384 B, 16-B aligned rows)
constexpr int G_APINV = 0;        // 8 rotors x float4: unit-arm pseudo-inverse rows
constexpr int G_ACOL = 32;        // 8 rotors x float4: unit-arm allocation columns
constexpr int G_UMIN = 64;
constexpr int G_UMAX = 65;
constexpr int G_ARM = 66;
constexpr int G_INV_ARM = 67;
constexpr int G_MASS = 68;
constexpr int G_INV_MASS = 69;
constexpr int G_J = 70;           // 3
constexpr int G_JINV = 73;        // 3
constexpr int G_GAINS = 76;       // 10
constexpr int G_NR = 86;          // rotor count, as float
// quad-X layout only: the unit-arm A^+ and A are one +-1 pattern scaled per
// row, so the kernels use butterflies on these five scales instead of the
// rows above: A^+ thrust / x-y moment / yaw coefficients, sin(pi/4), c_tau
constexpr int G_Q_F = 87, G_Q_XY = 88, G_Q_Z = 89, G_Q_S = 90, G_Q_CT = 91;

// Event-fed fused kernels (one vehicle per lane) copy up to kEvStage reset
// events (16 floats each) of every wavefront into LDS at tile start, after
// the tile's group entries and their offsets: that region starts at this
// float offset (16-byte aligned).
constexpr int kEvStage = 64;
__host__ __device__ constexpr size_t ev_stage_offset(int span) {
    return ((size_t)span * GSTRIDE + (size_t)span + 1 + 3) & ~(size_t)3;
}

// ---- per-vehicle parameter rows (vparams) ---------------------------------
constexpr int VP_MASS = 0, VP_J = 1, VP_GAINS = 4, VP_ARM = 14, VP_UMAX = 15;

struct Params {
    float m, inv_m;
    float J0, J1, J2, Ji0, Ji1, Ji2;
    float dJ0, dJ1, dJ2;       // J2 - J1, J0 - J2, J1 - J0
    float kx_xy, kx_z, kv_xy, kv_z;
    float kR0, kR1, kR2, kW0, kW1, kW2;
    float arm, inv_arm, umin, umax;
    // quad butterflies: u = clip(H^T (cq_f f, cq_x M_x, cq_x M_y, cq_z M_z)),
    // applied moment (armq X0, armq X1, ctq X2) with X the butterfly sums
    float cq_f, cq_x, cq_z, armq, ctq;
    int nr;
};

// Derived command: the 4 raw target values plus cos/sin of the command
// angles (psi_d in position mode, phi_d in attitude mode; theta_d).
struct Cmd {
    int mode;
    float t0, t1, t2, t3;
    float ca, sa, cb, sb;
    // trajectory rows of the tracking mode (kernels with trajectories only)
    float xd0, xd1, xd2, vd0, vd1, vd2, ad0, ad1, ad2, cpd, spd;
    float wd0, wd1, wd2, dwd0, dwd1, dwd2;
};

struct Wrench {
    float f, M0, M1, M2;       // commanded
    float fa, Ma0, Ma1, Ma2;   // applied after clamping
};

template <bool VP>
AG_DEV void load_params(Params& P, const float* __restrict__ gt, const float* __restrict__ vp,
                        int64_t ld, int64_t i) {
    P.umin = gt[G_UMIN];
    P.nr = (int)gt[G_NR];
    if constexpr (VP) {
        P.m = vp[VP_MASS * ld + i];
        P.J0 = vp[(VP_J + 0) * ld + i];
        P.J1 = vp[(VP_J + 1) * ld + i];
        P.J2 = vp[(VP_J + 2) * ld + i];
        P.kx_xy = vp[(VP_GAINS + 0) * ld + i];
        P.kx_z = vp[(VP_GAINS + 1) * ld + i];
        P.kv_xy = vp[(VP_GAINS + 2) * ld + i];
        P.kv_z = vp[(VP_GAINS + 3) * ld + i];
        P.kR0 = vp[(VP_GAINS + 4) * ld + i];
        P.kR1 = vp[(VP_GAINS + 5) * ld + i];
        P.kR2 = vp[(VP_GAINS + 6) * ld + i];
        P.kW0 = vp[(VP_GAINS + 7) * ld + i];
        P.kW1 = vp[(VP_GAINS + 8) * ld + i];
        P.kW2 = vp[(VP_GAINS + 9) * ld + i];
        P.arm = vp[VP_ARM * ld + i];
        P.umax = vp[VP_UMAX * ld + i];
        P.inv_m = 1.0f / P.m;
        P.Ji0 = 1.0f / P.J0;
        P.Ji1 = 1.0f / P.J1;
        P.Ji2 = 1.0f / P.J2;
        P.inv_arm = 1.0f / P.arm;
    } else {
        P.m = gt[G_MASS];
        P.inv_m = gt[G_INV_MASS];
        P.J0 = gt[G_J + 0];
        P.J1 = gt[G_J + 1];
        P.J2 = gt[G_J + 2];
        P.Ji0 = gt[G_JINV + 0];
        P.Ji1 = gt[G_JINV + 1];
        P.Ji2 = gt[G_JINV + 2];
        P.kx_xy = gt[G_GAINS + 0];
        P.kx_z = gt[G_GAINS + 1];
        P.kv_xy = gt[G_GAINS + 2];
        P.kv_z = gt[G_GAINS + 3];
        P.kR0 = gt[G_GAINS + 4];
        P.kR1 = gt[G_GAINS + 5];
        P.kR2 = gt[G_GAINS + 6];
        P.kW0 = gt[G_GAINS + 7];
        P.kW1 = gt[G_GAINS + 8];
        P.kW2 = gt[G_GAINS + 9];
        P.arm = gt[G_ARM];
        P.inv_arm = gt[G_INV_ARM];
        P.umax = gt[G_UMAX];
    }
    P.dJ0 = P.J2 - P.J1;
    P.dJ1 = P.J0 - P.J2;
    P.dJ2 = P.J1 - P.J0;
    P.cq_f = gt[G_Q_F];
    P.cq_x = gt[G_Q_XY] * P.inv_arm;
    P.cq_z = gt[G_Q_Z];
    P.armq = P.arm * gt[G_Q_S];
    P.ctq = gt[G_Q_CT];
}

// Reciprocal square root as the single hardware instruction (1 ulp); every
// argument here is a sum of squares that is of order one to a few hundred or
// carries a normal bias (kTiny2), never a denormal, so the denormal-range
// rescaling of rsqrtf is not needed.
AG_DEV float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Bias of the angle extractions (2^-60 and its square, both normal FP32).
constexpr float kTiny = 0x1p-60f, kTiny2 = 0x1p-120f;

// Rotor-count class of a kernel: 4, 6 or 8 when every group of the launch
// has that many rotors, 0 for a mix (8 slots, inactive slots masked).
template <int NRC>
struct RotorClass {
    static constexpr int NR = NRC == 0 ? 8 : NRC;
    static constexpr bool MIXED = NRC == 0;
};

// sin and cos of an angle in radians.  For |x| < 4096 (every command angle in
// practice): Cody-Waite reduction by pi/2 with pi/2 split into three FP32
// parts (fl(pi/2), then fl of each remainder), applied by fused multiply-adds
// (for |k| <= 2^12 the reduced argument carries an absolute error of a few
// 1e-8 at most), then the Taylor polynomials of sin (to r^9) and cos (to
// r^10) on [-pi/4, pi/4], whose truncation error is below 2e-9, and the
// quadrant of k.  Larger or non-finite arguments take sincosf, in a branch of
// their own lanes: a lane's result never depends on the other lanes.  This
// replaces two full sincosf per vehicle and launch, whose large-argument
// reduction (64-bit integer multiplies) is evaluated for every lane.
AG_DEV void sincos_rad(float x, float& s, float& c) {
    constexpr float kPio2a = 0x1.921fb6p+0f, kPio2b = -0x1.777a5cp-25f, kPio2c = -0x1.ee59dap-50f;
    constexpr float k2Opi = 0x1.45f306p-1f;
    const float k = __builtin_rintf(x * k2Opi);
    float r = __builtin_fmaf(-k, kPio2a, x);
    r = __builtin_fmaf(-k, kPio2b, r);
    r = __builtin_fmaf(-k, kPio2c, r);
    const float r2 = r * r;
    // 1/9!, 1/7!, 1/5!, 1/3! and 1/10!, ..., 1/2! rounded to FP32
    float ps = __builtin_fmaf(0x1.71de3ap-19f, r2, -0x1.a01a02p-13f);
    ps = __builtin_fmaf(ps, r2, 0x1.111112p-7f);
    ps = __builtin_fmaf(ps, r2, -0x1.555556p-3f);
    ps = ps * r2;
    float pc = __builtin_fmaf(-0x1.27e4fcp-22f, r2, 0x1.a01a02p-16f);
    pc = __builtin_fmaf(pc, r2, -0x1.6c16c2p-10f);
    pc = __builtin_fmaf(pc, r2, 0x1.555556p-5f);
    pc = __builtin_fmaf(pc, r2, -0.5f);
    // (sin of a signed zero keeps its sign)
    const float sr = x == 0.0f ? x : __builtin_fmaf(r, ps, r);
    const float cr = __builtin_fmaf(pc, r2, 1.0f);
    // quadrant q = k mod 4: (sin, cos) = (s_r, c_r), (c_r, -s_r), (-s_r, -c_r), (-c_r, s_r);
    // k is an integer of magnitude below 2^22 on this path, so k + 1.5 * 2^23
    // holds k mod 2^23 in its low mantissa bits (no float-to-int conversion,
    // which a non-finite k of the other path would make undefined)
    const int q = __float_as_int(k + 0x1.8p23f) & 3;
    const bool odd = (q & 1) != 0;
    const uint32_t sneg = (uint32_t)(q & 2) << 30, cneg = (uint32_t)((q + 1) & 2) << 30;
    s = __uint_as_float(__float_as_uint(odd ? cr : sr) ^ sneg);
    c = __uint_as_float(__float_as_uint(odd ? sr : cr) ^ cneg);
    if (!(__builtin_fabsf(x) < 4096.0f)) sincosf(x, &s, &c);
}

AG_DEV void derive_cmd(Cmd& C, int mode, float t0, float t1, float t2, float t3) {
    C.mode = mode;
    C.t0 = t0; C.t1 = t1; C.t2 = t2; C.t3 = t3;
    // position mode: angle a = psi_d; attitude mode: a = phi_d, b = theta_d.
    const float a = (mode == 0) ? t3 : ((mode == 2) ? t0 : 0.0f);
    const float b = (mode == 2) ? t1 : 0.0f;
    // (sincos_rad gives exactly (x, 1) at x = +-0, so wavefronts whose angles
    // are all zero skip it with the same results)
    C.sa = a; C.ca = 1.0f;
    C.sb = b; C.cb = 1.0f;
    if (__any(a != 0.0f)) sincos_rad(a, C.sa, C.ca);
    if (__any(b != 0.0f)) sincos_rad(b, C.sb, C.cb);
}

// Position-mode command to goal (gx, gy, gz) with psi_d = 0: the same fields
// as derive_cmd(C, 0, gx, gy, gz, 0) (sin 0 = 0 and cos 0 = 1 exactly).
AG_DEV void set_position_goal(Cmd& C, float gx, float gy, float gz) {
    C.mode = 0;
    C.t0 = gx; C.t1 = gy; C.t2 = gz; C.t3 = 0.0f;
    C.sa = 0.0f; C.ca = 1.0f; C.sb = 0.0f; C.cb = 1.0f;
}

// Trajectory rows of vehicle i (x_d, v_d, a_d, psi_d, Omega_d, dOmega_d).
AG_DEV void derive_traj(Cmd& C, const float* __restrict__ tr, int64_t ld, int64_t i) {
    C.xd0 = tr[i]; C.xd1 = tr[ld + i]; C.xd2 = tr[2 * ld + i];
    C.vd0 = tr[3 * ld + i]; C.vd1 = tr[4 * ld + i]; C.vd2 = tr[5 * ld + i];
    C.ad0 = tr[6 * ld + i]; C.ad1 = tr[7 * ld + i]; C.ad2 = tr[8 * ld + i];
    sincos_rad(tr[9 * ld + i], C.spd, C.cpd);
    C.wd0 = tr[10 * ld + i]; C.wd1 = tr[11 * ld + i]; C.wd2 = tr[12 * ld + i];
    C.dwd0 = tr[13 * ld + i]; C.dwd1 = tr[14 * ld + i]; C.dwd2 = tr[15 * ld + i];
}

// Reverse-mode state of one vehicle for the tracking loss
// sum_t |x_t - goal|^2 + w_omega |Omega_t|^2 over post-step states.
struct Adj {
    float lam[13];     // in: adjoint of the post-step state; out: of the pre-step state
    float gb[10];      // accumulated adjoint of the ten gains
    float gx, gy, gz;  // goal
    float w_omega;
};

// One step of one vehicle.  s: x0..2, v3..5, q6..9 (w,x,y,z), W10..12.
// gt points at the vehicle's group entry (LDS).  Returns the number of
// rotors whose raw command fell outside [u_min, u_max]; fills W (commanded
// and applied wrench) and u (clamped thrusts, zero-padded) when requested.
// With GRAD the same forward computation is followed by its hand-written
// reverse: the loss gradient at the post-step state is added to adj->lam,
// which is then pulled back through integration, allocation (clamp
// subgradient 1 inside [u_min, u_max], bounds included), the moment law,
// the tilt extraction, the yaw readout and R(q).
template <int NRC, bool WANT_W, bool WANT_U, bool GRAD, bool TRK = false, int MS = -1>
AG_DEV int step_core(float (&s)[13], const Cmd& C, const Params& P, const float* __restrict__ gt,
                     float dt, float g, Wrench* W, float* u_out, Adj* adj) {
    constexpr int NR = RotorClass<NRC>::NR;
    constexpr bool MIXED = RotorClass<NRC>::MIXED;
    const float qw = s[6], qx = s[7], qy = s[8], qz = s[9];
    // ---- R(q), unit-norm form, from the doubled components ----------------
    const float x2 = qx + qx, y2 = qy + qy, z2 = qz + qz;
    const float wz2 = qw * z2, wy2 = qw * y2, wx2 = qw * x2;
    const float omzz = 1.0f - qz * z2;
    const float R00 = omzz - qy * y2, R11 = omzz - qx * x2, R22 = (1.0f - qy * y2) - qx * x2;
    const float R01 = qx * y2 - wz2, R10 = qx * y2 + wz2;
    const float R02 = qx * z2 + wy2, R20 = qx * z2 - wy2;
    const float R12 = qy * z2 - wx2, R21 = qy * z2 + wx2;

    // ---- current yaw (Z-Y-X), trig-free -----------------------------------
    // Here and in the tilt below, cos and sin of the angle of a 2-vector
    // (c, s) come as ((c + 2^-60), s) / sqrt(c^2 + s^2 + 2^-120): for a zero
    // vector this gives the convention angle = 0 (cos 1, sin 0) without a
    // select, and otherwise it moves cos by at most 2^-60 / |(c, s)|.
    const float r2 = R00 * R00 + (R10 * R10 + kTiny2);
    const float ir = rsq(r2);
    const float cpsi = (R00 + kTiny) * ir;
    const float spsi = R10 * ir;

    // MS >= 0: every vehicle of the call has mode MS (the selects below fold
    // to one side; the arithmetic of the remaining side is unchanged).  Every
    // mode select is a statement of its own, never an operand inside a longer
    // expression: multiply-adds are contracted per expression from the form
    // of its operands, so a select that folds to a product would otherwise
    // contract differently in a specialised copy.
    const int mode = MS >= 0 ? MS : C.mode;
    const bool m0 = mode == 0, m1 = mode == 1, m2 = mode == 2, m3 = mode == 3;

    // ---- reference yaw frame: psi_d (position) or current psi -------------
    const float cr = m0 ? C.ca : cpsi;
    const float sr = m0 ? C.sa : spsi;

    // ---- commanded force in the reference frame (position / velocity) -----
    // F_V = m (kx e_V + kv (v_d - v_V) + g e3), e_V and v_V the position error
    // and the velocity rotated by R_z(psi_ref)^T; the x-y gains are equal, so
    // the rotation is applied after them:
    //   F_V,xy = R_z(psi_ref)^T (m kx' (x_d - x) - m kv v)_xy + m kv v_d,xy',
    //   F_V,z  = m kx' (z_d - z) - m kv v_z + m kv v_d,z' + m g,
    // with kx' = kx in position mode and 0 otherwise, v_d' = v_d in velocity
    // mode and 0 otherwise.  Products of per-vehicle constants are loop-
    // invariant in a fused launch.  (A non-finite position outside position
    // mode therefore makes F non-finite, where the plain formula ignores it.)
    const float vx = s[3], vy = s[4], vz = s[5];
    const float kxm_xy = m0 ? P.m * P.kx_xy : 0.0f, kxm_z = m0 ? P.m * P.kx_z : 0.0f;
    const float kvm_xy = P.m * P.kv_xy, kvm_z = P.m * P.kv_z;
    const float Kx = kxm_xy * C.t0, Ky = kxm_xy * C.t1;
    const float Vx = m1 ? kvm_xy * C.t0 : 0.0f, Vy = m1 ? kvm_xy * C.t1 : 0.0f;
    const float Vz = m1 ? kvm_z * C.t2 : 0.0f;
    const float Kz = kxm_z * C.t2 + (Vz + P.m * g);
    // the position terms are selects of their own (zero outside position
    // mode), so a velocity-mode copy of the step drops them
    const float Qx = m0 ? Kx - kxm_xy * s[0] : 0.0f;
    const float Qy = m0 ? Ky - kxm_xy * s[1] : 0.0f;
    const float Ax = Qx - kvm_xy * vx;
    const float Ay = Qy - kvm_xy * vy;
    const float Fx = cr * Ax + (sr * Ay + Vx);
    const float Fy = cr * Ay + (Vy - sr * Ax);
    const float Qz = m0 ? Kz - kxm_z * s[2] : Kz;
    const float Fz = Qz - kvm_z * vz;
    // the same quantities in the plain decomposition (reverse pass only)
    const float vVx = cr * vx + sr * vy;
    const float vVy = cr * vy - sr * vx;
    const float dxE = C.t0 - s[0], dyE = C.t1 - s[1], dzE = C.t2 - s[2];
    const float ex = m0 ? (cr * dxE + sr * dyE) : 0.0f;
    const float ey = m0 ? (cr * dyE - sr * dxE) : 0.0f;
    const float ez = m0 ? dzE : 0.0f;
    const float wvx = (m1 ? C.t0 : 0.0f) - vVx;
    const float wvy = (m1 ? C.t1 : 0.0f) - vVy;
    const float wvz = (m1 ? C.t2 : 0.0f) - vz;

    // ---- tilt from force, eqs. (8)-(9) without trig -----------------------
    // theta_d from (F_z, F_x), then phi_d from (h, -F_y), h = |(F_x, F_z)|;
    // h is itself biased by 2^-60 at most, so F = 0 gives theta_d = phi_d = 0
    const float h2 = Fx * Fx + (Fz * Fz + kTiny2);
    const float n2 = h2 + Fy * Fy;
    const float ih = rsq(h2), inn = rsq(n2);
    const float hh = h2 * ih;
    float cth = (Fz + kTiny) * ih;
    float sth = Fx * ih;
    float cph = hh * inn;
    float sph = -Fy * inn;
    cth = m2 ? C.cb : cth;
    sth = m2 ? C.sb : sth;
    cph = m2 ? C.ca : cph;
    sph = m2 ? C.sa : sph;

    // ---- P = R_z(psi_ref)^T R ---------------------------------------------
    const float P00 = cr * R00 + sr * R10, P01 = cr * R01 + sr * R11, P02 = cr * R02 + sr * R12;
    const float P10 = cr * R10 - sr * R00, P11 = cr * R11 - sr * R01, P12 = cr * R12 - sr * R02;
    const float P20 = R20, P21 = R21, P22 = R22;

    // ---- thrust: projection of F on b3 (modes 0, 1); command otherwise -----
    const float fproj = Fx * P02 + Fy * P12 + Fz * P22;
    float f = (m0 || m1) ? fproj : (m2 ? C.t3 : (m3 ? C.t0 : 0.0f));

    // ---- e_R = 1/2 vee(E - E^T), E = T^T P, T = R_y(theta) R_x(phi) --------
    const float T01 = sth * sph, T02 = sth * cph;
    const float T21 = cth * sph, T22 = cth * cph;
    // twice e_R, each difference of E entries as one multiply-add chain; the
    // 1/2 is folded into the gains of eq. (5) (exact scaling)
    float dR0 = T02 * P01 - sph * P11 + T22 * P21 - T01 * P02 - cph * P12 - T21 * P22;   // E21 - E12
    float dR1 = cth * P02 - sth * P22 - T02 * P00 + sph * P10 - T22 * P20;               // E02 - E20
    float dR2 = T01 * P00 + cph * P10 + T21 * P20 - cth * P01 + sth * P21;               // E10 - E01

    // ---- e_Omega = Omega - psidot_d R^T e3 ---------------------------------
    const float psidot = m1 ? C.t3 : (m2 ? C.t2 : 0.0f);
    const float w0 = s[10], w1 = s[11], w2 = s[12];
    // (psidot_d = 0 in position mode: e_Omega = Omega)
    float eW0 = m0 ? w0 : w0 - psidot * R20;
    float eW1 = m0 ? w1 : w1 - psidot * R21;
    float eW2 = m0 ? w2 : w2 - psidot * R22;

    // ---- gyroscopic term Omega x J Omega ------------------------------------
    // for diagonal J its components are (J2 - J1) w1 w2, (J0 - J2) w2 w0 and
    // (J1 - J0) w0 w1 (exactly zero about a symmetry axis)
    const float w12 = w1 * w2, w20 = w2 * w0, w01 = w0 * w1;

    // ---- mode 4: full geometric tracking law (kernels with trajectories) ----
    float ff0 = 0.0f, ff1 = 0.0f, ff2 = 0.0f;
    bool m4 = false;
    if constexpr (TRK) {
        m4 = mode == 4;
        // F = m (-kx e_x - kv e_v + a_d + g e3) in the inertial frame
        const float F4x = P.m * (-P.kx_xy * (s[0] - C.xd0) - P.kv_xy * (vx - C.vd0) + C.ad0);
        const float F4y = P.m * (-P.kx_xy * (s[1] - C.xd1) - P.kv_xy * (vy - C.vd1) + C.ad1);
        const float F4z = P.m * (-P.kx_z * (s[2] - C.xd2) - P.kv_z * (vz - C.vd2) + C.ad2 + g);
        const float f4 = F4x * R02 + F4y * R12 + F4z * R22;
        // desired frame: b3 = F/|F|, b2 = b3 x b1d / |.|, b1 = b2 x b3
        const float n4 = rsq(F4x * F4x + F4y * F4y + F4z * F4z);
        const float b3x = F4x * n4, b3y = F4y * n4, b3z = F4z * n4;
        float cx = -b3z * C.spd, cy = b3z * C.cpd, cz = b3x * C.spd - b3y * C.cpd;
        float nc2 = cx * cx + cy * cy + cz * cz;
        if (!(nc2 > 0.0f)) {          // heading parallel to b3: use e1, then e2
            cx = 0.0f; cy = b3z; cz = -b3y;
            nc2 = cy * cy + cz * cz;
            if (!(nc2 > 0.0f)) { cx = -b3z; cy = 0.0f; cz = b3x; nc2 = cx * cx + cz * cz; }
        }
        const float ic = rsq(nc2);
        const float b2x = cx * ic, b2y = cy * ic, b2z = cz * ic;
        const float b1x = b2y * b3z - b2z * b3y, b1y = b2z * b3x - b2x * b3z, b1z = b2x * b3y - b2y * b3x;
        // E = R_d^T R: E_ij = b_i . (column j of R)
        const float G21 = b3x * R01 + b3y * R11 + b3z * R21, G12 = b2x * R02 + b2y * R12 + b2z * R22;
        const float G02 = b1x * R02 + b1y * R12 + b1z * R22, G20 = b3x * R00 + b3y * R10 + b3z * R20;
        const float G10 = b2x * R00 + b2y * R10 + b2z * R20, G01 = b1x * R01 + b1y * R11 + b1z * R21;
        // R^T R_d Omega_d and R^T R_d dOmega_d
        const float ax = b1x * C.wd0 + b2x * C.wd1 + b3x * C.wd2;
        const float ay = b1y * C.wd0 + b2y * C.wd1 + b3y * C.wd2;
        const float az = b1z * C.wd0 + b2z * C.wd1 + b3z * C.wd2;
        const float c0 = R00 * ax + R10 * ay + R20 * az;
        const float c1 = R01 * ax + R11 * ay + R21 * az;
        const float c2 = R02 * ax + R12 * ay + R22 * az;
        const float dx = b1x * C.dwd0 + b2x * C.dwd1 + b3x * C.dwd2;
        const float dy = b1y * C.dwd0 + b2y * C.dwd1 + b3y * C.dwd2;
        const float dz = b1z * C.dwd0 + b2z * C.dwd1 + b3z * C.dwd2;
        const float d0 = R00 * dx + R10 * dy + R20 * dz;
        const float d1 = R01 * dx + R11 * dy + R21 * dz;
        const float d2 = R02 * dx + R12 * dy + R22 * dz;
        f = m4 ? f4 : f;
        dR0 = m4 ? G21 - G12 : dR0;
        dR1 = m4 ? G02 - G20 : dR1;
        dR2 = m4 ? G10 - G01 : dR2;
        eW0 = m4 ? w0 - c0 : eW0;
        eW1 = m4 ? w1 - c1 : eW1;
        eW2 = m4 ? w2 - c2 : eW2;
        // feed-forward J (Omega x R^T R_d Omega_d - R^T R_d dOmega_d)
        ff0 = m4 ? P.J0 * ((w1 * c2 - w2 * c1) - d0) : 0.0f;
        ff1 = m4 ? P.J1 * ((w2 * c0 - w0 * c2) - d1) : 0.0f;
        ff2 = m4 ? P.J2 * ((w0 * c1 - w1 * c0) - d2) : 0.0f;
    }

    // ---- M = -kR e_R - kW e_Omega + Omega x J Omega, eq. (5) ---------------
    // The allocation takes M scaled per axis, (cq_x M_x, cq_x M_y, cq_z M_z)
    // for the quad butterflies and (M_x / l, M_y / l, M_z) for the table, so
    // the law is evaluated directly in those units with pre-scaled constants
    // (loop-invariant products); the rate update below takes the scaled
    // gyroscopic term with dt J^-1 divided by the same scales.
    const bool quad = NRC == 4 || (MIXED && P.nr == 4);
    const float s01 = quad ? P.cq_x : P.inv_arm;
    const float s2 = quad ? P.cq_z : 1.0f;
    const float hkR0 = 0.5f * P.kR0, hkR1 = 0.5f * P.kR1, hkR2 = 0.5f * P.kR2;
    const float gs0 = (s01 * P.dJ0) * w12, gs1 = (s01 * P.dJ1) * w20, gs2 = (s2 * P.dJ2) * w01;
    float Ms0 = gs0 - (s01 * hkR0) * dR0 - (s01 * P.kW0) * eW0;
    float Ms1 = gs1 - (s01 * hkR1) * dR1 - (s01 * P.kW1) * eW1;
    float Ms2 = gs2 - (s2 * hkR2) * dR2 - (s2 * P.kW2) * eW2;
    if constexpr (TRK) {
        Ms0 -= s01 * ff0;
        Ms1 -= s01 * ff1;
        Ms2 -= s2 * ff2;
    }
    // mode 3 takes the commanded moment, an unknown mode a zero wrench (one
    // select per component against per-vehicle constants)
    const bool direct = m3 || !(m0 || m1 || m2 || m4);
    Ms0 = direct ? s01 * (m3 ? C.t1 : 0.0f) : Ms0;
    Ms1 = direct ? s01 * (m3 ? C.t2 : 0.0f) : Ms1;
    Ms2 = direct ? s2 * (m3 ? C.t3 : 0.0f) : Ms2;

    // ---- allocation and clamping ------------------------------------------
    // applied wrench (fa, k01 X0, k01 X1, k2 X2)
    float fa, X0, X1, X2, k01, k2;
    int nsat = 0;
    float raws[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        raws[r] = 0.0f;
        if constexpr (WANT_U) u_out[r] = 0.0f;
    }
    // clamp to [u_min, u_max] as one median-of-three
    auto clamp_rotor = [&](int r, float raw) -> float {
        raws[r] = raw;
        const float u = __builtin_amdgcn_fmed3f(raw, P.umin, P.umax);
        nsat += (int)((raw < P.umin) | (raw > P.umax));
        if constexpr (WANT_U) u_out[r] = u;
        return u;
    };
    // Quad X (rotors at 45, 135, 225, 315 degrees, spins + - + -): rotor i's
    // raw thrust is cq_f f + sx_i cq_x M_x + sy_i cq_x M_y + sz_i cq_z M_z with
    // sx = (+ + - -), sy = (- + + -), sz = (+ - + -), and the applied wrench
    // sums the thrusts with the same signs, so both products are 4-point
    // butterflies (8 additions each instead of 16 multiply-adds).
    auto quad_alloc = [&]() {
        const float a = P.cq_f * f + Ms2, b = P.cq_f * f - Ms2;
        const float c = Ms0 - Ms1, d = Ms0 + Ms1;
        const float u0 = clamp_rotor(0, a + c), u1 = clamp_rotor(1, b + d);
        const float u2 = clamp_rotor(2, a - c), u3 = clamp_rotor(3, b - d);
        const float e = u0 + u2, o = u1 + u3, ge = u0 - u2, ho = u1 - u3;
        fa = e + o;
        X0 = ge + ho;
        X1 = ho - ge;
        X2 = e - o;
        k01 = P.armq;
        k2 = P.ctq;
    };
    // Hexa and octo: rotor i + n/2 sits opposite rotor i (angle + pi), so its
    // row of A1^+ (and of A1) has the x-y terms negated and the yaw term
    // times (-1)^(n/2).  With L_i the x-y part of rotor i's row, rotor i
    // takes c_f f + s_i Z + L_i and rotor i + n/2 takes c_f f + s_(i+n/2) Z
    // - L_i; the applied sums run over the pair differences and sums, the
    // yaw sum without c_tau (applied as k2).
    auto pair_alloc = [&](auto n_tag) {
        constexpr int N = decltype(n_tag)::value, H = N / 2;
        const float4 p0 = *reinterpret_cast<const float4*>(gt + G_APINV);
        const float4 c0 = *reinterpret_cast<const float4*>(gt + G_ACOL);
        const float cf = p0.x * f, zs = p0.w * Ms2;
        const float cp = cf + zs, cm = cf - zs;      // spin + and spin - rotors
        float yaw = 0.0f;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const float4 ap = *reinterpret_cast<const float4*>(gt + G_APINV + 4 * i);
            const float4 ac = *reinterpret_cast<const float4*>(gt + G_ACOL + 4 * i);
            const float L = ap.y * Ms0 + ap.z * Ms1;
            const bool sp = (i & 1) == 0;                       // spin of rotor i
            const bool so = (H & 1) ? !sp : sp;                 // spin of rotor i + H
            const float ui = clamp_rotor(i, (sp ? cp : cm) + L);
            const float uo = clamp_rotor(i + H, (so ? cp : cm) - L);
            const float d = ui - uo, sm = ui + uo;
            const float ys = (H & 1) ? d : sm;                  // yaw: s_i (u_i -+ u_o)
            if (i == 0) {
                fa = sm;
                X0 = ac.y * d;
                X1 = ac.z * d;
                yaw = ys;
            } else {
                fa += sm;
                X0 += ac.y * d;
                X1 += ac.z * d;
                yaw = sp ? yaw + ys : yaw - ys;
            }
        }
        X2 = yaw;
        k01 = P.arm;
        k2 = c0.w;
    };
    // every kernel that meets a quad takes the butterflies, and hexa and
    // octo the pairs, so a group rounds identically in a launch of its own
    // layout and in a mixed launch
    if constexpr (NRC == 4) {
        quad_alloc();
    } else if constexpr (NRC == 6) {
        pair_alloc(std::integral_constant<int, 6>{});
    } else if constexpr (NRC == 8) {
        pair_alloc(std::integral_constant<int, 8>{});
    } else {
        if (P.nr == 4) quad_alloc();
        else if (P.nr == 6) pair_alloc(std::integral_constant<int, 6>{});
        else pair_alloc(std::integral_constant<int, 8>{});
    }
    if constexpr (WANT_W) {
        // the commanded moment in N m (the same law, unscaled)
        float M0 = P.dJ0 * w12 - hkR0 * dR0 - P.kW0 * eW0;
        float M1 = P.dJ1 * w20 - hkR1 * dR1 - P.kW1 * eW1;
        float M2 = P.dJ2 * w01 - hkR2 * dR2 - P.kW2 * eW2;
        if constexpr (TRK) {
            M0 -= ff0;
            M1 -= ff1;
            M2 -= ff2;
        }
        W->f = f;
        W->M0 = direct ? (m3 ? C.t1 : 0.0f) : M0;
        W->M1 = direct ? (m3 ? C.t2 : 0.0f) : M1;
        W->M2 = direct ? (m3 ? C.t3 : 0.0f) : M2;
        W->fa = fa; W->Ma0 = k01 * X0; W->Ma1 = k01 * X1; W->Ma2 = k2 * X2;
    }

    // ---- semi-implicit Euler ----------------------------------------------
    // dt is folded into 1/m and J^-1 (loop-invariant products in a fused launch)
    const float dt_m = dt * P.inv_m, dtg = dt * g;
    // (k01 X0 - gy0) dt/J0 = (k01 s01 X0 - gs0) (dt/J0) / s01, likewise for
    // axes 1 and 2; loop-invariant constants
    const float Ds0 = (dt * P.Ji0) / s01, Ds1 = (dt * P.Ji1) / s01, Ds2 = (dt * P.Ji2) / s2;
    const float Ks01 = k01 * s01, Ks2 = k2 * s2;
    const float dva = fa * dt_m;
    const float nvx = dva * R02 + vx;
    const float nvy = dva * R12 + vy;
    const float nvz = dva * R22 + (vz - dtg);
    s[0] = s[0] + dt * nvx;
    s[1] = s[1] + dt * nvy;
    s[2] = s[2] + dt * nvz;
    s[3] = nvx; s[4] = nvy; s[5] = nvz;
    const float nw0 = (Ks01 * X0 - gs0) * Ds0 + w0;
    const float nw1 = (Ks01 * X1 - gs1) * Ds1 + w1;
    const float nw2 = (Ks2 * X2 - gs2) * Ds2 + w2;
    s[10] = nw0; s[11] = nw1; s[12] = nw2;
    // q <- normalize(q + dt/2 q (x) (0, Omega+))
    // with h = (dt/2) Omega+ first: t = q + q (x) (0, h), one chain per component
    const float hd = 0.5f * dt;
    const float h0 = hd * nw0, h1 = hd * nw1, h2q = hd * nw2;
    const float tw = qw - qx * h0 - qy * h1 - qz * h2q;
    const float tx = qx + qw * h0 + qy * h2q - qz * h1;
    const float ty = qy + qw * h1 + qz * h0 - qx * h2q;
    const float tz = qz + qw * h2q + qx * h1 - qy * h0;
    const float iq = rsq(tw * tw + tx * tx + ty * ty + tz * tz);
    s[6] = tw * iq; s[7] = tx * iq; s[8] = ty * iq; s[9] = tz * iq;

    if constexpr (GRAD) {
        float* L = adj->lam;
        float* gb = adj->gb;
        // loss at the post-step state
        L[0] += 2.0f * (s[0] - adj->gx);
        L[1] += 2.0f * (s[1] - adj->gy);
        L[2] += 2.0f * (s[2] - adj->gz);
        L[10] += 2.0f * adj->w_omega * nw0;
        L[11] += 2.0f * adj->w_omega * nw1;
        L[12] += 2.0f * adj->w_omega * nw2;

        // ---- quaternion update: q+ = (q + hd q (x) (0, w+)) / |.| ----------
        const float nq0 = s[6], nq1 = s[7], nq2 = s[8], nq3 = s[9];
        const float dot = nq0 * L[6] + nq1 * L[7] + nq2 * L[8] + nq3 * L[9];
        const float bt0 = iq * (L[6] - nq0 * dot), bt1 = iq * (L[7] - nq1 * dot);
        const float bt2 = iq * (L[8] - nq2 * dot), bt3 = iq * (L[9] - nq3 * dot);
        const float bdw = hd * bt0, bdx = hd * bt1, bdy = hd * bt2, bdz = hd * bt3;
        float bqw = bt0 + bdx * nw0 + bdy * nw1 + bdz * nw2;
        float bqx = bt1 - bdw * nw0 - bdy * nw2 + bdz * nw1;
        float bqy = bt2 - bdw * nw1 + bdx * nw2 - bdz * nw0;
        float bqz = bt3 - bdw * nw2 - bdx * nw1 + bdy * nw0;
        const float bnw0 = L[10] - bdw * qx + bdx * qw + bdy * qz - bdz * qy;
        const float bnw1 = L[11] - bdw * qy - bdx * qz + bdy * qw + bdz * qx;
        const float bnw2 = L[12] - bdw * qz + bdx * qy - bdy * qx + bdz * qw;

        // ---- rate update: w+ = w + dt J^-1 (M' - w x J w) -----------------
        float bw0 = bnw0, bw1 = bnw1, bw2 = bnw2;
        const float bMa0 = dt * (P.Ji0 * bnw0), bMa1 = dt * (P.Ji1 * bnw1), bMa2 = dt * (P.Ji2 * bnw2);
        float bgy0 = -bMa0, bgy1 = -bMa1, bgy2 = -bMa2;

        // ---- translation: x+ = x + dt v+, v+ = v + dt (acc b3 - g e3) ------
        const float bnv0 = L[3] + dt * L[0], bnv1 = L[4] + dt * L[1], bnv2 = L[5] + dt * L[2];
        float bx0 = L[0], bx1 = L[1], bx2 = L[2];
        float bv0 = bnv0, bv1 = bnv1, bv2 = bnv2;
        const float bacc = dt * (bnv0 * R02 + bnv1 * R12 + bnv2 * R22);
        float bR00 = 0.0f, bR01 = 0.0f, bR10 = 0.0f, bR11 = 0.0f, bR20 = 0.0f, bR21 = 0.0f;
        const float acc = fa * P.inv_m;
        float bR02 = dt * (acc * bnv0), bR12 = dt * (acc * bnv1), bR22 = dt * (acc * bnv2);
        const float bfa = bacc * P.inv_m;

        // ---- allocation and clamp ----------------------------------------
        // adjoint of the applied wrench's sums X, then of the raw thrusts
        // (clamp subgradient), then of (f, M): the transposes of the forward
        // products, as butterflies for the quad
        // (the table products below take the yaw sum with c_tau inside)
        const float bX0 = k01 * bMa0, bX1 = k01 * bMa1, bX2 = quad ? k2 * bMa2 : bMa2;
        float bf, bM0, bM1, bM2;
        auto pass = [&](int r) { return (raws[r] >= P.umin) & (raws[r] <= P.umax); };
        auto quad_rev = [&]() {
            const float be = bfa + bX2, bo = bfa - bX2;
            const float bge = bX0 - bX1, bho = bX0 + bX1;
            const float br0 = pass(0) ? be + bge : 0.0f, br2 = pass(2) ? be - bge : 0.0f;
            const float br1 = pass(1) ? bo + bho : 0.0f, br3 = pass(3) ? bo - bho : 0.0f;
            const float ba = br0 + br2, bc = br0 - br2, bb = br1 + br3, bd = br1 - br3;
            bf = P.cq_f * (ba + bb);
            bM2 = P.cq_z * (ba - bb);
            bM0 = P.cq_x * (bc + bd);
            bM1 = P.cq_x * (bd - bc);
        };
        auto table_rev = [&]() {
            float sf = 0.0f, ba1 = 0.0f, ba2 = 0.0f, sM2 = 0.0f;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const float4 ap = *reinterpret_cast<const float4*>(gt + G_APINV + 4 * r);
                const float4 ac = *reinterpret_cast<const float4*>(gt + G_ACOL + 4 * r);
                const float bu = bfa * ac.x + bX0 * ac.y + bX1 * ac.z + bX2 * ac.w;
                const float braw = ((MIXED ? r < P.nr : true) & pass(r)) ? bu : 0.0f;
                sf += braw * ap.x;
                ba1 += braw * ap.y;
                ba2 += braw * ap.z;
                sM2 += braw * ap.w;
            }
            bf = sf;
            bM0 = ba1 * P.inv_arm;
            bM1 = ba2 * P.inv_arm;
            bM2 = sM2;
        };
        if constexpr (NRC == 4) {
            quad_rev();
        } else if constexpr (MIXED) {
            if (P.nr == 4) quad_rev();
            else table_rev();
        } else {
            table_rev();
        }
        const bool ctl = m0 || m1 || m2;       // M depends on the state
        const bool frc = m0 || m1;             // f and the tilt depend on the state
        bM0 = ctl ? bM0 : 0.0f;
        bM1 = ctl ? bM1 : 0.0f;
        bM2 = ctl ? bM2 : 0.0f;
        bf = frc ? bf : 0.0f;

        // ---- moment law, eq. (5) -------------------------------------------
        const float eR0 = 0.5f * dR0, eR1 = 0.5f * dR1, eR2 = 0.5f * dR2;
        gb[4] -= bM0 * eR0; gb[5] -= bM1 * eR1; gb[6] -= bM2 * eR2;
        gb[7] -= bM0 * eW0; gb[8] -= bM1 * eW1; gb[9] -= bM2 * eW2;
        const float beR0 = -P.kR0 * bM0, beR1 = -P.kR1 * bM1, beR2 = -P.kR2 * bM2;
        const float beW0 = -P.kW0 * bM0, beW1 = -P.kW1 * bM1, beW2 = -P.kW2 * bM2;
        bgy0 += bM0; bgy1 += bM1; bgy2 += bM2;
        const float cg0 = P.dJ0 * bgy0, cg1 = P.dJ1 * bgy1, cg2 = P.dJ2 * bgy2;
        bw0 += cg1 * w2 + cg2 * w1 + beW0;
        bw1 += cg0 * w2 + cg2 * w0 + beW1;
        bw2 += cg0 * w1 + cg1 * w0 + beW2;
        bR20 -= psidot * beW0; bR21 -= psidot * beW1; bR22 -= psidot * beW2;

        // ---- attitude error, eq. (3) -------------------------------------
        const float bE21 = 0.5f * beR0, bE12 = -0.5f * beR0;
        const float bE02 = 0.5f * beR1, bE20 = -0.5f * beR1;
        const float bE10 = 0.5f * beR2, bE01 = -0.5f * beR2;
        float bP00 = 0.0f, bP01 = 0.0f, bP02 = 0.0f, bP10 = 0.0f, bP11 = 0.0f, bP12 = 0.0f;
        float bP20 = 0.0f, bP21 = 0.0f, bP22 = 0.0f;
        float bT01 = 0.0f, bT02 = 0.0f, bT21 = 0.0f, bT22 = 0.0f;
        float bcth = 0.0f, bsth = 0.0f, bcph = 0.0f, bsph = 0.0f;
        bT02 += bE21 * P01; bP01 += bE21 * T02; bsph -= bE21 * P11; bP11 -= bE21 * sph;
        bT22 += bE21 * P21; bP21 += bE21 * T22;
        bT01 += bE12 * P02; bP02 += bE12 * T01; bcph += bE12 * P12; bP12 += bE12 * cph;
        bT21 += bE12 * P22; bP22 += bE12 * T21;
        bcth += bE02 * P02; bP02 += bE02 * cth; bsth -= bE02 * P22; bP22 -= bE02 * sth;
        bT02 += bE20 * P00; bP00 += bE20 * T02; bsph -= bE20 * P10; bP10 -= bE20 * sph;
        bT22 += bE20 * P20; bP20 += bE20 * T22;
        bT01 += bE10 * P00; bP00 += bE10 * T01; bcph += bE10 * P10; bP10 += bE10 * cph;
        bT21 += bE10 * P20; bP20 += bE10 * T21;
        bcth += bE01 * P01; bP01 += bE01 * cth; bsth -= bE01 * P21; bP21 -= bE01 * sth;
        bsth += bT01 * sph + bT02 * cph;
        bsph += bT01 * sth + bT21 * cth;
        bcph += bT02 * sth + bT22 * cth;
        bcth += bT21 * sph + bT22 * cph;

        // ---- thrust projection ---------------------------------------------
        float bFx = bf * P02, bFy = bf * P12, bFz = bf * P22;
        bP02 += bf * Fx; bP12 += bf * Fy; bP22 += bf * Fz;

        // ---- P = R_z(psi_ref)^T R -------------------------------------------
        bR00 += cr * bP00 - sr * bP10; bR10 += sr * bP00 + cr * bP10; bR20 += bP20;
        bR01 += cr * bP01 - sr * bP11; bR11 += sr * bP01 + cr * bP11; bR21 += bP21;
        bR02 += cr * bP02 - sr * bP12; bR12 += sr * bP02 + cr * bP12; bR22 += bP22;
        float bcr = bP00 * R00 + bP10 * R10 + bP01 * R01 + bP11 * R11 + bP02 * R02 + bP12 * R12;
        float bsr = bP00 * R10 - bP10 * R00 + bP01 * R11 - bP11 * R01 + bP02 * R12 - bP12 * R02;

        // ---- tilt extraction, eqs. (8)-(9) ----------------------------------
        if (Fx * Fx + Fz * Fz > 0.0f) {     // zero (F_x, F_z): convention branch, no derivative
            const float ih3 = ih * ih * ih;
            const float D = (bcth * Fx - bsth * Fz) * ih3;
            bFx -= Fz * D;
            bFz += Fx * D;
            const float inn3 = inn * inn * inn;
            const float Gq = (bcph * (Fy * Fy) * ih + bsph * Fy) * inn3;
            bFx += Fx * Gq;
            bFz += Fz * Gq;
            bFy -= (bcph * hh * Fy + bsph * h2) * inn3;
        }
        bFx = frc ? bFx : 0.0f;
        bFy = frc ? bFy : 0.0f;
        bFz = frc ? bFz : 0.0f;

        // ---- commanded force: F = m a, a = kx e + kv (v_d - v_V) ------------
        const float bax = P.m * bFx, bay = P.m * bFy, baz = P.m * bFz;
        gb[0] += bax * ex + bay * ey;
        gb[1] += baz * ez;
        gb[2] += bax * wvx + bay * wvy;
        gb[3] += baz * wvz;
        const float bex = P.kx_xy * bax, bey = P.kx_xy * bay, bez = P.kx_z * baz;
        const float bvVx = -(P.kv_xy * bax), bvVy = -(P.kv_xy * bay);
        bv2 -= P.kv_z * baz;
        if (m0) {
            bx0 -= cr * bex - sr * bey;
            bx1 -= sr * bex + cr * bey;
            bx2 -= bez;
            bcr += bex * dxE + bey * dyE;
            bsr += bex * dyE - bey * dxE;
        }
        bv0 += cr * bvVx - sr * bvVy;
        bv1 += sr * bvVx + cr * bvVy;
        bcr += bvVx * vx + bvVy * vy;
        bsr += bvVx * vy - bvVy * vx;

        // ---- yaw readout (reference frame of velocity / attitude modes) -----
        if (!m0 && R00 * R00 + R10 * R10 > 0.0f) {
            const float D2 = (bcr * R10 - bsr * R00) * (ir * ir * ir);
            bR00 += R10 * D2;
            bR10 -= R00 * D2;
        }

        // ---- R(q) -----------------------------------------------------------
        const float bxx = -2.0f * (bR11 + bR22), byy = -2.0f * (bR00 + bR22), bzz = -2.0f * (bR00 + bR11);
        const float bxy = 2.0f * (bR01 + bR10), bxz = 2.0f * (bR02 + bR20), byz = 2.0f * (bR12 + bR21);
        const float bwx = 2.0f * (bR21 - bR12), bwy = 2.0f * (bR02 - bR20), bwz = 2.0f * (bR10 - bR01);
        bqx += 2.0f * qx * bxx + qy * bxy + qz * bxz + qw * bwx;
        bqy += 2.0f * qy * byy + qx * bxy + qz * byz + qw * bwy;
        bqz += 2.0f * qz * bzz + qx * bxz + qy * byz + qw * bwz;
        bqw += qx * bwx + qy * bwy + qz * bwz;

        L[0] = bx0; L[1] = bx1; L[2] = bx2;
        L[3] = bv0; L[4] = bv1; L[5] = bv2;
        L[6] = bqw; L[7] = bqx; L[8] = bqy; L[9] = bqz;
        L[10] = bw0; L[11] = bw1; L[12] = bw2;
    }
    return nsat;
}

template <int NRC, bool WANT_W, bool WANT_U, bool TRK = false, int MS = -1>
AG_DEV int step(float (&s)[13], const Cmd& C, const Params& P, const float* __restrict__ gt,
                float dt, float g, Wrench* W, float* u_out) {
    return step_core<NRC, WANT_W, WANT_U, false, TRK, MS>(s, C, P, gt, dt, g, W, u_out, nullptr);
}

// ---- Philox4x32-10 (Salmon et al., SC'11) ---------------------------------
constexpr uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;
constexpr uint32_t TAG_MASK = 0x4D41534Bu, TAG_DRAW = 0x44520000u;

// a ^ b ^ c in one instruction (gfx950's three-input bitwise operation;
// 0x96 is the truth table of the three-way exclusive or)
AG_DEV uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); }

AG_DEV uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)PHILOX_M0 * c.x;
        const uint64_t p1 = (uint64_t)PHILOX_M1 * c.z;
        c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1,
                       xor3((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0);
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    return c;
}

// Reset decision of global vehicle gi before global step t: word (t mod 4) of
// Philox(counter = (gi, lo(t/4), hi(t/4), TAG_MASK)) compared with thr.
// One Philox call serves four consecutive steps: mask_block gives the words of
// steps 4 tb .. 4 tb + 3, mask_hit picks the word of step t.
AG_DEV uint4 mask_block(uint32_t gi, uint64_t tb, uint32_t k0, uint32_t k1) {
    return philox(make_uint4(gi, (uint32_t)tb, (uint32_t)(tb >> 32), TAG_MASK), k0, k1);
}

AG_DEV bool mask_hit(uint4 w, int64_t t, uint64_t thr) {
    const int sel = (int)(t & 3);
    const uint32_t word = sel == 0 ? w.x : (sel == 1 ? w.y : (sel == 2 ? w.z : w.w));
    return (uint64_t)word < thr;
}

AG_DEV bool reset_mask(uint32_t gi, int64_t t, uint32_t k0, uint32_t k1, uint64_t thr) {
    return mask_hit(mask_block(gi, (uint64_t)t >> 2, k0, k1), t, thr);
}

AG_DEV float u24(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-8f; }   // 2^-24

// Redraw state s and goal (gx, gy, gz) for global vehicle gi at step t.
// Words 0-2 position, 3-5 goal, 6 tilt axis angle, 7 tilt, 8 yaw, Box-Muller
// pairs (9,10), (11,12), (13,14) -> 3 velocity and 3 body-rate normals.
AG_DEV void redraw(float (&s)[13], float& gx, float& gy, float& gz, uint32_t gi, int64_t t,
                   uint32_t k0, uint32_t k1, const float* lo, const float* hi) {
    const uint64_t tu = (uint64_t)t;
    float u[16];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint4 w = philox(make_uint4(gi, (uint32_t)tu, (uint32_t)(tu >> 32), TAG_DRAW | j), k0, k1);
        u[4 * j + 0] = u24(w.x);
        u[4 * j + 1] = u24(w.y);
        u[4 * j + 2] = u24(w.z);
        u[4 * j + 3] = u24(w.w);
    }
    s[0] = lo[0] + (hi[0] - lo[0]) * u[0];
    s[1] = lo[1] + (hi[1] - lo[1]) * u[1];
    s[2] = lo[2] + (hi[2] - lo[2]) * u[2];
    gx = lo[0] + (hi[0] - lo[0]) * u[3];
    gy = lo[1] + (hi[1] - lo[1]) * u[4];
    gz = lo[2] + (hi[2] - lo[2]) * u[5];
    // angles in units of pi: beta = -1 + 2 u6, yaw = -1 + 2 u8 (both exact in FP32)
    float cb, sb, ct, st, cy, sy;
    sincospif(-1.0f + 2.0f * u[6], &sb, &cb);
    sincospif(u[7] * (1.0f / 12.0f), &st, &ct);        // tau / 2 = (pi/6) u7 / 2
    sincospif(0.5f * (-1.0f + 2.0f * u[8]), &sy, &cy); // psi / 2
    const float b1 = st * cb, b2 = st * sb;
    s[6] = cy * ct;
    s[7] = cy * b1 - sy * b2;
    s[8] = cy * b2 + sy * b1;
    s[9] = sy * ct;
    float nrm[6];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const float r = sqrtf(-2.0f * logf(1.0f - u[9 + 2 * p]));
        float sn, cs;
        sincospif(2.0f * u[10 + 2 * p], &sn, &cs);
        nrm[2 * p] = r * cs;
        nrm[2 * p + 1] = r * sn;
    }
    s[3] = 0.5f * nrm[0]; s[4] = 0.5f * nrm[1]; s[5] = 0.5f * nrm[2];
    s[10] = 0.2f * nrm[3]; s[11] = 0.2f * nrm[4]; s[12] = 0.2f * nrm[5];
}

}  // namespace ag
