"""Planted mistakes in the oracle (on the CPU) must be caught by the pins:
each test swaps one plausible error into an oracle function and checks that
the matching pin test then fails."""
import pytest
import torch

import oracle.allocation as allocation
import oracle.controller as controller
import oracle.dynamics as dynamics
from oracle import so3
import test_oracle_allocation as ta
import test_oracle_controller as tc
import test_oracle_dynamics as td
import test_oracle_grad as tg


def test_transposed_attitude_error_is_caught(monkeypatch):
    def bad(R, R_d, Omega, Omega_d):
        e_R = 0.5 * so3.vee(R.transpose(-1, -2) @ R_d - R_d.transpose(-1, -2) @ R)
        return e_R, Omega - so3.mv(R.transpose(-1, -2) @ R_d, Omega_d)
    monkeypatch.setattr(controller, "attitude_errors", bad)
    with pytest.raises(AssertionError):
        tc.test_attitude_error_closed_form()


def test_gyroscopic_sign_is_caught(monkeypatch):
    def bad(e_R, e_W, Omega, J, kR, kW):
        return -kR * e_R - kW * e_W - torch.cross(Omega, J * Omega, dim=-1)
    monkeypatch.setattr(controller, "moment", bad)
    with pytest.raises(AssertionError):
        tc.test_attitude_mode_on_target_gives_gyroscopic_moment_only()


def test_swapped_tilt_angles_are_caught(monkeypatch):
    orig = controller.tilt_from_force
    monkeypatch.setattr(controller, "tilt_from_force", lambda F: tuple(reversed(orig(F))))
    with pytest.raises(AssertionError):
        tc.test_desired_rotation_aligns_b3_with_force()


def test_wrong_spin_sign_is_caught(monkeypatch):
    orig = allocation.layout
    monkeypatch.setattr(allocation, "layout", lambda n: (orig(n)[0], -orig(n)[1]))
    with pytest.raises(AssertionError):
        ta.test_x_layout_geometry()
    with pytest.raises(AssertionError):
        ta.test_pseudo_inverse_closed_form(6)


def test_pre_step_rate_in_quaternion_update_is_caught(monkeypatch):
    def bad(x, v, q, Omega, f_app, M_app, fleet, dt, g):
        xn, vn, qn, Wn = orig(x, v, q, Omega, f_app, M_app, fleet, dt, g)
        zero = torch.zeros_like(Omega[:, :1])
        q_t = q + 0.5 * dt * so3.quat_mul(torch.cat([zero, Omega], -1), q)   # inertial-frame rate
        return xn, vn, q_t / q_t.norm(dim=-1, keepdim=True), Wn
    orig = dynamics.integrate
    import oracle.step as ostep
    monkeypatch.setattr(ostep, "integrate", bad)
    with pytest.raises(AssertionError):
        td.test_quaternion_update_constant_body_rate()


def test_loss_counting_initial_state_is_caught(monkeypatch):
    import oracle.step as ostep
    orig = ostep.per_vehicle_loss

    def bad(state0, mode, target, fleet, dt, g, steps, w_omega):
        li, s = orig(state0, mode, target, fleet, dt, g, steps, w_omega)
        return li + ((state0[:, 0:3] - target[:, 0:3]) ** 2).sum(-1), s
    monkeypatch.setattr(ostep, "per_vehicle_loss", bad)
    with pytest.raises(AssertionError):
        tg.test_loss_is_sum_over_post_step_states()


# ---- position / velocity commands with split gains ---------------------------
def test_swapped_gain_split_is_caught(monkeypatch):
    def bad(gains):
        kx = torch.stack([gains[:, 1], gains[:, 1], gains[:, 0]], -1)
        kv = torch.stack([gains[:, 3], gains[:, 3], gains[:, 2]], -1)
        return kx, kv, gains[:, 4:7], gains[:, 7:10]
    monkeypatch.setattr(controller, "gain_vectors", bad)
    for pin in (tc.test_position_mode_vertical_velocity_is_damped_by_kv_z,
                tc.test_position_mode_horizontal_velocity_tilts_against_it,
                tc.test_position_mode_offset_uses_kx_xy_and_kx_z,
                tc.test_velocity_mode_split_gains_at_nonzero_velocity):
        with pytest.raises(AssertionError):
            pin()


def test_flipped_position_damping_is_caught(monkeypatch):
    monkeypatch.setattr(controller, "position_accel", lambda kx, kv, xd, x, v: kx * (xd - x) + kv * v)
    with pytest.raises(AssertionError):
        tc.test_position_mode_vertical_velocity_is_damped_by_kv_z()
    with pytest.raises(AssertionError):
        tc.test_position_mode_horizontal_velocity_tilts_against_it()


def test_flipped_velocity_error_is_caught(monkeypatch):
    monkeypatch.setattr(controller, "velocity_accel", lambda kv, vd, vV: kv * (vV - vd))
    with pytest.raises(AssertionError):
        tc.test_velocity_mode_split_gains_at_nonzero_velocity()


# ---- Box-Muller normals of the reset redraw ------------------------------------
import numpy as np  # noqa: E402
import math  # noqa: E402

import oracle.reset as oreset  # noqa: E402
import oracle.stats as ostats  # noqa: E402
import oracle.task as otask  # noqa: E402
import test_oracle_philox_reset as tr  # noqa: E402
import test_oracle_task_stats as tts  # noqa: E402


def test_box_muller_log_of_u_is_caught(monkeypatch):
    def bad(ua, ub):
        r = np.sqrt(-2.0 * np.log(np.maximum(ua, 1e-300)))
        return r * np.cos(2 * math.pi * ub), r * np.sin(2 * math.pi * ub)
    monkeypatch.setattr(oreset, "box_muller", bad)
    with pytest.raises(AssertionError):
        tr.test_redraw_normals_closed_form()


def test_box_muller_swapped_cos_sin_is_caught(monkeypatch):
    orig = oreset.box_muller
    monkeypatch.setattr(oreset, "box_muller", lambda ua, ub: tuple(reversed(orig(ua, ub))))
    with pytest.raises(AssertionError):
        tr.test_redraw_normals_closed_form()


def test_swapped_reset_sigmas_are_caught(monkeypatch):
    monkeypatch.setattr(oreset, "VEL_SIGMA", 0.2)
    monkeypatch.setattr(oreset, "RATE_SIGMA", 0.5)
    with pytest.raises(AssertionError):
        tr.test_redraw_normals_closed_form()
    with pytest.raises(AssertionError):
        tr.test_redraw_normals_statistics()


# ---- goal-reaching task ----------------------------------------------------------
def _task_variant(change):
    orig = otask.observe

    def bad(state, goal, episode, w_v, w_omega, bonus, r_goal, r_far, max_steps):
        obs, rew, done, ep = orig(state, goal, episode, w_v, w_omega, bonus, r_goal, r_far, max_steps)
        s = np.asarray(state, np.float64)
        dist = np.linalg.norm(np.asarray(goal, np.float64) - s[:, 0:3], axis=-1)
        return change(s, dist, np.asarray(episode), obs, rew, done, ep, (w_v, w_omega, bonus, r_goal, r_far))
    return bad


TASK_MISTAKES = {
    "speed term with the wrong sign": lambda s, d, e, o, r, dn, ep, p: (
        o, r + 2 * p[0] * np.linalg.norm(s[:, 3:6], axis=-1), dn, ep),
    "bonus at the boundary": lambda s, d, e, o, r, dn, ep, p: (o, r + np.where(d == p[3], p[2], 0.0), dn, ep),
    "episode counter not restarted": lambda s, d, e, o, r, dn, ep, p: (o, r, dn, e + 1),
    "non-finite state not done": lambda s, d, e, o, r, dn, ep, p: (
        o, r, dn & np.isfinite(s).all(-1), ep),
    "non-finite observation kept": lambda s, d, e, o, r, dn, ep, p: (
        np.where(np.isfinite(s).all(-1)[:, None], o, s), r, dn, ep),
    "termination at r_far itself": lambda s, d, e, o, r, dn, ep, p: (o, r, dn | (d >= p[4]), ep),
}


@pytest.mark.parametrize("name", sorted(TASK_MISTAKES))
def test_task_mistakes_are_caught(monkeypatch, name):
    monkeypatch.setattr(otask, "observe", _task_variant(TASK_MISTAKES[name]))
    with pytest.raises(AssertionError):
        tts.test_task_hand_computed_cases()


# ---- batch statistics --------------------------------------------------------------
def test_stats_mistakes_are_caught(monkeypatch):
    orig = ostats.final_state_stats

    def omega_over_all(state, mode, target):
        r = orig(state, mode, target)
        r["omega_sum"] = float(torch.linalg.vector_norm(state[:, 10:13], dim=-1).sum())
        return r

    def error_over_all_modes(state, mode, target):
        r = orig(state, mode, target)
        fin = torch.isfinite(state).all(-1)
        err = torch.linalg.vector_norm(state[:, 0:3] - target[:, 0:3], dim=-1)
        r["pos_err_sum"] = float(err[fin].sum())
        r["n_position"] = int(fin.sum())
        return r

    for bad in (omega_over_all, error_over_all_modes):
        monkeypatch.setattr(ostats, "final_state_stats", bad)
        with pytest.raises(AssertionError):
            tts.test_stats_hand_built_state()


def test_clamp_distance_against_one_bound_only_is_caught(monkeypatch):
    def bad(raw, fleet):
        N = raw.shape[0]
        d = torch.full((N,), float("inf"), dtype=raw.dtype)
        for nr in sorted(set(int(k) for k in fleet.n_rotors.tolist())):
            idx = (fleet.n_rotors == nr).nonzero().squeeze(-1)
            d[idx] = (raw[idx, :nr] - fleet.u_min[idx, None]).abs().min(-1).values / fleet.u_max[idx]
        return d
    monkeypatch.setattr(allocation, "clamp_distance", bad)
    with pytest.raises(AssertionError):
        ta.test_clamp_distance_closed_form_and_rotor_columns()
