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
