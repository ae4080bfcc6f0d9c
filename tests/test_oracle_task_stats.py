"""Pins of the goal-reaching task (Gym-style observation, reward and
termination of Sec. III / Sec. I, reading R32) and of the batch statistics,
on hand-built states whose results are worked out by hand."""
import math

import numpy as np
import torch

import oracle.stats as ostats
import oracle.task as otask

NAN = float("nan")
# w_v, w_omega, bonus, r_goal, r_far, max_steps
TASK = (0.05, 0.01, 1.0, 0.2, 20.0, 10)


def _state(x, v, q, w):
    return np.array(list(x) + list(v) + list(q) + list(w), np.float64)


def task_cases():
    q0 = (1.0, 0.0, 0.0, 0.0)
    qh = (0.5, 0.5, -0.5, 0.5)
    rows = [
        # x, v, q, Omega, goal, episode
        ((1, 2, 3), (0, 0, 2), q0, (1, 2, 2), (4, 6, 3), 0),        # ordinary step
        ((1, 1, 1), (0, 0, 0), qh, (0, 0, 0), (1, 1, 1), 3),        # at the goal: bonus
        ((0, 0, 0), (0, 0, 0), q0, (0, 0, 0), (0, 0, 25), 4),       # beyond r_far: done
        ((0, 0, 0), (3, 0, 4), q0, (0, 0, 0), (1, 0, 0), 9),        # last step of the episode
        ((0, 0, 0), (NAN, 0, 0), q0, (0, 0, 0), (1, 0, 0), 2),      # non-finite state
        ((0, 0, 0), (0, 0, 0), q0, (0, 0, 0), (0.2, 0, 0), 0),      # exactly r_goal away: no bonus
        ((0, 0, 0), (0, 0, 0), q0, (0, 0, 0), (0, 20, 0), 1),       # exactly r_far away: not done
    ]
    state = np.stack([_state(x, v, q, w) for x, v, q, w, _, _ in rows])
    goal = np.array([r[4] for r in rows], np.float64)
    ep = np.array([r[5] for r in rows], np.int64)
    return state, goal, ep


def test_task_hand_computed_cases():
    state, goal, ep = task_cases()
    obs, rew, done, ep2 = otask.observe(state, goal, ep, *TASK)
    w_v, w_o, bonus = TASK[0], TASK[1], TASK[2]
    # 0: goal - x = (3, 4, 0), |.| = 5; |v| = 2; |Omega| = 3
    assert np.array_equal(obs[0], [3, 4, 0, 0, 0, 2, 1, 0, 0, 0, 1, 2, 2])
    assert abs(rew[0] - (-5.0 - w_v * 2.0 - w_o * 3.0)) < 1e-15
    assert not done[0] and ep2[0] == 1
    # 1: at the goal: only the bonus; the observation carries q unchanged
    assert np.array_equal(obs[1], [0, 0, 0, 0, 0, 0, 0.5, 0.5, -0.5, 0.5, 0, 0, 0])
    assert rew[1] == bonus and not done[1] and ep2[1] == 4
    # 2: 25 m away, beyond r_far = 20: done, counter restarts
    assert rew[2] == -25.0 and done[2] and ep2[2] == 0
    # 3: the 10th step of a 10-step episode: done; |v| = 5
    assert abs(rew[3] - (-1.0 - w_v * 5.0)) < 1e-15 and done[3] and ep2[3] == 0
    # 4: non-finite: zero observation and reward, done
    assert np.array_equal(obs[4], np.zeros(13)) and rew[4] == 0.0 and done[4] and ep2[4] == 0
    # 5: the bonus needs |goal - x| < r_goal strictly
    assert rew[5] == -0.2 and not done[5]
    # 6: termination needs |goal - x| > r_far strictly
    assert rew[6] == -20.0 and not done[6] and ep2[6] == 2


def stats_cases():
    s = np.zeros((5, 13))
    s[:, 6] = 1.0
    s[0, 0:3] = (3, 4, 0); s[0, 10:13] = (0, 3, 4)          # position mode: err 5, |Omega| 5
    s[1, 0:3] = (1, 1, 1); s[1, 10:13] = (2, 0, 0)          # velocity mode: |Omega| 2
    s[2, 0:3] = (1, -2, 3); s[2, 10:13] = (0, 0, 0)         # position mode: err 1
    s[3, 0:3] = (3, 0, 0); s[3, 3] = NAN; s[3, 12] = 7.0    # position mode, non-finite
    s[4, 0:3] = (5, 5, 5); s[4, 10:13] = (0, -1, 0)         # attitude mode: |Omega| 1
    mode = np.array([0, 1, 0, 0, 2])
    target = np.zeros((5, 4))
    target[1, 0:3] = (9, 9, 9)                              # a velocity command, not a goal
    target[2, 0:3] = (1, -2, 2)
    return torch.as_tensor(s), mode, torch.as_tensor(target)


def test_stats_hand_built_state():
    s, mode, target = stats_cases()
    r = ostats.final_state_stats(s, mode, target)
    assert r["n_nonfinite"] == 1 and r["n_finite"] == 4
    assert r["n_position"] == 2
    assert r["pos_err_sum"] == 6.0
    assert r["omega_sum"] == 8.0
    assert math.isfinite(r["omega_sum"]) and math.isfinite(r["pos_err_sum"])


def test_fleet_rows_land_in_their_fields():
    """Per-vehicle parameter rows (m, J1, J2, J3, 10 gains, arm, u_max) reach
    the matching oracle fields; group defaults fill the rest."""
    from oracle.fleet import Fleet
    from workloads import Group
    n = 3
    vp = np.zeros((16, n), np.float32)
    for r in range(16):
        vp[r] = (r + 1) * 1.0 + np.arange(n) * 0.125
    f = Fleet.from_groups([Group(0, n, c_tau=0.03125, u_min=0.5)], n, vp)
    col = lambda r: torch.as_tensor(vp[r].astype(np.float64))
    assert torch.equal(f.m, col(0))
    for k in range(3):
        assert torch.equal(f.J[:, k], col(1 + k))
    for k in range(10):
        assert torch.equal(f.gains[:, k], col(4 + k))
    assert torch.equal(f.arm, col(14)) and torch.equal(f.u_max, col(15))
    assert (f.c_tau == 0.03125).all() and (f.u_min == 0.5).all() and (f.n_rotors == 4).all()
