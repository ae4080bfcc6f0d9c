"""Goal-reaching task kernels (actions, observation, reward, termination)
and the Gym-style environment on the GPU, against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import task as otask
from parity import need_gpu

pytestmark = pytest.mark.gpu


def test_observation_reward_done_match_oracle():
    need_gpu()
    from paper_2305_16510_amd import lib as L
    from paper_2305_16510_amd.sim import Sim
    n = 10_007
    wl = workloads.c1_parity(n=n, seed=100)
    rng = np.random.default_rng(101)
    wl.state0[0:3] = rng.uniform(-12, 12, (3, n)).astype(np.float32)
    wl.state0[7, 5] = np.nan
    goal = rng.uniform(-5, 5, (3, n)).astype(np.float32)
    goal[:, :50] = wl.state0[0:3, :50] + 0.05                # near the goal: bonus
    episode = rng.integers(0, 30, n).astype(np.int32)
    sim = Sim.from_workload(wl, goal=goal)
    task = L.Task(0.05, 0.01, 1.0, 0.2, 15.0, 30)
    obs = torch.zeros(13, n, device="cuda")
    rew = torch.zeros(n, device="cuda")
    done = torch.zeros(n, dtype=torch.uint8, device="cuda")
    ep = torch.as_tensor(episode).cuda()
    sim.observe(task, obs, rew, done, ep, advance=True)
    sim.sync()
    sim.close()
    o, r, d, e = otask.observe(wl.state0.T, goal.T, episode, 0.05, 0.01, 1.0, 0.2, 15.0, 30)
    dist = np.linalg.norm(goal.T.astype(np.float64) - wl.state0[0:3].T, axis=-1)
    safe = (np.abs(dist - 15.0) > 1e-4) & (np.abs(dist - 0.2) > 1e-4)
    assert np.abs(obs.cpu().numpy().T - o)[safe].max() <= 1e-6
    assert np.abs(rew.cpu().numpy() - r)[safe].max() <= 1e-5 * np.abs(r).max()
    assert np.array_equal(done.cpu().numpy().astype(bool)[safe], d[safe])
    assert np.array_equal(ep.cpu().numpy()[safe], e[safe])
    assert d[5] and (r[:50] > 0).any()


def test_actions_map_to_commands():
    need_gpu()
    from paper_2305_16510_amd.sim import Sim
    n = 3000
    wl = workloads.c1_parity(n=n, seed=102)
    sim = Sim.from_workload(wl)
    a = np.random.default_rng(103).uniform(-1.5, 1.5, (4, n)).astype(np.float32)
    scale, offset = (0.5, 0.5, 1.0, 7.5), (0.0, 0.0, 0.0, 12.5)
    sim.apply_actions(torch.as_tensor(a), 2, scale, offset)
    sim.sync()
    tgt = sim.target.cpu().numpy()
    mode = sim.mode.cpu().numpy()
    sim.close()
    ref = np.array(offset)[:, None] + np.array(scale)[:, None] * np.clip(a, -1, 1)
    assert np.abs(tgt - ref).max() <= 2e-6 * np.abs(ref).max()
    assert (mode == 2).all()


@pytest.mark.parametrize("interface", ["velocity", "attitude"])
def test_goal_reach_env_episode_resets(interface):
    """All episodes end after max_steps; finished vehicles get the counter-based
    redraw of state and goal, and their observation is of the new state."""
    need_gpu()
    from paper_2305_16510_amd import lib as L
    from paper_2305_16510_amd.env import GoalReachEnv
    n, T = 4096, 12
    env = GoalReachEnv(n, interface=interface, max_steps=T, seed=5,
                       task=L.Task(0.05, 0.01, 1.0, 0.2, 1e6, T))
    obs = env.reset()
    rng = np.random.default_rng(6)
    for t in range(T):
        obs, rew, done, _ = env.step(torch.as_tensor(rng.uniform(-1, 1, (4, n)).astype(np.float32)).cuda())
        env.sim.sync()
        d = done.cpu().numpy().astype(bool)
        assert d.all() == (t == T - 1) and (d.any() == (t == T - 1))
        assert torch.isfinite(rew).all()
    s = env.sim.state.cpu().numpy().T.astype(np.float64)
    g = env.sim.goal.cpu().numpy().T.astype(np.float64)
    s_ref, g_ref = oracle.reset.redraw(np.arange(n), T, 5, (-5.0,) * 3, (5.0,) * 3)
    assert np.abs(s - s_ref.numpy()).max() <= 2e-6 and np.abs(g - g_ref.numpy()).max() <= 1e-6
    o = obs.cpu().numpy().T
    assert np.abs(o[:, 0:3] - (g - s[:, 0:3])).max() <= 1e-5
    assert (env.episode.cpu().numpy() == 0).all()
    env.close()
