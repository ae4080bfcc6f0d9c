"""Gym-style vectorised goal-reaching environment over the C ABI.

The paper imitates standard RL environments (Sec. III) and trains goal
reaching with attitude or velocity commands (Sec. I).  ``GoalReachEnv``
holds n vehicles with goals drawn by the counter-based reset; an action is
a [4, n] tensor in [-1, 1] mapped to velocity commands (v_d in the vehicle
frame, yaw rate) or attitude commands (roll, pitch, yaw rate, thrust).  One
``step`` = apply actions (kernel), ``decimation`` simulator steps, observe
(kernel: observation, reward, termination), reset of the finished vehicles
(counter-based redraw of state and goal) and their new observation.
"""
import torch

from . import lib as L
from .sim import Group, Sim

INTERFACES = {
    # mode, scale, offset of the 4 command rows
    "velocity": (1, (2.0, 2.0, 2.0, 1.0), (0.0, 0.0, 0.0, 0.0)),
    "attitude": (2, (0.5, 0.5, 1.0, 7.5), (0.0, 0.0, 0.0, 12.5)),
}


class GoalReachEnv:
    def __init__(self, n, interface="velocity", decimation=1, max_steps=500, seed=0, dt=0.01,
                 box=5.0, task=None, device="cuda:0"):
        self.mode, self.scale, self.offset = INTERFACES[interface]
        # every vehicle at rest at the origin, level, until reset() redraws it
        state0 = torch.zeros(13, n)
        state0[6] = 1.0
        self.sim = Sim([Group(0, n)], state0, torch.full((n,), self.mode, dtype=torch.int8),
                       torch.zeros(4, n), dt=dt, seed=seed, reset_prob=0.0, reset_lo=(-box,) * 3,
                       reset_hi=(box,) * 3, goal=torch.zeros(3, n), device=device)
        self.n = n
        self.decimation = decimation
        self.task = task or L.Task(0.05, 0.01, 1.0, 0.2, 4.0 * box, max_steps)
        dev = self.sim.device
        self.obs = torch.zeros(13, n, device=dev)
        self.reward = torch.zeros(n, device=dev)
        self.done = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.episode = torch.zeros(n, dtype=torch.int32, device=dev)
        self.t = 0

    def reset(self):
        """Redraw every vehicle's state and goal; returns the observation [13, n]."""
        ones = torch.ones(self.n, dtype=torch.uint8, device=self.sim.device)
        self.sim.reset(self.t, mask=ones, want_indices=False)
        self.episode.zero_()
        self.sim.observe(self.task, self.obs, advance=False)
        return self.obs

    def step(self, actions):
        self.sim.apply_actions(actions, self.mode, self.scale, self.offset)
        self.sim.step(self.decimation)
        self.t += self.decimation
        self.sim.observe(self.task, self.obs, self.reward, self.done, self.episode, advance=True)
        self.sim.reset(self.t, mask=self.done, want_indices=False)
        self.sim.observe(self.task, self.obs, advance=False)
        return self.obs, self.reward, self.done, {}

    def close(self):
        self.sim.close()
