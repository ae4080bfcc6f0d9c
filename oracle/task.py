"""Goal-reaching task of a Gym-style vectorised environment, FP64 (oracle;
test infrastructure only).

The paper exposes its simulator through Gym-style reset/step interfaces
(Sec. III) and trains goal reaching with attitude and velocity commands
(Sec. I).  Reading (R32) of the task computed after every environment step:

  obs    = (goal - x, v, q, Omega)                 13 values per vehicle
  reward = -|goal - x| - w_v |v| - w_omega |Omega| + bonus [|goal - x| < r_goal]
  done   = episode step >= max_steps, or |goal - x| > r_far, or a non-finite
           state (the episode counter of a finished vehicle restarts at 0)

The goal is the position-mode target (rows 0-2).
"""
import numpy as np


def observe(state, goal, episode, w_v, w_omega, bonus, r_goal, r_far, max_steps):
    """state [n,13], goal [n,3], episode int [n] (steps already taken in the
    episode, before this one) -> obs [n,13], reward [n], done bool [n], new episode [n]."""
    s = np.asarray(state, np.float64)
    e = np.asarray(goal, np.float64) - s[:, 0:3]
    dist = np.linalg.norm(e, axis=-1)
    obs = np.concatenate([e, s[:, 3:13]], -1)
    reward = (-dist - w_v * np.linalg.norm(s[:, 3:6], axis=-1) - w_omega * np.linalg.norm(s[:, 10:13], axis=-1)
              + np.where(dist < r_goal, bonus, 0.0))
    ep = np.asarray(episode, np.int64) + 1
    finite = np.isfinite(s).all(-1)
    done = (ep >= max_steps) | (dist > r_far) | ~finite
    reward = np.where(finite, reward, 0.0)
    obs = np.where(finite[:, None], obs, 0.0)
    return obs, reward, done, np.where(done, 0, ep)
