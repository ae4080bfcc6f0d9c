"""FP64 CPU oracle of the batched multirotor step (test infrastructure only).

This package is the checker, not the product.  Only the test suite, the smoke
check of ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path: it is written from the paper
(Kulkarni, Forgaard, Alexis, "Aerial Gym -- Isaac Gym Simulator for Aerial
Robots", arXiv 2305.16510, Sec. IV, eqs. (1)-(9)) and from the published
definitions of the pieces the paper delegates to its physics engine.

Everything is plain ``torch.float64`` on the CPU, vectorised over vehicles,
written in the order and notation of the paper so that it can be read against
it.  Readings of silent or garbled passages are collected in ``readings.py``.

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
"""
from . import so3, controller, allocation, dynamics, step, philox, reset, stats  # noqa: F401
from .fleet import Fleet  # noqa: F401
