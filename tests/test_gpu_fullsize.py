"""The 1,048,576-quad mixed-mode workload at full size, in the launch
configuration the benchmark times (autotuned fused policy replayed from a HIP
graph) against plain per-step launches and the FP64 oracle on sampled
vehicles.

* fused (autotuned, and each fused form in the shapes the benchmark tunes
  to) and per-step final states bitwise identical after 1,000 steps;
* one step from the GPU's FP32 state at step 999 reproduces the GPU's step
  1,000 within FP32 rounding of the oracle (relative 1e-5, unit floor), on
  4,096 sampled vehicles of every mode;
* position-mode vehicles (sampled) after 500 steps within 1e-4 m of an FP64
  oracle rollout from the initial state.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from parity import need_gpu, oracle_inputs, to_vm64, same_rotation_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full_c2():
    need_gpu()
    from paper_2305_16510_amd.sim import Sim
    wl = workloads.c2_scale()
    assert wl.n == 1_048_576
    # fused, autotuned and graph-replayed (the benchmark's configuration)
    fused = Sim.from_workload(wl, autotune_scratch=True)
    tuned = fused.autotune(64)
    print("autotuned", tuned, flush=True)
    fused.step(500)
    mid = fused.state.clone()
    fused.step(499)
    pre = fused.state.clone()
    fused.step(1)
    fused.sync()
    out = {"tuned": tuned, "mid": to_vm64(mid), "pre": to_vm64(pre), "fused": fused.state.clone()}
    fused.close()
    plain = Sim.from_workload(wl)
    plain.set_exec(kind=0, block=64, use_graph=0)
    plain.step(1000)
    plain.sync()
    out["plain"] = plain.state.clone()
    plain.close()
    return wl, out


def test_fused_equals_per_step_at_full_size(full_c2):
    _, r = full_c2
    assert torch.equal(r["fused"], r["plain"])


@pytest.mark.parametrize("policy", [dict(kind=2, block=64, vpl=1, k=20, grid=0, use_graph=1),
                                    dict(kind=2, block=64, vpl=1, k=512, grid=0, use_graph=1),
                                    dict(kind=1, block=256, vpl=1, k=20, grid=0, use_graph=1)])
def test_each_fused_form_at_full_size(full_c2, policy):
    """Both fused forms (work queues and one block per tile) in the shapes the
    benchmark tunes to, 1,000 steps in 20-step calls and in one call,
    against the per-step launches."""
    wl, r = full_c2
    from paper_2305_16510_amd.sim import Sim
    sim = Sim.from_workload(wl)
    sim.set_exec(**policy)
    if policy["k"] == 20:
        sim.prepare(20)
        for _ in range(50):
            sim.step(20)
    else:
        sim.step(1000)
    sim.sync()
    got = sim.state.clone()
    sim.close()
    assert torch.equal(got, r["plain"]), policy


def test_sampled_one_step_parity_at_step_1000(full_c2):
    wl, r = full_c2
    rng = np.random.default_rng(70)
    idx = torch.as_tensor(np.sort(rng.choice(wl.n, 4096, replace=False)))
    _, mode, tgt, fleet = oracle_inputs(wl)
    pre = r["pre"][idx]
    gpu = to_vm64(r["fused"])[idx]
    ref, _ = oracle.step.step(pre, mode[idx], tgt[idx], fleet.select(idx), wl.dt, wl.g)
    finite = torch.isfinite(pre).all(-1)
    err = ((gpu - ref).abs() / torch.clamp(ref.abs(), min=1.0))[finite].max()
    print("modes sampled:", np.bincount(mode[idx].numpy(), minlength=3).tolist(),
          "one-step max rel err at step 1000:", float(err))
    assert finite.all()
    assert err <= 1e-5


def test_sampled_position_mode_after_500_steps(full_c2):
    wl, r = full_c2
    s0, mode, tgt, fleet = oracle_inputs(wl)
    pos = torch.nonzero(mode == 0).flatten()
    rng = np.random.default_rng(71)
    idx = pos[torch.as_tensor(np.sort(rng.choice(pos.numel(), 2048, replace=False)))]
    ref, _, _ = oracle.step.rollout(s0[idx], mode[idx], tgt[idx], fleet.select(idx), wl.dt, wl.g, 500)
    gpu = r["mid"][idx]
    dx = (gpu[:, 0:3] - ref[:, 0:3]).norm(dim=-1)
    print("position error after 500 steps (2,048 sampled position-mode vehicles): max %.3e median %.3e" %
          (dx.max(), dx.median()))
    assert dx.max() <= 1e-4
    assert same_rotation_err(gpu[:, 6:10], ref[:, 6:10]).max() <= 1e-4
