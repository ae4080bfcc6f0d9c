"""ag_rollout_grad_noalloc (the forward and adjoint of the differentiable
rollout on the library's static scratch) against ag_rollout_forward +
ag_rollout_adjoint on a caller workspace: bitwise equal per-vehicle loss,
batch loss and gradients, on two calls in a row (the 65,536-vehicle
200-step rollout, then a smaller one on another handle, which reuses the
scratch the first call left behind); free device memory unchanged by the
calls (measured after the workspace calls have launched the same kernels);
an oversized rollout rejected with AG_E_NOMEM, the handle still usable."""
import ctypes as C

import pytest
import torch

import workloads
from parity import need_gpu

pytestmark = pytest.mark.gpu


def reference(sim, T, m, seed):
    ws = sim.new_rollout_workspace(T, m)
    loss, batch, _ = sim.rollout_forward(T, m, 0.01, ws=ws)
    dg, dx = sim.rollout_adjoint(T, m, 0.01, seed_grad=seed, ws=ws)
    sim.sync()
    return loss, batch, dg, dx


def outputs(sim):
    return (torch.empty(sim.n, device="cuda"), torch.empty(1, device="cuda"),
            torch.empty(10, sim.n, device="cuda"), torch.empty(13, sim.n, device="cuda"))


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_equals_workspace_calls(order):
    need_gpu()
    from paper_2305_16510_amd.sim import Sim
    big = workloads.c4_grad()                                   # 65,536 x 200, checkpoint every 20
    small = workloads.c4_grad(n=3001, seed=81, steps=60)
    cases = [(Sim.from_workload(big), big.steps, 20, 1.0), (Sim.from_workload(small), 60, 7, 2.5)]
    for j, (sim, T, m, seed) in enumerate(cases):
        print(f"call {j + 1}: n={sim.n} T={T} m={m}", flush=True)
        # the workspace calls first: the runtime's own set-up of these kernels
        # (code objects, their private segments) happens there
        ref = reference(sim, T, m, seed)
        out = outputs(sim)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        got = sim.rollout_grad_noalloc(T, m, 0.01, seed_grad=seed, out=out)
        sim.sync()
        free1, _ = torch.cuda.mem_get_info()
        for a, b, name in zip(got, ref, ("loss", "batch", "dgains", "dx0")):
            assert torch.equal(a, b), (j, name)
        assert free1 == free0, (j, free0 - free1)
        sim.close()


def test_noalloc_rejects_oversized_rollout():
    need_gpu()
    from paper_2305_16510_amd import lib as L
    from paper_2305_16510_amd.sim import Sim
    wl = workloads.c4_grad(n=65_536, seed=82, steps=40)
    sim = Sim.from_workload(wl)
    # 1,000 steps checkpointed every 500: 2 + 1,000 states of 52 B per vehicle, 3.4 GB
    with pytest.raises(L.AgError) as ei:
        sim.rollout_grad_noalloc(1000, 500)
    assert ei.value.status == L.AG_E_NOMEM and "static scratch" in str(ei.value)
    loss, batch, dg, dx = sim.rollout_grad_noalloc(40, 10)     # the handle still works
    sim.sync()
    assert torch.isfinite(dg).all() and torch.isfinite(batch).all()
    sim.close()
