"""Argument errors of calls on a live handle, through the C ABI: each is
rejected on the host before any launch with the documented status, and the
handle stays usable (an invalid argument is not a sticky error)."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads
from parity import need_gpu

pytestmark = pytest.mark.gpu


def make(**kw):
    from paper_2305_16510_amd.sim import Sim
    return Sim.from_workload(workloads.c2_scale(n=3000, seed=90), **kw)


def expect(status, fn):
    from paper_2305_16510_amd import lib as L
    with pytest.raises(L.AgError) as e:
        fn()
    assert e.value.status == status, str(e.value)
    return str(e.value)


@pytest.mark.parametrize("bad", [dict(kind=3), dict(kind=2), dict(kind=2, block=64, vpl=2), dict(block=100), dict(block=1024), dict(vpl=3),
                                 dict(kind=1, k=0), dict(grid=-1)])
def test_invalid_exec_policies(bad):
    need_gpu()
    from paper_2305_16510_amd import lib as L
    sim = make()
    pol = dict(kind=1, block=256, vpl=1, k=16, grid=0, use_graph=1)
    pol.update(bad)
    before = sim.get_exec()
    expect(L.AG_E_INVALID, lambda: sim.set_exec(**pol))
    assert sim.get_exec() == before                       # the policy is unchanged
    sim.close()


def test_automatic_resets_limit_k():
    need_gpu()
    from paper_2305_16510_amd import lib as L
    sim = make(auto_reset=True, reset_prob=0.01)
    msg = expect(L.AG_E_INVALID, lambda: sim.set_exec(kind=1, block=256, vpl=1, k=65, grid=0, use_graph=1))
    assert "64" in msg
    sim.set_exec(kind=1, block=256, vpl=1, k=64, grid=0, use_graph=1)
    sim.step(70)
    sim.sync()
    assert torch.isfinite(sim.state).all()
    sim.close()


def test_rollout_needs_per_vehicle_parameters_and_workspace():
    need_gpu()
    from paper_2305_16510_amd import lib as L
    sim = make()                                          # no vparams
    expect(L.AG_E_UNSUPPORTED, lambda: sim.rollout_forward(10, 5))
    sim.close()
    wl = workloads.c4_grad(n=2048)
    from paper_2305_16510_amd.sim import Sim
    sim = Sim.from_workload(wl)
    need = sim.rollout_workspace(10, 5).numel()
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    loss = torch.empty(sim.n, device="cuda")
    st = sim._lib.ag_rollout_forward(sim.h, C.c_void_p(0), C.c_void_p(0), 10, 5, C.c_float(0.01),
                                     C.c_void_p(small.data_ptr()), C.c_size_t(small.numel()),
                                     C.c_void_p(loss.data_ptr()), C.c_void_p(0), C.c_void_p(0))
    assert st == L.AG_E_NOMEM
    loss2, _, _ = sim.rollout_forward(10, 5)              # the handle still works
    sim.sync()
    assert torch.isfinite(loss2).all()
    sim.close()


def test_camera_and_target_ranges():
    need_gpu()
    from paper_2305_16510_amd import lib as L
    sim = make()
    shapes = np.zeros((257, 8), np.float32)
    obst = torch.zeros(7, sim.n * 257, device="cuda")
    expect(L.AG_E_INVALID, lambda: sim.render_depth(shapes, obst, 64, 4, 1.0, 10.0))
    expect(L.AG_E_INVALID, lambda: sim.render_depth(None, None, 64, 4, 3.5, 10.0))          # hfov >= pi
    expect(L.AG_E_INVALID, lambda: sim.set_targets(sim.n - 10, 20, target=torch.zeros(4, 20)))
    ref = sim.state.clone()
    sim.step(3)
    sim.sync()
    assert not torch.equal(ref, sim.state) and torch.isfinite(sim.state).all()
    sim.close()
