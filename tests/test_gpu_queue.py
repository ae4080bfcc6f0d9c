"""The work-queue form of the fused kernel (exec kind 2) against plain
per-step launches, bitwise: mixed command modes (wrench mode and an unknown
code included) in mode order and in calls too short for the order, each
rotor layout, fewer tiles than queues and ragged last tiles,
repeated calls and graph replays over the same queues (which the last
wavefront of each launch clears), and the configurations it refuses."""
import numpy as np
import pytest
import torch

import workloads
from parity import need_gpu

pytestmark = pytest.mark.gpu

PLAIN = dict(kind=0, block=256, use_graph=0)


def mixed(n, seed):
    wl = workloads.c2_scale(n=n, seed=seed, steps=100)
    rng = np.random.default_rng(seed)
    sel = rng.random(n)
    w3 = sel < 0.08
    wl.mode[w3] = 3
    wl.target[:, w3] = np.stack([rng.uniform(0, 20, w3.sum()), rng.normal(0, 0.05, w3.sum()),
                                 rng.normal(0, 0.05, w3.sum()), rng.normal(0, 0.01, w3.sum())]
                                ).astype(np.float32)
    wl.mode[sel > 0.99] = 9
    return wl


def run(wl, policy, calls):
    from paper_2305_16510_amd.sim import Sim
    sim = Sim.from_workload(wl)
    sim.set_exec(**policy)
    for n in calls:
        sim.step(n)
    sim.sync()
    out = sim.state.clone()
    assert sim.step_counter == sum(calls)
    sim.close()
    return out


@pytest.mark.parametrize("k,grid,graph", [(16, 0, 1), (7, 8, 0), (64, 24, 1), (45, 1000, 0), (48, 0, 0)])
def test_mixed_modes_in_mode_order(k, grid, graph):
    need_gpu()
    wl = mixed(100_003, 81)
    ref = run(wl, PLAIN, [45, 3])
    got = run(wl, dict(kind=2, block=64, vpl=1, k=k, grid=grid, use_graph=graph), [45, 3])
    assert torch.equal(got, ref)


@pytest.mark.parametrize("n,modes", [(600_011, None), (300_000, 0)])
def test_queues_with_whole_segments(n, modes):
    """Queues longer than a segment of the mode order (64 tiles), so that
    wavefronts take tiles on demand long after their first; a ragged fleet
    with every mode, and an all-position fleet (n = 300,000: 146 or 147
    tiles a queue)."""
    need_gpu()
    wl = mixed(n, 84)
    if modes is not None:
        wl.mode[:] = modes
    assert (n + 63) // 64 // 32 >= 64                      # at least 64 tiles a queue
    ref = run(wl, PLAIN, [40])
    got = run(wl, dict(kind=2, block=64, vpl=1, k=13, grid=0, use_graph=1), [40])
    assert torch.equal(got, ref)


def test_short_calls_without_order():
    need_gpu()
    wl = mixed(30_001, 82)
    ref = run(wl, PLAIN, [5, 9, 2])
    got = run(wl, dict(kind=2, block=64, vpl=1, k=4, grid=0, use_graph=1), [5, 9, 2])
    assert torch.equal(got, ref)


@pytest.mark.parametrize("nr", [6, 8])
def test_hexa_and_octo_layouts(nr):
    need_gpu()
    wl = mixed(20_000, 83 + nr)
    wl.groups = [workloads.Group(first=0, count=wl.n, n_rotors=nr, u_max=24.0 / nr)]
    ref = run(wl, PLAIN, [30])
    got = run(wl, dict(kind=2, block=64, vpl=1, k=10, grid=0, use_graph=1), [30])
    assert torch.equal(got, ref)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 300, 511, 513, 4097])
def test_few_tiles_and_ragged_tails(n):
    """Fewer tiles than the 32 queues (n <= 1984: some queues hand out
    nothing) and last tiles of 1 to 63 vehicles."""
    need_gpu()
    wl = mixed(n, 90 + n)
    ref = run(wl, PLAIN, [12, 20])
    got = run(wl, dict(kind=2, block=64, vpl=1, k=5, grid=0, use_graph=1), [12, 20])
    assert torch.equal(got, ref)


def test_repeated_calls_and_graph_replays():
    """Six calls replaying one cached graph of four launches, a one-step
    call and a 40-step direct launch: each launch finds the queues cleared."""
    need_gpu()
    wl = mixed(70_001, 96)
    calls = [20] * 6 + [1, 40]
    ref = run(wl, PLAIN, calls)
    from paper_2305_16510_amd.sim import Sim
    sim = Sim.from_workload(wl)
    sim.set_exec(kind=2, block=64, vpl=1, k=5, grid=64, use_graph=1)
    for c in calls[:-1]:
        sim.step(c)
    sim.set_exec(kind=2, block=64, vpl=1, k=40, grid=0, use_graph=0)
    sim.step(calls[-1])
    sim.sync()
    got = sim.state.clone()
    sim.close()
    assert torch.equal(got, ref)


def test_refused_configurations():
    """Observers, per-vehicle parameters and several groups need the other
    kinds; the handle keeps its policy."""
    need_gpu()
    from paper_2305_16510_amd import lib as L
    from paper_2305_16510_amd.sim import Sim
    q = dict(kind=2, block=64, vpl=1, k=8, grid=0, use_graph=1)
    cases = [(workloads.c2_scale(n=3000, seed=97), dict(collect_stats=True)),
             (workloads.c2_scale(n=3000, seed=97), dict(outputs=True)),
             (workloads.c3_uneven(scale=0.005, seed=98), {})]
    for wl, kw in cases:
        sim = Sim.from_workload(wl, **kw)
        before = sim.get_exec()
        with pytest.raises(L.AgError) as e:
            sim.set_exec(**q)
        assert e.value.status == L.AG_E_INVALID and "kind 2" in str(e.value)
        assert sim.get_exec() == before
        sim.close()
