"""The autotuner's cache: a second simulator of the same shape takes the
cached policy without timing candidates, different call lengths are tuned
separately, a cache file carries choices to a new process, and every choice
gives bitwise the results of plain per-step launches."""
import os
import subprocess
import sys
import textwrap
import time

import pytest
import torch

import workloads
from parity import need_gpu

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def make_sim(wl, **kw):
    from paper_2305_16510_amd.sim import Sim
    return Sim.from_workload(wl, autotune_scratch=True, **kw)


def test_second_simulator_takes_cached_policy():
    need_gpu()
    wl = workloads.c2_scale(n=150_001, seed=61)
    s1 = make_sim(wl)
    t0 = time.perf_counter()
    e1 = s1.autotune(48)
    t_search = time.perf_counter() - t0
    s1.close()
    s2 = make_sim(wl)
    before = s2.state.clone()
    t0 = time.perf_counter()
    e2 = s2.autotune(48)
    t_cached = time.perf_counter() - t0
    s2.sync()
    print("search %.3f s, cached %.4f s, %s" % (t_search, t_cached, e1))
    assert e1 == e2
    assert t_cached < 0.1 * t_search
    assert torch.equal(s2.state, before)            # the cached path runs nothing
    s2.step(48)
    s2.sync()
    fused = s2.state.clone()
    s2.close()
    s3 = make_sim(wl)
    s3.set_exec(kind=0, block=256, use_graph=0)
    s3.step(48)
    s3.sync()
    assert torch.equal(fused, s3.state)
    s3.close()


def test_call_lengths_tuned_separately():
    need_gpu()
    wl = workloads.c2_scale(n=70_000, seed=62)
    sim = make_sim(wl)
    short = sim.autotune(12)
    assert short["k"] <= 12
    long_ = sim.autotune(300)
    assert sim.autotune(12) == short and sim.autotune(300) == long_
    sim.close()


def test_cache_file_carries_choice_to_new_process(tmp_path):
    need_gpu()
    path = tmp_path / "tune.txt"
    code = textwrap.dedent(f"""
        import sys, time
        sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})
        import workloads
        from paper_2305_16510_amd.sim import Sim
        wl = workloads.c2_scale(n=40_000, seed=63)
        sim = Sim.from_workload(wl, autotune_scratch=True)
        t0 = time.perf_counter()
        e = sim.autotune(40)
        print(time.perf_counter() - t0, e["block"], e["vpl"], e["k"], e["grid"], flush=True)
        sim.close()
    """)
    env = dict(os.environ, AG_AUTOTUNE_CACHE=str(path))
    outs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        outs.append(r.stdout.split())
    lines = path.read_text().splitlines()
    print(lines, outs)
    assert len(lines) == 1 and "/n40000/" in lines[0] and "/L40 " in lines[0]
    assert outs[0][1:] == outs[1][1:]
    assert float(outs[1][0]) < 0.1 * float(outs[0][0])
