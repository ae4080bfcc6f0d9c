#!/usr/bin/env python
"""Throughput of the batched multirotor step on one MI355X.

Workload (default): 1,048,576 X-quads, command mode drawn per vehicle from
{position, velocity, attitude}, dt = 0.01 s.  A bench step is one step of
every vehicle (controller, allocation, clamping, integration).  The timed
region runs K steps with the autotuned fused policy (k steps per launch,
state in registers, replayed from a HIP graph); the same K steps are also
timed as K plain per-step launches (no graph) and as K host calls of
ag_step(1).  Inputs are resident in HBM before timing starts.  Prints one
JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per vehicle-step.  Bytes of the per-step kernel: state in
# and out, 4-float command, mode byte.  Flops: the headline figure is the
# hot-path estimate for one quad step in position mode, about 380 FP32 flops
# (196 VALU operations, FMAs counted twice, plus 4 reciprocal square roots).
# A second figure counts one quad step per command mode operation by
# operation on that mode's path (an FMA as two, a reciprocal square root as
# one, per-vehicle constants hoisted, products with structural zeros and the
# 2^-60 biases excluded): position 215, velocity 221, attitude 188, wrench or
# unknown code 117.
BYTES_PER_VSTEP = 52 + 52 + 16 + 1
FLOPS_PER_VSTEP = 380.0
FLOPS_BY_MODE = {0: 215, 1: 221, 2: 188}
FLOPS_OTHER_MODE = 117


def flops_per_vstep(mode):
    """Mean counted flops per vehicle-step over a fleet's modes."""
    import numpy as np
    m = np.asarray(mode).astype(np.int64)
    f = np.full(m.shape, float(FLOPS_OTHER_MODE))
    for code, fl in FLOPS_BY_MODE.items():
        f[m == code] = fl
    return float(f.mean())


HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3         # MI355X published FP32 vector peak
# HBM bytes per dispatch from rocprofv3 FETCH_SIZE / WRITE_SIZE on the
# 1,048,576-quad workload, scaled by what the same counters read for a plain
# 512 MiB copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0): per-step kernel, and a
# fused launch of each fused form (exec kind 1: one block per tile; kind 2:
# work queues) at 20 steps (one load and one store of the state per launch,
# whatever k); VALU instructions per vehicle-step of each form (SQ_INSTS_VALU
# x 64 lanes / vehicles / steps) for 20-step and 512-step launches.  Valid
# only while the step-kernel sources hash to ``src``.
COUNTERS = {
    "src": "3b6bb056554e2e7b",
    "per_step_bytes": 127001805.0,
    "fused": {1: {"bytes": 131977216.0, "valu_per_vstep": {20: 151.2, 512: 140.0}},
              2: {"bytes": 151706829.0, "valu_per_vstep": {20: 147.1, 512: 139.8}}},
    "per_step_4M_bytes": 508684288.0,
    "profile": "profiles/fused_step_1M_quads.md",
}
FUSED_KERNELS = {1: "k_step fused (one block per tile)", 2: "k_step_q fused (work queues)"}


def fused_counters(kind):
    return COUNTERS["fused"].get(kind, {"bytes": None, "valu_per_vstep": {20: None, 512: None}})


def valu_per_vstep(kind, steps_per_launch):
    """Counted VALU instructions per vehicle-step of fused launches of this
    form and this many steps (the per-launch set-up spreads over fewer steps
    in short launches: the 20-step figure below 64 steps, the 512-step figure
    from there)."""
    v = fused_counters(kind)["valu_per_vstep"]
    return v[20] if steps_per_launch < 64 else v[512]


# The same for the rollout kernels of the 65,536-quad differentiation leg
# (200 steps per call): VALU instructions per vehicle-step (forward; adjoint
# counting its reverse and recompute wavefronts) and bytes per call.
ROLLOUT_COUNTERS = {
    "fwd_valu_per_vstep": 157.0,
    "adj_valu_per_vstep": 640.7,
    "fwd_bytes": 43080233.0,
    "adj_bytes": 1405851648.0,
    "profile": "profiles/rollout_65536_quads.md",
}
ROLLOUT_SOURCES = ("paper_2305_16510_amd/csrc/ag_step.h", "paper_2305_16510_amd/csrc/ag_rollout.hip",
                   "paper_2305_16510_amd/csrc/ag_internal.h")
ROLLOUT_SRC = "d7f2827642ee4154"
STEP_SOURCES = ("paper_2305_16510_amd/csrc/ag_step.h", "paper_2305_16510_amd/csrc/ag_kernels.hip",
                "paper_2305_16510_amd/csrc/ag_internal.h")
PAPER_VSTEPS = 3.8e6             # Sec. VI: 2^17 robots, attitude/velocity commands, RTX 3090


def step_source_hash(sources=None):
    import hashlib
    h = hashlib.sha256()
    for p in sources or STEP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def rollout_counters_valid():
    return ROLLOUT_SRC == step_source_hash(ROLLOUT_SOURCES)


def counters_valid():
    return COUNTERS["src"] == step_source_hash()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, sync):
    sync()
    t0 = time.perf_counter()
    fn()
    sync()
    return time.perf_counter() - t0


_EVENTS = []


def _events():
    """Two timing events, created and recorded once up front so that their
    first-use cost stays out of any timed region."""
    import torch
    if not _EVENTS:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        for e in ev:
            e.record()
        torch.cuda.synchronize()
        _EVENTS.extend(ev)
    return _EVENTS


def event_time(stream, fn):
    """Seconds between events recorded on `stream` around fn()'s launches."""
    e0, e1 = _events()
    e0.record(stream)
    fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3


def timed_with_events(stream, fn, sync):
    """(wall seconds, event seconds) of fn()'s launches: the wall clock runs
    from a device synchronisation before the launches to one after them, and
    events recorded on `stream` around the launches give the device time
    (read after the closing synchronisation).  The first event is recorded
    just before the wall clock starts, so that its host-side cost is not
    part of the timed work (the device interval then also holds the host's
    launch of the work, a conservative kernel time)."""
    e0, e1 = _events()
    sync()
    e0.record(stream)
    t0 = time.perf_counter()
    fn()
    e1.record(stream)
    sync()
    t = time.perf_counter() - t0
    return t, e0.elapsed_time(e1) / 1e3


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def time_oracle(sub, steps):
    import oracle
    s0, mode, tgt = oracle.step.from_workload_arrays(sub.state0, sub.mode, sub.target)
    fleet = oracle.Fleet.from_groups(sub.groups, sub.n, sub.vparams)
    t0 = time.perf_counter()
    oracle.step.rollout(s0, mode, tgt, fleet, sub.dt, sub.g, steps)
    return time.perf_counter() - t0


def cpu_baseline(wl, n_sample, steps):
    """The FP64 oracle, as it stands, on the host's cores: a slice of the
    benchmark workload, the same on one thread (smaller slice), and the
    1,024-quad 500-step position-mode parity workload."""
    import torch
    import workloads
    torch.set_num_threads(max(1, len(os.sched_getaffinity(0))))
    cores = torch.get_num_threads()
    dt = time_oracle(workloads.subset(wl, n_sample), steps)
    c1 = workloads.c1_parity()
    dt_c1 = time_oracle(c1, c1.steps)
    n1, s1 = max(1, n_sample // 8), max(1, steps // 3)
    torch.set_num_threads(1)
    dt1 = time_oracle(workloads.subset(wl, n1), s1)
    torch.set_num_threads(cores)
    return {"value": n_sample * steps / dt, "unit": "vehicle-steps/s", "cores": cores,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"first {n_sample} vehicles of the workload x {steps} steps (FP64 torch on CPU)",
            "seconds": dt,
            "parity_workload": {"value": c1.n * c1.steps / dt_c1, "cores": cores, "seconds": dt_c1,
                                "sample": f"{c1.n} quads x {c1.steps} steps, position mode, dt={c1.dt}"},
            "single_thread": {"value": n1 * s1 / dt1, "cores": 1,
                              "sample": f"first {n1} vehicles x {s1} steps", "seconds": dt1}}


def bench_adjoint(sync, reps=3):
    """Differentiation workload: 65,536 quads, 200-step position rollout,
    checkpoint every 20 steps; forward (with the batch loss) + hand-written
    adjoint."""
    import workloads
    from paper_2305_16510_amd.sim import Sim
    wl = workloads.c4_grad()
    T, m = wl.steps, wl.meta["ckpt_every"]
    sim = Sim.from_workload(wl)
    sim.rollout_forward(T, m, want_loss_i=False)
    sim.rollout_adjoint(T, m)
    sync()
    tf, ta = [], []
    for _ in range(reps):
        tf.append(event_time(sim.stream, lambda: sim.rollout_forward(T, m, want_loss_i=False)))
        ta.append(event_time(sim.stream, lambda: sim.rollout_adjoint(T, m)))
    sim.close()
    f, a = min(tf), min(ta)
    log(f"adjoint: forward {f * 1e3:.3f} ms, adjoint {a * 1e3:.3f} ms for {T} steps of {wl.n} vehicles")
    out = {"workload": "65,536 quads, 200-step position rollout, checkpoint every 20, 10 gain + 13 state "
                       "gradients per vehicle", "n_vehicles": wl.n, "steps": T,
           "forward_s_per_step": f / T, "adjoint_s_per_step": a / T, "fwd_plus_adj_s_per_step": (f + a) / T,
           "vehicle_steps_per_s_fwd_adj": wl.n * T / (f + a)}
    if rollout_counters_valid():
        # VALU issue against the chip's peak issue rate, and bytes moved per
        # second (the adjoint writes and reads back a 13-float state per
        # vehicle-step through its tape)
        peak_issue = FP32_PEAK_TFLOPS * 1e12 / 2
        rc = ROLLOUT_COUNTERS
        out["forward_valu_issue_frac_of_peak"] = rc["fwd_valu_per_vstep"] * wl.n * T / f / peak_issue
        out["adjoint_valu_issue_frac_of_peak"] = rc["adj_valu_per_vstep"] * wl.n * T / a / peak_issue
        out["adjoint_traffic_GBs"] = rc["adj_bytes"] / a / 1e9
        out["counters"] = rc["profile"]
    return out


def bench_uneven(sync):
    """48 groups (log-uniform sizes 512..131,072; 4/6/8 rotors; per-vehicle
    parameters), 2,000 steps in one autotuned graph-replayed rollout."""
    import workloads
    from paper_2305_16510_amd.sim import Sim
    wl = workloads.c3_uneven()
    sim = Sim.from_workload(wl, autotune_scratch=True)
    tuned = sim.autotune(512)
    sim.prepare(wl.steps)
    sim.raw_step(wl.steps)
    sync()
    t = timed(lambda: sim.raw_step(wl.steps), sync)
    sim.close()
    log(f"uneven groups: {wl.n} vehicles, {wl.n * wl.steps / t:.3e} vehicle-steps/s ({tuned})")
    return {"workload": "48 uneven groups, quad/hexa/octo, per-vehicle mass/inertia/gains, position mode",
            "n_vehicles": wl.n, "steps": wl.steps, "value": wl.n * wl.steps / t, "exec": tuned}


def bench_large(sync):
    """4,194,304 quads, 2,000 steps at dt = 0.005 with 1% counter-based resets
    per step (timed without observers, then again with the batch statistics,
    which count the resets), then a forward + adjoint gain-tuning pass (100
    steps) with one SGD step on the first 262,144 vehicles."""
    import torch
    import workloads
    from paper_2305_16510_amd.autograd import rollout_loss
    from paper_2305_16510_amd.sim import Sim
    wl = workloads.c5_large()
    torch.cuda.reset_peak_memory_stats()

    def run(stats):
        # the configuration's workload (resets, no observer), then the same
        # with the batch statistics bound (they count the resets)
        sim = Sim.from_workload(wl, auto_reset=True, collect_stats=stats, autotune_scratch=True)
        # trials of 64 steps: with automatic resets k goes up to 64, and the
        # autotuner tries no k above the trial length
        tuned = sim.autotune(64)
        sim.prepare(wl.steps)
        sync()
        t = timed(lambda: sim.raw_step(wl.steps), sync)
        st = sim.stats() if stats else None
        free, total = torch.cuda.mem_get_info()
        sim.close()
        return t, tuned, st, total - free

    t, tuned, _, used = run(False)
    t_st, tuned_st, st, used_st = run(True)
    peak = torch.cuda.max_memory_allocated()
    sub = workloads.subset(wl, wl.meta["tune_subset"])
    sub.vparams = workloads.per_vehicle_defaults(sub.n)
    ss = Sim.from_workload(sub)
    gains = ss.vparams[4:14].clone().requires_grad_(True)
    x0 = ss.state.clone()
    T = wl.meta["tune_steps"]

    def tune():
        loss = rollout_loss(ss, gains, x0, T, 20, 0.01)
        loss.backward()
        with torch.no_grad():
            gains.sub_(0.05 * gains.grad).clamp_(min=1e-3)
            gains.grad = None
        return loss

    tune()
    sync()
    tt = timed(tune, sync)
    ss.close()
    log(f"large: {wl.n * wl.steps / t:.3e} vehicle-steps/s with resets; {wl.n * wl.steps / t_st:.3e} with "
        f"statistics ({st['n_resets']} resets); tuning pass {tt * 1e3:.1f} ms; peak torch memory {peak / 2**20:.0f} MiB")
    return {"workload": "4,194,304 quads, 2,000 steps dt=0.005, 1% counter-based resets per step",
            "n_vehicles": wl.n, "steps": wl.steps, "value": wl.n * wl.steps / t, "exec": tuned,
            "with_statistics": {"value": wl.n * wl.steps / t_st, "exec": tuned_st,
                                "what": "the same run with the batch statistics bound (they count the resets)"},
            "resets": st["n_resets"], "expected_resets": 0.01 * wl.n * wl.steps,
            "peak_torch_allocated_bytes": peak, "device_used_bytes": max(used, used_st),
            "tuning_pass": {"n_vehicles": sub.n, "steps": T, "seconds": tt,
                            "what": "forward + adjoint + one SGD step on the 10 gains"}}


def bench_per_step_large(sync, steps=200):
    """Per-step kernel at 4,194,304 quads (position mode, dt = 0.005, no
    resets): 507 MB of state, commands and mode per step, twice the 256 MB
    Infinity Cache, so the bytes come from HBM."""
    import workloads
    from paper_2305_16510_amd.sim import Sim
    wl = workloads.c5_large()
    sim = Sim.from_workload(wl, reset_prob=0.0)
    best = None
    for blk in (64, 128, 256, 512):
        sim.set_exec(kind=0, block=blk, use_graph=0)
        sim.raw_step(10)
        sync()
        t = event_time(sim.stream, lambda: sim.raw_step(steps))
        if best is None or t < best[0]:
            best = (t, blk)
    sim.close()
    t, blk = best
    gbs = BYTES_PER_VSTEP * wl.n * steps / t / 1e9
    log(f"per-step at {wl.n}: {t / steps * 1e6:.1f} us per launch = {gbs:.0f} GB/s (block {blk})")
    return {"workload": "4,194,304 quads, position mode, dt=0.005, plain per-step launches",
            "n_vehicles": wl.n, "steps": steps, "block": blk, "kernel_avg_us": t / steps * 1e6,
            "value": wl.n * steps / t,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "traffic": COUNTERS["per_step_4M_bytes"] if counters_valid() else None,
                         "algorithmic_bytes": BYTES_PER_VSTEP * wl.n,
                         "note": "507 MB per launch, twice the 256 MB Infinity Cache: the bytes come from HBM"}}


def bench_camera(sync, n=1024, n_obs=20, W=480, H=270, reps=5):
    """Depth cameras: 2^10 vehicles with 270 x 480 images (the paper's camera
    benchmark shape, Sec. VI) in environments with 20 primitive obstacles
    placed by the reset randomisation."""
    import math
    import numpy as np
    import torch
    import workloads
    from paper_2305_16510_amd.sim import Sim
    wl = workloads.c1_parity(n=n, seed=90)
    wl.state0[0:3] = np.array([[0.5], [5.0], [1.5]], np.float32) + wl.state0[0:3] * 0.2
    sim = Sim.from_workload(wl)
    rng = np.random.default_rng(91)
    shapes = np.zeros((n_obs, 8), np.float32)
    shapes[:, 0] = np.arange(n_obs) % 3
    shapes[:, 1:4] = rng.uniform(0.2, 0.8, (n_obs, 3))
    slot = [0.55, 0.05, 0.1, 0.95, 0.95, 0.9, -1, -1, -math.pi, 1, 1, math.pi, 0, 0, 0, 0, 0, 0, 0, 0]
    slots = np.array([slot] * n_obs, np.float32)
    obst = torch.zeros(7, n * n_obs, device="cuda")
    obst[3] = 1.0
    sim.randomize_obstacles(slots, obst, step=1, box_lo=(0.0, 0.0, 0.0), box_hi=(10.0, 10.0, 3.0))
    out = torch.empty(n, H, W, device="cuda")
    sh = torch.as_tensor(shapes).cuda()
    sim.render_depth(sh, obst, W, H, 1.5, 10.0, floor_z=0.0, out=out)
    sync()
    ts = [event_time(sim.stream, lambda: sim.render_depth(sh, obst, W, H, 1.5, 10.0, floor_z=0.0, out=out))
          for _ in range(reps)]
    t_obs = event_time(sim.stream, lambda: sim.randomize_obstacles(slots, obst, step=2, box_lo=(0.0, 0.0, 0.0),
                                                                   box_hi=(10.0, 10.0, 3.0)))
    sim.close()
    t = min(ts)
    log(f"depth cameras: {n} x {W}x{H}, {n_obs} obstacles: {t * 1e3:.2f} ms per frame set = {n / t:.3e} images/s")
    return {"workload": f"{n} vehicles, {W}x{H} depth images, {n_obs} box/sphere/cylinder obstacles per env",
            "seconds_per_frame_set": t, "images_per_s": n / t, "rays_per_s": n * W * H / t,
            "obstacle_randomisation_s": t_obs,
            "paper_context": {"images_per_s": 1800, "hardware": "RTX 3090, engine renderer (Sec. VI)"}}


LEGS = {"adjoint": bench_adjoint, "uneven_groups": bench_uneven, "large_resets": bench_large,
        "per_step_4M": bench_per_step_large, "depth_cameras": bench_camera}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=1024)
    ap.add_argument("--n", type=int, default=1_048_576)
    ap.add_argument("--probe-steps", type=int, default=0,
                    help="steps per autotuning trial (also the largest k tried); 0: the timed call length")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-per-step", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--exec", type=str, default="",
                    help="fixed fused policy '[kind,]block,vpl,k,grid' (kind 1 if omitted; skips tuning)")
    ap.add_argument("--per-step-block", type=int, default=0, help="fixed block of the per-step kernel (skips its sweep)")
    ap.add_argument("--cpu-sample", type=int, default=65_536)
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--only", choices=sorted(LEGS), default="",
                    help="run one secondary leg alone and print its record (profiling runs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: vehicles are independent, so N GPUs would each run "
              "their own shard of the batch with no communication; run it once per GPU.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import bench_probe as probe
    from paper_2305_16510_amd.sim import Sim

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.only:
        rec = {args.only: LEGS[args.only](torch.cuda.synchronize)}
        if args.copy_calib_mib:
            probe.copy_once(args.copy_calib_mib << 20)
            rec["copy_calibration"] = {"kernel": "k_copy (agp_copy)", "bytes_read": args.copy_calib_mib << 20,
                                       "bytes_written": args.copy_calib_mib << 20, "dispatches": 3}
        print(json.dumps(rec), flush=True)
        return
    K, W = args.steps, args.warmup
    wl = workloads.c2_scale(n=args.n)
    log(f"workload {wl.name}: n={wl.n}")
    sim = Sim.from_workload(wl, autotune_scratch=True)
    sync = torch.cuda.synchronize
    # the timing events exist before any timed region, so that nothing but
    # the warm-up steps runs between the search and the timed call
    _events()
    if args.exec:
        f = [int(x) for x in args.exec.split(",")]
        kd, b, v, k, g = f if len(f) == 5 else [1] + f
        sim.set_exec(kind=kd, block=b, vpl=v, k=k, grid=g, use_graph=1)
        tuned = sim.get_exec()
    else:
        # the policy for calls of K steps, from trials of K-step calls
        t0 = time.perf_counter()
        tuned = sim.autotune(args.probe_steps or K)
        log(f"autotuned {tuned} for {args.probe_steps or K}-step calls in {time.perf_counter() - t0:.1f}s")
    k = tuned["k"]

    # ---- fused, graph-replayed ------------------------------------------------
    # ag_prepare builds and uploads the K-step graph (when K needs more than one
    # launch) and computes the mode order, so the timed call only launches
    sim.prepare(K)
    sim.prepare(W)
    sim.raw_step(W)
    sync()
    t_evt = {}
    t_fused, t_evt["fused"] = timed_with_events(sim.stream, lambda: sim.raw_step(K), sync)
    # the same K steps timed four more times (spread of the measurement)
    repeats = [timed(lambda: sim.raw_step(K), sync) for _ in range(4)]
    launches = math.ceil(K / k)
    kern_fused = t_evt["fused"] / launches
    value = wl.n * K / t_fused
    log(f"fused: {t_fused * 1e3:.3f} ms for {K} steps -> {value:.3e} vehicle-steps/s; "
        f"kernel avg {kern_fused * 1e6:.1f} us over {launches} launches")

    # ---- plain per-step launches ----------------------------------------------
    # K kernel launches without a graph, issued by the library's own launch
    # loop (ag_step(K) under the per-step policy); the same K steps as K host
    # calls of ag_step(1) are timed as well, where the host's per-call time
    # can leave the GPU idle between launches.  Timed right after the fused
    # call, each after its own short search (block sweep, autotune), so that
    # the GPU's clocks are in the same state for both (the 1,024-step leg's
    # search below keeps the GPU busy for about a second and raises them).
    per_step = None
    if not args.no_per_step:
        sweep = {}
        blocks = (args.per_step_block,) if args.per_step_block else (64, 128, 256, 512)
        for _ in range(2):                       # two interleaved passes, best of each block
            for blk in blocks:
                sim.set_exec(kind=0, block=blk, use_graph=0)
                sim.raw_step(20)
                sync()
                t = event_time(sim.stream, lambda: sim.raw_step(100)) / 100
                sweep[blk] = min(t, sweep.get(blk, t))
        best = min((t, blk) for blk, t in sweep.items())
        log("per-step block sweep (us): " + ", ".join(f"{b}: {t * 1e6:.2f}" for b, t in sweep.items()))
        sim.set_exec(kind=0, block=best[1], use_graph=0)
        sim.raw_step(W)
        sync()

        t_plain, t_evt["plain"] = timed_with_events(sim.stream, lambda: sim.raw_step(K), sync)
        kern_plain = t_evt["plain"] / K

        def run_calls():
            for _ in range(K):
                sim.raw_step(1)

        t_calls = timed(run_calls, sync)
        gbs = BYTES_PER_VSTEP * wl.n / kern_plain / 1e9
        per_step = {
            "value": wl.n * K / t_plain, "ms_per_step": t_plain / K * 1e3, "block": best[1],
            "block_sweep_us": {str(b): t * 1e6 for b, t in sweep.items()},
            "kernel_avg_us": kern_plain * 1e6,
            "host_calls": {"value": wl.n * K / t_calls, "ms_per_step": t_calls / K * 1e3,
                           "what": "K host calls of ag_step(1)"},
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "traffic": COUNTERS["per_step_bytes"] if counters_valid() else None,
                         "algorithmic_bytes": BYTES_PER_VSTEP * wl.n,
                         "note": "127 MB per launch fits the 256 MB Infinity Cache; per_step_4M is the HBM figure"},
        }
        log(f"per-step: {t_plain * 1e3:.2f} ms -> {per_step['value']:.3e} vehicle-steps/s, "
            f"kernel {kern_plain * 1e6:.1f} us = {gbs:.0f} GB/s; as host calls {t_calls * 1e3:.2f} ms")

    # ---- the profiled launch shape: 1,024 steps under the same policy --------
    # (outside the headline timing; with k = 512 these are two full launches,
    # the shape of the committed counter profile)
    fixed_steps = 1024
    if args.exec:
        sim.set_exec(**tuned)
        tuned_fixed = tuned
    else:
        tuned_fixed = sim.autotune(fixed_steps)
    k_fixed = tuned_fixed["k"]
    sim.prepare(fixed_steps)
    sim.raw_step(fixed_steps)
    sync()
    t_fix = min(event_time(sim.stream, lambda: sim.raw_step(fixed_steps)) for _ in range(3))
    fix_launches = math.ceil(fixed_steps / k_fixed)
    fix_tflops = FLOPS_PER_VSTEP * wl.n * fixed_steps / t_fix / 1e12
    fc_fixed = fused_counters(tuned_fixed["kind"])
    fix_valu = valu_per_vstep(tuned_fixed["kind"], min(fixed_steps, k_fixed)) if counters_valid() else None
    roofline_fixed = {"kernel": FUSED_KERNELS.get(tuned_fixed["kind"]),
                      "valu_instr_per_vehicle_step": fix_valu,
                      "valu_issue_frac_of_peak": (fix_valu * wl.n * fixed_steps / t_fix) / (FP32_PEAK_TFLOPS * 1e12 / 2)
                      if fix_valu else None,
                      "traffic": fc_fixed["bytes"] if counters_valid() else None,
                      "steps": fixed_steps, "exec": tuned_fixed, "launches": fix_launches,
                      "steps_per_launch": min(fixed_steps, k_fixed),
                      "kernel_avg_us": t_fix / fix_launches * 1e6, "us_per_step": t_fix / fixed_steps * 1e6,
                      "value": wl.n * fixed_steps / t_fix, "achieved": fix_tflops, "unit": "TFLOP/s",
                      "frac": fix_tflops / FP32_PEAK_TFLOPS,
                      "counted_frac": flops_per_vstep(wl.mode) * wl.n * fixed_steps / t_fix / 1e12 / FP32_PEAK_TFLOPS}
    log(f"fixed shape: {fixed_steps} steps in {fix_launches} launches, {t_fix / fixed_steps * 1e6:.2f} us/step, "
        f"frac {roofline_fixed['frac']:.3f}")

    # achieved = algorithmic flops of the timed launches / their event time
    # (the last launch of a K that k does not divide runs fewer steps)
    fl_count = flops_per_vstep(wl.mode)
    tflops = FLOPS_PER_VSTEP * wl.n * K / t_evt["fused"] / 1e12
    tflops_count = fl_count * wl.n * K / t_evt["fused"] / 1e12
    valid = counters_valid()
    # VALU utilisation: lane-instructions issued per second against the chip's
    # peak issue rate (157.3 TFLOP/s = 78.6e12 single-lane FMAs per second)
    valu_vstep = valu_per_vstep(tuned["kind"], min(K, k)) if valid else None
    valu_util = (valu_vstep * wl.n * K / t_evt["fused"]) / (FP32_PEAK_TFLOPS * 1e12 / 2) if valu_vstep else None
    out = {
        "metric": "vehicle-steps/s at 1M quads (fused vs per-step), %HBM/VALU peak; adjoint s/step",
        "value": value,
        "unit": "vehicle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": t_fused / K * 1e3,
        "repeat_ms_per_step": [t / K * 1e3 for t in repeats],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1,048,576 X-quads, modes uniform over position/velocity/attitude, "
                               "dt=0.01 s (seeded synthetic)", "n_vehicles": wl.n, "seq_len": 1,
                   "global_batch": wl.n, "parallelism": "none (1 GPU)", "exec": tuned},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP32_PEAK_TFLOPS,
                     # one load and one store of the state per launch, whatever k
                     "traffic": fused_counters(tuned["kind"])["bytes"] if valid else None,
                     "kernel": FUSED_KERNELS.get(tuned["kind"]), "kernel_avg_us": kern_fused * 1e6,
                     "launches": launches, "steps_per_launch": min(K, k),
                     "flops_per_vehicle_step": FLOPS_PER_VSTEP,
                     "counted": {"flops_per_vehicle_step": fl_count, "achieved": tflops_count,
                                 "frac": tflops_count / FP32_PEAK_TFLOPS,
                                 "what": "per-mode operation count of the fleet's modes (not the headline)"},
                     "valu_instr_per_vehicle_step": valu_vstep,
                     "valu_issue_frac_of_peak": valu_util,
                     "counters": COUNTERS["profile"] if valid else "stale: kernel changed since counters"},
        "roofline_fixed_shape": roofline_fixed,
        "per_step": per_step,
        "fused_over_per_step": (value / per_step["value"]) if per_step else None,
        "env": {"device": torch.cuda.get_device_name(0),
                "compute_units": torch.cuda.get_device_properties(0).multi_processor_count,
                "torch": torch.__version__, "hip": torch.version.hip, "clocks": "not locked"},
        "paper_context": {"value": PAPER_VSTEPS, "unit": "vehicle-steps/s",
                          "hardware": "2x RTX 3090 (use of the second GPU not stated)",
                          "workload": "2^17 robots, attitude/velocity commands (Sec. VI)"},
    }

    if not args.no_extras:
        wp = workloads.paper_context()
        sp = Sim.from_workload(wp, autotune_scratch=True)
        tuned_p = sp.autotune(args.probe_steps or K)
        sp.prepare(K)
        sp.raw_step(K)
        sync()
        tp = timed(lambda: sp.raw_step(K), sync)
        out["paper_shape"] = {"value": wp.n * K / tp, "n_vehicles": wp.n, "exec": tuned_p,
                              "workload": "2^17 quads, constant attitude or velocity commands, dt=0.01"}
        sp.close()
        log(f"paper shape 2^17: {wp.n * K / tp:.3e} vehicle-steps/s ({tuned_p})")
        out["adjoint"] = bench_adjoint(sync)
        out["uneven_groups"] = bench_uneven(sync)
        out["large_resets"] = bench_large(sync)
        out["per_step_4M"] = bench_per_step_large(sync)
        out["depth_cameras"] = bench_camera(sync)

    sim.close()
    del sim
    if args.copy_calib_mib:
        # a plain device copy of known size: calibrates the HBM byte counters
        nb = args.copy_calib_mib << 20
        probe.copy_once(nb)
        out["copy_calibration"] = {"kernel": "k_copy (agp_copy)", "bytes_read": nb, "bytes_written": nb,
                                   "dispatches": 3}
    if not args.no_extras:
        fma = probe.valu_fma_peak()
        cbw, by_grid = probe.copy_bandwidth()
        out["measured_peaks"] = {"fp32_fma_lane_ops_per_s": fma, "fp32_fma_tflops": 2 * fma / 1e12,
                                 "copy_GBs": cbw / 1e9,
                                 "copy_GBs_by_grid": {str(g): r / 1e9 for g, r in by_grid.items()}}
        out["roofline"]["frac_of_measured_peak"] = out["roofline"]["achieved"] / (2 * fma / 1e12)
        if valid:
            # VALU issue rate against the rate a pure-FMA probe kernel reaches
            issue = valu_vstep * wl.n * K / t_evt["fused"]
            out["roofline"]["valu_issue_frac_of_measured"] = issue / fma
        if per_step:
            per_step["roofline"]["frac_of_measured_copy"] = per_step["roofline"]["achieved"] / (cbw / 1e9)
        log(f"measured peaks: FP32 FMA {2 * fma / 1e12:.1f} TFLOP/s, copy {cbw / 1e9:.0f} GB/s")
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample, args.cpu_steps)
        log(f"oracle: {out['cpu_baseline']['value']:.3e} vehicle-steps/s on {out['cpu_baseline']['cores']} threads")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
