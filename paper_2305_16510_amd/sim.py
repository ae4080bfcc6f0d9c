"""A batch of simulated multirotors on one GPU, driven through the C ABI.

PyTorch supplies the device buffers (state, commands, parameters, outputs,
workspaces) and the stream; every step of the method runs in the HIP
kernels of ``libag.so``.
"""
import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import lib as L

F32 = torch.float32


@dataclass
class Group:
    """A contiguous range of vehicles sharing a rotor layout and default
    parameters (the defaults: an X-quadrotor of 1 kg with a 0.13 m arm)."""
    first: int
    count: int
    n_rotors: int = 4
    arm: float = 0.13
    c_tau: float = 0.016
    u_min: float = 0.0
    u_max: float = 6.0
    mass: float = 1.0
    inertia: tuple = (0.007, 0.007, 0.012)
    gains: tuple = (2.0, 2.0, 2.0, 2.0, 1.6, 1.6, 0.6, 0.5, 0.5, 0.2)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _group_array(groups):
    arr = (L.GroupDesc * len(groups))()
    for k, gr in enumerate(groups):
        d = arr[k]
        d.first, d.count, d.n_rotors = int(gr.first), int(gr.count), int(gr.n_rotors)
        d.arm, d.c_tau, d.u_min, d.u_max = gr.arm, gr.c_tau, gr.u_min, gr.u_max
        d.mass = gr.mass
        for j in range(3):
            d.inertia[j] = gr.inertia[j]
        for j in range(L.NGAINS):
            d.gains[j] = gr.gains[j]
    return arr


def _dev(x, dtype, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=device, dtype=dtype).contiguous()


class Sim:
    """Owns device buffers for n vehicles and one library handle.

    Arrays are structure-of-arrays with leading dimension n: state [13, n],
    target [4, n], mode [n] (int8), vparams [16, n] or None, traj [16, n]
    (tracking-mode trajectory rows) or None.
    """

    def __init__(self, groups, state0, mode, target, vparams=None, *, dt=0.01, g=9.81, seed=0,
                 index_base=0, reset_prob=0.0, auto_reset=False, reset_lo=(-5.0, -5.0, -5.0),
                 reset_hi=(5.0, 5.0, 5.0), collect_stats=False, outputs=False,
                 autotune_scratch=False, traj=None, goal=None, device="cuda:0"):
        self._lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required (no CPU fallback)")
        self.device = torch.device(device)
        self.state = _dev(state0, F32, self.device)
        self.n = int(self.state.shape[1])
        self.mode = _dev(mode, torch.int8, self.device)
        self.target = _dev(target, F32, self.device)
        self.vparams = None if vparams is None else _dev(vparams, F32, self.device)
        if self.state.shape != (L.STATE_DIM, self.n) or self.target.shape != (L.TARGET_DIM, self.n) \
                or self.mode.shape != (self.n,):
            raise ValueError("state [13,n], target [4,n], mode [n] expected")
        if self.vparams is not None and self.vparams.shape != (L.VPARAM_DIM, self.n):
            raise ValueError("vparams [16,n] expected")
        self.traj = None if traj is None else _dev(traj, F32, self.device)
        if self.traj is not None and self.traj.shape != (L.TRAJ_DIM, self.n):
            raise ValueError("traj [16,n] expected")
        self.goal = None if goal is None else _dev(goal, F32, self.device)
        if self.goal is not None and self.goal.shape != (3, self.n):
            raise ValueError("goal [3,n] expected")
        self.wrench = self.rotors = self.flags = None
        if outputs:
            self.wrench = torch.zeros(L.WRENCH_DIM, self.n, dtype=F32, device=self.device)
            self.rotors = torch.zeros(8, self.n, dtype=F32, device=self.device)
            self.flags = torch.zeros(self.n, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.groups = list(groups)
        self._garr = _group_array(self.groups)
        cfg = L.Config()
        cfg.n, cfg.ld, cfg.dt, cfg.g = self.n, self.n, dt, g
        cfg.seed, cfg.index_base = int(seed), int(index_base)
        cfg.stream = C.c_void_p(self.stream.cuda_stream)
        cfg.n_groups = len(self.groups)
        cfg.groups = self._garr
        cfg.state, cfg.mode, cfg.target = _ptr(self.state), _ptr(self.mode), _ptr(self.target)
        cfg.vparams = _ptr(self.vparams)
        cfg.wrench_out, cfg.rotor_out, cfg.flags_out = _ptr(self.wrench), _ptr(self.rotors), _ptr(self.flags)
        cfg.reset_prob, cfg.auto_reset = float(reset_prob), int(bool(auto_reset))
        for j in range(3):
            cfg.reset_lo[j], cfg.reset_hi[j] = reset_lo[j], reset_hi[j]
        cfg.collect_stats = int(bool(collect_stats))
        cfg.autotune_scratch = int(bool(autotune_scratch))
        cfg.traj = _ptr(self.traj)
        cfg.goal = _ptr(self.goal)
        self._cfg = cfg
        nbytes = C.c_size_t(0)
        L.check(self._lib.ag_workspace_size(C.byref(cfg), C.byref(nbytes)), None, "ag_workspace_size")
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        h = C.c_void_p()
        L.check(self._lib.ag_create(C.byref(cfg), _ptr(self.workspace), C.c_size_t(self.workspace.numel()),
                                    C.byref(h)), None, "ag_create")
        self.h = h
        self._rollout_ws = None

    @classmethod
    def from_workload(cls, wl, **kw):
        kw.setdefault("dt", wl.dt)
        kw.setdefault("g", wl.g)
        kw.setdefault("seed", wl.seed)
        kw.setdefault("reset_prob", wl.reset_prob)
        kw.setdefault("reset_lo", wl.reset_lo)
        kw.setdefault("reset_hi", wl.reset_hi)
        return cls(wl.groups, wl.state0, wl.mode, wl.target, wl.vparams, **kw)

    # ---- plumbing -----------------------------------------------------------
    def _call(self, name, *args):
        # Order the library's stream after torch's current stream and back, so
        # tensors read or written by torch around a call see its results.
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        L.check(getattr(self._lib, name)(self.h, *args), self.h, name)
        cur.wait_stream(self.stream)

    def raw_step(self, n_steps=1):
        """ag_step without stream ordering (timing loops; caller synchronises)."""
        L.check(self._lib.ag_step(self.h, int(n_steps)), self.h, "ag_step")

    def sync(self):
        L.check(self._lib.ag_sync(self.h), self.h, "ag_sync")

    def close(self):
        if getattr(self, "h", None):
            self._lib.ag_sync(self.h)
            self._lib.ag_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- API ----------------------------------------------------------------
    def step(self, n_steps=1):
        self._call("ag_step", C.c_int32(int(n_steps)))

    def prepare(self, n_steps):
        """Build the graph ag_step(n_steps) will replay, without launching it."""
        self._call("ag_prepare", C.c_int32(int(n_steps)))

    def set_exec(self, kind=1, block=256, vpl=1, k=16, grid=0, use_graph=1):
        e = L.Exec(int(kind), int(block), int(vpl), int(k), int(grid), int(use_graph))
        self._call("ag_set_exec", C.byref(e))

    def get_exec(self):
        e = L.Exec()
        L.check(self._lib.ag_get_exec(self.h, C.byref(e)), self.h, "ag_get_exec")
        return e.as_dict()

    def autotune(self, probe_steps=64):
        e = L.Exec()
        self._call("ag_autotune", C.c_int32(int(probe_steps)), C.byref(e))
        return e.as_dict()

    def set_targets(self, first, count, mode=None, target=None):
        m = None if mode is None else _dev(mode, torch.int8, self.device)
        t = None if target is None else _dev(target, F32, self.device)
        ld = 0 if t is None else int(t.shape[1])
        self._call("ag_set_targets", C.c_int64(first), C.c_int64(count), _ptr(m), _ptr(t), C.c_int64(ld))
        self._keep = (m, t)

    def reset(self, step, mask=None, want_indices=True):
        """Reset before global step ``step``; returns (mask uint8 [n], indices int32
        [count]) after synchronising, or None when want_indices is False."""
        m_in = None if mask is None else _dev(mask, torch.uint8, self.device)
        if not want_indices:
            self._call("ag_reset", _ptr(m_in), C.c_int64(int(step)), C.c_void_p(0), C.c_void_p(0),
                       C.c_void_p(0))
            return None
        m_out = torch.empty(self.n, dtype=torch.uint8, device=self.device)
        idx = torch.empty(self.n, dtype=torch.int32, device=self.device)
        cnt = torch.empty(1, dtype=torch.int32, device=self.device)
        self._call("ag_reset", _ptr(m_in), C.c_int64(int(step)), _ptr(m_out), _ptr(idx), _ptr(cnt))
        self.sync()
        return m_out, idx[: int(cnt.item())]

    def randomize_obstacles(self, slots, out, step, mask=None, env_lo=None, env_hi=None, box_lo=None,
                            box_hi=None):
        """Redraw obstacle poses (rows x, y, z, qw, qx, qy, qz of ``out`` [7, >= n*n_obs])
        of the environments in ``mask`` (all when None); slots [n_obs, 20]."""
        sl = _dev(slots, F32, self.device)
        m = None if mask is None else _dev(mask, torch.uint8, self.device)
        lo = None if env_lo is None else _dev(env_lo, F32, self.device)
        hi = None if env_hi is None else _dev(env_hi, F32, self.device)
        blo = None if box_lo is None else (C.c_float * 3)(*box_lo)
        bhi = None if box_hi is None else (C.c_float * 3)(*box_hi)
        self._call("ag_randomize_obstacles", C.c_int32(int(sl.shape[0])), _ptr(sl), _ptr(lo), _ptr(hi), blo, bhi,
                   _ptr(m), C.c_int64(int(step)), _ptr(out), C.c_int64(int(out.shape[1])))
        self._keep = (sl, m, lo, hi)

    def render_depth(self, shapes, obst, width, height, hfov, max_depth, floor_z=float("nan"),
                     mount_pos=(0.0, 0.0, 0.0), mount_quat=(1.0, 0.0, 0.0, 0.0), first=0, count=None, out=None):
        """Depth images [count, height, width] of vehicles [first, first+count)."""
        count = self.n - first if count is None else count
        cam = L.Camera(int(width), int(height), float(hfov), float(max_depth), float(floor_z),
                       (C.c_float * 3)(*mount_pos), (C.c_float * 4)(*mount_quat))
        sh = None if shapes is None else _dev(shapes, F32, self.device)
        n_obs = 0 if sh is None else int(sh.shape[0])
        if out is None:
            out = torch.empty(count, height, width, dtype=F32, device=self.device)
        self._call("ag_render_depth", C.byref(cam), C.c_int32(n_obs), _ptr(sh), _ptr(obst),
                   C.c_int64(0 if obst is None else int(obst.shape[1])), C.c_int64(first), C.c_int64(count),
                   _ptr(out))
        self._keep = (sh,)
        return out

    def apply_actions(self, actions, mode, scale, offset):
        """Commands target = offset + scale * clamp(actions, -1, 1) for all vehicles (actions [4, n])."""
        act = _dev(actions, F32, self.device)
        self._call("ag_apply_actions", _ptr(act), C.c_int64(int(act.shape[1])), C.c_int32(int(mode)),
                   (C.c_float * 4)(*scale), (C.c_float * 4)(*offset))
        self._keep = (act,)

    def observe(self, task, obs, reward=None, done=None, episode=None, advance=True):
        """Goal-reaching observation [13, n], reward [n], done [n] (uint8), episode counters [n] (int32)."""
        self._call("ag_observe", C.byref(task), C.c_int32(int(bool(advance))), _ptr(obs),
                   C.c_int64(int(obs.shape[1])), _ptr(reward), _ptr(done), _ptr(episode))

    def stats(self, clear=False):
        s = L.Stats()
        self._call("ag_get_stats", C.byref(s), C.c_int32(int(bool(clear))))
        return s.as_dict()

    @property
    def step_counter(self):
        v = C.c_int64()
        L.check(self._lib.ag_get_step(self.h, C.byref(v)), self.h, "ag_get_step")
        return int(v.value)

    def set_step_counter(self, t):
        self._call("ag_set_step", C.c_int64(int(t)))

    # ---- differentiable rollout ---------------------------------------------
    def rollout_workspace_bytes(self, n_steps, ckpt_every):
        nbytes = C.c_size_t(0)
        L.check(self._lib.ag_rollout_workspace_size(self.h, int(n_steps), int(ckpt_every), C.byref(nbytes)),
                self.h, "ag_rollout_workspace_size")
        return max(int(nbytes.value), 256)

    def new_rollout_workspace(self, n_steps, ckpt_every):
        """A fresh rollout workspace (checkpoints, tapes, loss partials)."""
        return torch.empty(self.rollout_workspace_bytes(n_steps, ckpt_every), dtype=torch.uint8,
                           device=self.device)

    def rollout_workspace(self, n_steps, ckpt_every):
        """The Sim's shared rollout workspace, grown as needed (for paired
        rollout_forward / rollout_adjoint calls with no other rollout between)."""
        need = self.rollout_workspace_bytes(n_steps, ckpt_every)
        if self._rollout_ws is None or self._rollout_ws.numel() < need:
            self._rollout_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._rollout_ws

    def rollout_forward(self, n_steps, ckpt_every, w_omega=0.01, x0=None, want_final=False, gains=None,
                        ws=None, want_loss_i=True):
        """Per-vehicle loss [n] (or None), batch loss (device [1]) and final state
        [13, n] (or None) of the rollout; checkpoints go to ``ws`` (default: the
        shared workspace)."""
        ws = self.rollout_workspace(n_steps, ckpt_every) if ws is None else ws
        loss = torch.empty(self.n, dtype=F32, device=self.device) if want_loss_i else None
        batch = torch.empty(1, dtype=F32, device=self.device)
        final = torch.empty(L.STATE_DIM, self.n, dtype=F32, device=self.device) if want_final else None
        self._call("ag_rollout_forward", _ptr(x0), _ptr(gains), C.c_int32(int(n_steps)), C.c_int32(int(ckpt_every)),
                   C.c_float(w_omega), _ptr(ws), C.c_size_t(ws.numel()), _ptr(loss), _ptr(batch), _ptr(final))
        return loss, batch, final

    def rollout_adjoint(self, n_steps, ckpt_every, w_omega=0.01, seed_grad=1.0, x0=None, gains=None, ws=None,
                        seed_dev=None):
        """dL/dgains [10, n] and dL/dx0 [13, n] times seed_grad (and times the
        device scalar ``seed_dev`` when given)."""
        ws = self.rollout_workspace(n_steps, ckpt_every) if ws is None else ws
        dg = torch.empty(L.NGAINS, self.n, dtype=F32, device=self.device)
        dx = torch.empty(L.STATE_DIM, self.n, dtype=F32, device=self.device)
        self._call("ag_rollout_adjoint", _ptr(x0), _ptr(gains), C.c_int32(int(n_steps)), C.c_int32(int(ckpt_every)),
                   C.c_float(w_omega), C.c_float(seed_grad), _ptr(seed_dev), _ptr(ws), C.c_size_t(ws.numel()),
                   _ptr(dg), _ptr(dx))
        return dg, dx

    def rollout_grad_noalloc(self, n_steps, ckpt_every, w_omega=0.01, seed_grad=1.0, x0=None, gains=None,
                             out=None):
        """Forward and adjoint in one call on the library's static scratch (no
        device allocation by the library).  ``out``: optional preallocated
        (loss [n], batch [1], dgains [10, n], dx0 [13, n]) tensors."""
        if out is None:
            out = (torch.empty(self.n, dtype=F32, device=self.device), torch.empty(1, dtype=F32, device=self.device),
                   torch.empty(L.NGAINS, self.n, dtype=F32, device=self.device),
                   torch.empty(L.STATE_DIM, self.n, dtype=F32, device=self.device))
        loss, batch, dg, dx = out
        self._call("ag_rollout_grad_noalloc", _ptr(x0), _ptr(gains), C.c_int32(int(n_steps)),
                   C.c_int32(int(ckpt_every)), C.c_float(w_omega), C.c_float(seed_grad), _ptr(loss), _ptr(batch),
                   _ptr(dg), _ptr(dx))
        return loss, batch, dg, dx
