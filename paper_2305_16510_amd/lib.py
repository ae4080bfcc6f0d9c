"""ctypes binding of include/ag.h (argument marshalling only)."""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libag.so")

STATE_DIM, TARGET_DIM, VPARAM_DIM, NGAINS, WRENCH_DIM, TRAJ_DIM = 13, 4, 16, 10, 8, 16
AG_OK, AG_E_INVALID, AG_E_HIP, AG_E_NOMEM, AG_E_STATE, AG_E_UNSUPPORTED = range(6)
FLAG_NONFINITE, FLAG_SATURATED, FLAG_RESET = 1, 2, 4

EXPORTS = [
    "ag_workspace_size", "ag_create", "ag_destroy", "ag_set_targets", "ag_step", "ag_prepare", "ag_set_exec",
    "ag_get_exec", "ag_autotune", "ag_reset", "ag_randomize_obstacles", "ag_render_depth", "ag_apply_actions", "ag_observe", "ag_get_stats", "ag_get_step", "ag_set_step",
    "ag_rollout_workspace_size", "ag_rollout_forward", "ag_rollout_adjoint", "ag_rollout_grad_noalloc", "ag_sync",
    "ag_last_error", "ag_status_string",
]


class GroupDesc(C.Structure):
    _fields_ = [("first", C.c_int64), ("count", C.c_int64), ("n_rotors", C.c_int32),
                ("arm", C.c_float), ("c_tau", C.c_float), ("u_min", C.c_float), ("u_max", C.c_float),
                ("mass", C.c_float), ("inertia", C.c_float * 3), ("gains", C.c_float * NGAINS)]


class Config(C.Structure):
    _fields_ = [("n", C.c_int64), ("ld", C.c_int64), ("dt", C.c_float), ("g", C.c_float),
                ("seed", C.c_uint64), ("index_base", C.c_int64), ("stream", C.c_void_p),
                ("n_groups", C.c_int32), ("groups", C.POINTER(GroupDesc)),
                ("state", C.c_void_p), ("mode", C.c_void_p), ("target", C.c_void_p),
                ("vparams", C.c_void_p), ("wrench_out", C.c_void_p), ("rotor_out", C.c_void_p),
                ("flags_out", C.c_void_p), ("reset_prob", C.c_float), ("auto_reset", C.c_int32),
                ("reset_lo", C.c_float * 3), ("reset_hi", C.c_float * 3),
                ("collect_stats", C.c_int32), ("autotune_scratch", C.c_int32), ("traj", C.c_void_p),
                ("goal", C.c_void_p)]


class Exec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("block", C.c_int32), ("vpl", C.c_int32), ("k", C.c_int32),
                ("grid", C.c_int32), ("use_graph", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Task(C.Structure):
    _fields_ = [("w_v", C.c_float), ("w_omega", C.c_float), ("bonus", C.c_float), ("r_goal", C.c_float),
                ("r_far", C.c_float), ("max_steps", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("n_saturated", C.c_int64), ("n_resets", C.c_int64),
                ("n_invalid_mode", C.c_int64), ("n_nonfinite", C.c_int64), ("n_finite", C.c_int64),
                ("n_position", C.c_int64), ("pos_err_sum", C.c_double), ("omega_sum", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Load libag.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or paper_2305_16510_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    P = C.c_void_p
    sig = {
        "ag_workspace_size": ([C.POINTER(Config), C.POINTER(C.c_size_t)], C.c_int),
        "ag_create": ([C.POINTER(Config), P, C.c_size_t, C.POINTER(H)], C.c_int),
        "ag_destroy": ([H], C.c_int),
        "ag_set_targets": ([H, C.c_int64, C.c_int64, P, P, C.c_int64], C.c_int),
        "ag_step": ([H, C.c_int32], C.c_int),
        "ag_prepare": ([H, C.c_int32], C.c_int),
        "ag_set_exec": ([H, C.POINTER(Exec)], C.c_int),
        "ag_get_exec": ([H, C.POINTER(Exec)], C.c_int),
        "ag_autotune": ([H, C.c_int32, C.POINTER(Exec)], C.c_int),
        "ag_reset": ([H, P, C.c_int64, P, P, P], C.c_int),
        "ag_randomize_obstacles": ([H, C.c_int32, P, P, P, C.POINTER(C.c_float), C.POINTER(C.c_float), P,
                                    C.c_int64, P, C.c_int64], C.c_int),
        "ag_render_depth": ([H, C.POINTER(Camera), C.c_int32, P, P, C.c_int64, C.c_int64, C.c_int64, P], C.c_int),
        "ag_apply_actions": ([H, P, C.c_int64, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float)], C.c_int),
        "ag_observe": ([H, C.POINTER(Task), C.c_int32, P, C.c_int64, P, P, P], C.c_int),
        "ag_get_stats": ([H, C.POINTER(Stats), C.c_int32], C.c_int),
        "ag_get_step": ([H, C.POINTER(C.c_int64)], C.c_int),
        "ag_set_step": ([H, C.c_int64], C.c_int),
        "ag_rollout_workspace_size": ([H, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)], C.c_int),
        "ag_rollout_forward": ([H, P, P, C.c_int32, C.c_int32, C.c_float, P, C.c_size_t, P, P, P], C.c_int),
        "ag_rollout_adjoint": ([H, P, P, C.c_int32, C.c_int32, C.c_float, C.c_float, P, P, C.c_size_t, P, P],
                               C.c_int),
        "ag_rollout_grad_noalloc": ([H, P, P, C.c_int32, C.c_int32, C.c_float, C.c_float, P, P, P, P], C.c_int),
        "ag_sync": ([H], C.c_int),
        "ag_last_error": ([H], C.c_char_p),
        "ag_status_string": ([C.c_int], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


class AgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status, handle=None, what=""):
    if status != AG_OK:
        L = load()
        detail = L.ag_last_error(handle).decode() if handle else L.ag_status_string(status).decode()
        raise AgError(status, f"{what}: {detail}")


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("hfov", C.c_float), ("max_depth", C.c_float),
                ("floor_z", C.c_float), ("mount_pos", C.c_float * 3), ("mount_quat", C.c_float * 4)]
