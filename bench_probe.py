"""Calibration probes of the benchmark (kernels in bench_probe.hip): the
measured FP32 FMA issue rate and device copy bandwidth, and a plain copy of
known size for calibrating the HBM byte counters.  Not part of the library."""
import ctypes as C
import os
import subprocess

ROOT = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(ROOT, "bench_probe.hip")
PATH = os.path.join(ROOT, "_probe", "libagprobe.so")
_lib = None


def build():
    """Compile bench_probe.hip for gfx950 into _probe/libagprobe.so."""
    from paper_2305_16510_amd.build import HIP_FLAGS, hipcc
    os.makedirs(os.path.dirname(PATH), exist_ok=True)
    tmp = PATH + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, "-shared", SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, PATH)
    return PATH


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(PATH):
            raise RuntimeError(f"probe library not built: {PATH}")
        _lib = C.CDLL(PATH)
        _lib.agp_valu_fma.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]
        _lib.agp_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32]
    return _lib


def _time(stream, fn, reps=5):
    import torch
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        best = t if best is None else min(best, t)
    return best


def valu_fma_peak(blocks=4096, iters=4096):
    """Measured FP32 FMA lane-operations per second (non-packed v_fma_f32)."""
    import torch
    L = load()
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    run = lambda: L.agp_valu_fma(C.c_void_p(s.cuda_stream), C.c_void_p(out.data_ptr()), blocks, iters)
    run()
    t = _time(s, run)
    return blocks * 256 * iters * 8 / t


def copy_bandwidth(nbytes=1 << 30, grids=(0, 2048, 8192, 32768)):
    """Measured device copy bandwidth (bytes read + written per second): the
    best of plain copies with one lane per 16-byte element (grid 0) and
    grid-stride copies of the given block counts; also returns the rate of
    each grid."""
    import torch
    L = load()
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    rates = {}
    for g in grids:
        run = lambda: L.agp_copy(C.c_void_p(s.cuda_stream), C.c_void_p(dst.data_ptr()),
                                 C.c_void_p(src.data_ptr()), nbytes, g)
        run()
        rates[g] = 2 * nbytes / _time(s, run)
    return max(rates.values()), rates


def copy_once(nbytes):
    """One plain copy of nbytes (for counter calibration runs)."""
    import torch
    L = load()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    for _ in range(3):
        L.agp_copy(C.c_void_p(s.cuda_stream), C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes, 2048)
    torch.cuda.synchronize()
