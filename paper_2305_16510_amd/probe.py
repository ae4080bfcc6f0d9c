"""Calibration probes (include/ag_probe.h): measured FP32 FMA and copy peaks."""
import ctypes as C
import os

import torch

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libagprobe.so")
_lib = None


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
    L = load()
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    for _ in range(3):
        L.agp_copy(C.c_void_p(s.cuda_stream), C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes, 2048)
    torch.cuda.synchronize()
