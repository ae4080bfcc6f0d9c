"""MI355X-native batched multirotor step (arXiv 2305.16510, Sec. IV).

The compute path is the HIP library ``_lib/libag.so`` (kernels under
``csrc/``) behind the C ABI of ``include/ag.h``.  ``lib`` marshals arguments
through ctypes; ``sim.Sim`` owns torch device buffers for one batch of
vehicles; ``autograd.RolloutFn`` exposes the hand-written adjoint.  There is
no CPU fallback: loading fails loudly when the library has not been built.
"""
__all__ = ["lib", "sim", "autograd", "build"]
