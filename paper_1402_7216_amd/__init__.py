"""MI355X-native multilevel summation method (MSM) electrostatics.

The compute path is the HIP library ``libmsm.so`` (hand-written gfx950
kernels behind a C ABI, declared in ``include/msm.h``).  ``paper_1402_7216_amd.msm``
binds it with ctypes; PyTorch supplies device memory and the stream.
Submodules are imported lazily so that ``inputs`` and ``workmodel`` load
without a GPU.
"""
__all__ = ["inputs", "workmodel", "msm"]
