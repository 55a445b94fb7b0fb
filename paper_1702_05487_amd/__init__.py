"""RKL2 super-time-stepping for field-aligned thermal conduction on MI355X.

The compute path is the C-ABI library ``librkl.so`` (hand-written HIP kernels
for gfx950); ``paper_1702_05487_amd.rkl`` is its thin ctypes binding and
``paper_1702_05487_amd.inputs`` makes the seeded synthetic workloads.
Nothing is imported eagerly so that input generation never loads the GPU
library.
"""
__all__ = ["rkl", "inputs"]
