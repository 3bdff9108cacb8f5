"""MI355X-native FMM-ForceAtlas2 / Kamada-Kawai graph layout (gfx950 HIP).

The compute path lives in ``libfa2lay.so`` (hand-written HIP kernels behind a
C ABI, declared in ``include/fa2lay.h``); ``paper_2403_03504_amd.fa2lay`` is the
thin Python binding.  Submodules are imported lazily so that the seeded
workload generators can be used without loading the GPU library.
"""
__all__ = ["workloads", "fa2lay"]
