"""MI355X-native neural-implicit-surface collision handling (arXiv 2110.01614).

The compute path is ``libsdfcollide.so`` (hand-written HIP for gfx950) behind
the C ABI in ``include/sdfcollide.h``; ``paper_2110_01614_amd.binding`` is its
ctypes binding (import it explicitly; it raises if the library is not built).
``paper_2110_01614_amd.inputs`` draws the seeded synthetic workloads.
"""
