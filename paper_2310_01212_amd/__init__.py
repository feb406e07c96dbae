"""LightKernel persistent-thread dispatch for AMD Instinct MI355X (gfx950).

The native library (liblk.so: HIP kernels and the C ABI of include/lk.h) is loaded
lazily by :mod:`paper_2310_01212_amd.lk`; :mod:`paper_2310_01212_amd.workloads` only
draws seeded synthetic inputs.
"""
