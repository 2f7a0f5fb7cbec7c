"""MI355X-native symmetric FMM gravity solve and HHS integrator.

Hot path (HIP, gfx950) behind the C ABI of include/fmm355.h; this package
holds the ctypes binding (``fmm``), the seeded workload generators
(``workloads``) and the build script (``build``).
"""
