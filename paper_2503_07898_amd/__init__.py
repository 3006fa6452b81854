"""MI355X-native D3Q19 lattice-Boltzmann hot path in a disaggregated layout.

The compute runs in liblbm.so (hand-written HIP kernels for gfx950 behind a
C ABI, declared in include/lbm.h).  This package holds the ctypes binding
(`lbm`), the seeded synthetic workload generators (`workloads`) and the
build script (`build`).
"""
