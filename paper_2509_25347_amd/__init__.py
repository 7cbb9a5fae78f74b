"""MI355X-native drag update v(t+dt) = exp(dt K) v (arXiv:2509.25347).

Hand-written HIP kernels for gfx950 behind a C ABI (``include/dragexp.h``);
this package holds the thin Python binding and the seeded workload
generators.
"""
