"""MI355X-native exact ddKS (arXiv:2106.13706): the O(2^d N^2) orthant-counting
sweep as hand-written HIP for gfx950 behind a C ABI (libddks.so).

Submodules: ``native`` (ctypes binding of libddks.so; raises if the library
is missing) and ``workloads`` (seeded input generators).  Neither is
imported here, so the generators can be used without the native library.
"""
