"""MI355X-native exact ddKS (arXiv:2106.13706): the O(2^d N^2) orthant-counting
sweep as hand-written HIP for gfx950 behind a C ABI (libddks.so).

The Python binding lives in ``paper_2106_13706_amd.native``; it is imported
lazily so that ``workloads`` (seeded input generators) can be used without
the native library.
"""
__all__ = ["native", "workloads"]


def __getattr__(name):
    if name == "native":
        from . import native as _n
        return _n
    if name == "workloads":
        from . import workloads as _w
        return _w
    raise AttributeError(name)
