"""ctypes binding of libddks.so (include/ddks.h): argument marshalling only.

Every computation runs in the library's gfx950 kernels.  There is no CPU
fallback: if libddks.so is missing or no gfx950 device is present the calls
raise.  Inputs may be numpy arrays (host memory) or torch tensors on the
context's device (passed as device pointers).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddks.so")

DDKS_OK = 0
DDKS_E_INVALID_ARG = -1
DDKS_E_NO_DEVICE = -2
DDKS_E_DEVICE = -3
DDKS_E_NOMEM = -4
DDKS_E_NONFINITE = -5
DDKS_E_AGAIN = -6
DDKS_E_PENDING = -7
DDKS_E_UNKNOWN_TICKET = -8
DDKS_E_NOT_SUPPORTED = -9

DDKS_DEVICE_PTRS = 0x1
DDKS_FORCE_F32 = 0x2
DDKS_NO_AUTOTUNE = 0x4
DDKS_PROFILE_KERNELS = 0x8
DDKS_FORCE_RANK16 = 0x10
DDKS_WITH_SIGNIFICANCE = 0x20
DDKS_SIG_POISSON = 0x40

# Every symbol include/ddks.h declares.
EXPORTS = (
    "ddks_default_options", "ddks_create", "ddks_destroy", "ddks_distance",
    "ddks_permutation_batch", "ddks_significance", "ddks_serve_submit", "ddks_serve_poll",
    "ddks_serve_stats_get", "ddks_profile_get", "ddks_status_string", "ddks_last_error",
    "ddks_version", "ddks_vdks", "ddks_rdks", "ddks_distance_noalloc", "ddks_perm_summary_of",
)


class DDKSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("mem_budget", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("serve_streams", ctypes.c_int32), ("serve_queue_depth", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]


class _Result(ctypes.Structure):
    _fields_ = [("num", ctypes.c_uint64), ("den", ctypes.c_uint64), ("D", ctypes.c_double),
                ("argmax_origin", ctypes.c_int64), ("argmax_orthant", ctypes.c_int32),
                ("d", ctypes.c_int32), ("n_p", ctypes.c_int64), ("n_q", ctypes.c_int64),
                ("S", ctypes.c_double)]


class _Request(ctypes.Structure):
    _fields_ = [("P", ctypes.c_void_p), ("n_p", ctypes.c_int64), ("Q", ctypes.c_void_p),
                ("n_q", ctypes.c_int64), ("d", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class _ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected_again", ctypes.c_uint64), ("rejected_nomem", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("p50_latency_us", ctypes.c_double),
                ("p99_latency_us", ctypes.c_double), ("mean_batch", ctypes.c_double),
                ("resident_bytes", ctypes.c_uint64), ("busy_us", ctypes.c_double),
                ("shifted_tests", ctypes.c_uint64)]


class _PermSummary(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int64), ("n_ge", ctypes.c_uint64), ("p_value", ctypes.c_double),
                ("fraction", ctypes.c_double)]


class _Profile(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_uint64), ("sweep_ms", ctypes.c_double),
                ("score_ms", ctypes.c_double), ("batch_ms", ctypes.c_double),
                ("compares", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("graph_calls", ctypes.c_uint64), ("shifted_calls", ctypes.c_uint64)]


@dataclass
class Result:
    num: int
    den: int
    D: float
    argmax_origin: int
    argmax_orthant: int
    d: int
    n_p: int
    n_q: int
    S: float = -1.0  # analytic significance when asked for (DDKS_WITH_SIGNIFICANCE)

    @classmethod
    def _from(cls, r: _Result) -> "Result":
        return cls(r.num, r.den, r.D, r.argmax_origin, r.argmax_orthant, r.d, r.n_p, r.n_q, r.S)


_lib = None


def load(path: str = LIB_PATH):
    """Loads libddks.so and declares its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libddks.so not found at {path}; build it with "
                          "python -m paper_2106_13706_amd.build (or __graft_entry__.build())")
    # torch ships its own HIP runtime (same sonames as /opt/rocm's).  Loading it
    # first makes libddks bind to that one copy, so torch and libddks share a
    # single HIP runtime in the process; two runtimes cannot both open the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i64, i32, u32, u64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                              ctypes.c_uint64)
    lib.ddks_default_options.argtypes = [ctypes.POINTER(_Options)]
    lib.ddks_default_options.restype = None
    lib.ddks_create.argtypes = [ctypes.POINTER(_Options), ctypes.POINTER(vp)]
    lib.ddks_destroy.argtypes = [vp]
    lib.ddks_distance.argtypes = [vp, vp, i64, vp, i64, i32, u32, ctypes.POINTER(_Result), vp]
    lib.ddks_distance_noalloc.argtypes = [vp, vp, i64, vp, i64, i32, u32, ctypes.POINTER(_Result), vp]
    lib.ddks_perm_summary_of.argtypes = [vp, i32, u64, ctypes.POINTER(_PermSummary)]
    lib.ddks_permutation_batch.argtypes = [vp, vp, i64, i32, i64, vp, i32, u32, vp,
                                           ctypes.POINTER(_Result), ctypes.POINTER(_PermSummary)]
    lib.ddks_significance.argtypes = [vp, vp, i64, i64, i32, u64, u32,
                                      ctypes.POINTER(ctypes.c_double)]
    lib.ddks_serve_submit.argtypes = [vp, ctypes.POINTER(_Request), ctypes.POINTER(u64)]
    lib.ddks_serve_poll.argtypes = [vp, u64, i32, ctypes.POINTER(_Result)]
    lib.ddks_serve_stats_get.argtypes = [vp, ctypes.POINTER(_ServeStats), i32]
    lib.ddks_vdks.argtypes = [vp, vp, i64, vp, i64, i32, i32, u32, ctypes.POINTER(_Result),
                              ctypes.POINTER(i64)]
    lib.ddks_rdks.argtypes = [vp, vp, i64, vp, i64, i32, u32, ctypes.POINTER(_Result), vp]
    lib.ddks_profile_get.argtypes = [vp, ctypes.POINTER(_Profile), i32]
    lib.ddks_status_string.argtypes = [ctypes.c_int]
    lib.ddks_status_string.restype = ctypes.c_char_p
    lib.ddks_last_error.argtypes = [vp]
    lib.ddks_last_error.restype = ctypes.c_char_p
    lib.ddks_version.restype = ctypes.c_char_p
    for name in ("ddks_create", "ddks_destroy", "ddks_distance", "ddks_permutation_batch",
                 "ddks_significance", "ddks_serve_submit", "ddks_serve_poll",
                 "ddks_serve_stats_get", "ddks_profile_get"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _points(x, d=None):
    """(pointer, rows, d, keepalive, is_device) for a numpy array or torch tensor."""
    if _is_torch(x):
        import torch
        if x.dtype != torch.float32 or not x.is_contiguous():
            raise ValueError("torch inputs must be contiguous float32")
        if not x.is_cuda:
            return _points(x.numpy(), d)
        shape = x.shape
        if len(shape) == 2:  # the usual case, without building a reshaped view
            return x.data_ptr(), shape[0], shape[1], x, True
        t = x.reshape(shape[0], -1) if len(shape) > 1 else x.reshape(-1, 1)
        return t.data_ptr(), t.shape[0], t.shape[1], t, True
    a = np.ascontiguousarray(x, dtype=np.float32)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return a.ctypes.data, a.shape[0], a.shape[1], a, False


class Context:
    """One libddks context (device, stream, buffers, serving loop)."""

    def __init__(self, device: int = 0, stream=None, mem_budget: int = 0, flags: int = 0,
                 serve_streams: int = 0, serve_queue_depth: int = 0, tune_cache: str | None = None):
        self._lib = load()
        o = _Options()
        self._lib.ddks_default_options(ctypes.byref(o))
        o.device = device
        if stream is not None:
            o.stream = stream if isinstance(stream, int) else stream.cuda_stream
        o.mem_budget = mem_budget
        o.flags = flags
        o.serve_streams = serve_streams
        o.serve_queue_depth = serve_queue_depth
        self._cache = tune_cache.encode() if tune_cache else None
        o.tune_cache = self._cache
        h = ctypes.c_void_p()
        st = self._lib.ddks_create(ctypes.byref(o), ctypes.byref(h))
        if st != DDKS_OK:
            raise DDKSError(st, "ddks_create failed: "
                            + self._lib.ddks_status_string(st).decode())
        self._h = h

    # -------------------------------------------------------------- helpers
    def _check(self, st: int, what: str):
        if st != DDKS_OK:
            err = self._lib.ddks_last_error(self._h).decode()
            raise DDKSError(st, f"{what}: {err or self._lib.ddks_status_string(st).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ddks_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self) -> int:
        return self._h.value

    # -------------------------------------------------------------- calls
    def distance(self, P, Q, *, counts: bool = False, flags: int = 0):
        """Exact ddKS of P and Q.  Returns Result, or (Result, counts[N, 2^d, 2])
        when counts=True (a numpy array for host inputs, a torch int32 tensor
        holding the uint32 bits for device inputs)."""
        pp, n_p, d, kp, dev_p = _points(P)
        qp, n_q, dq, kq, dev_q = _points(Q)
        if d != dq:
            raise ValueError("P and Q must have the same number of columns")
        if dev_p != dev_q:
            raise ValueError("P and Q must both be host arrays or both device tensors")
        if dev_p:
            flags |= DDKS_DEVICE_PTRS
        cbuf = None
        cptr = None
        if counts:
            N = n_p + n_q
            if dev_p:
                import torch
                cbuf = torch.empty((N, 1 << d, 2), dtype=torch.int32, device=kp.device)
                cptr = cbuf.data_ptr()
            else:
                cbuf = np.empty((N, 1 << d, 2), dtype=np.uint32)
                cptr = cbuf.ctypes.data
        r = _Result()
        st = self._lib.ddks_distance(self._h, pp, n_p, qp, n_q, d, flags, ctypes.byref(r), cptr)
        self._check(st, "ddks_distance")
        res = Result._from(r)
        return (res, cbuf) if counts else res

    def distance_noalloc(self, P, Q, *, counts=None, flags: int = 0):
        """ddks_distance_noalloc: the exact statistic of device tensors P and Q
        computed in the library's static scratch (no device allocation).
        counts: None or a caller-allocated device tensor of N * 2^d * 2 32-bit
        words that receives the membership counts."""
        pp, n_p, d, kp, dev_p = _points(P)
        qp, n_q, dq, kq, dev_q = _points(Q)
        if d != dq:
            raise ValueError("P and Q must have the same number of columns")
        if not (dev_p and dev_q):
            raise ValueError("the no-allocation call takes device tensors only")
        cptr = None
        if counts is not None:
            if not (_is_torch(counts) and counts.is_cuda and counts.is_contiguous()
                    and counts.numel() * counts.element_size() == (n_p + n_q) * (2 << d) * 4):
                raise ValueError("counts must be a contiguous device tensor of N * 2^d * 2 words")
            cptr = counts.data_ptr()
        r = _Result()
        st = self._lib.ddks_distance_noalloc(self._h, pp, n_p, qp, n_q, d, flags | DDKS_DEVICE_PTRS,
                                             ctypes.byref(r), cptr)
        self._check(st, "ddks_distance_noalloc")
        return Result._from(r)

    def permutation_batch(self, Z, n_p: int, labels, *, flags: int = 0):
        """Numerators for every relabelling row (labels: [B, ceil(n/32)] uint32
        words), the Result of the split 'first n_p rows' and the p-value summary
        {B, n_ge, p_value, fraction}."""
        zp, n, d, kz, dev = _points(Z)
        if dev:
            flags |= DDKS_DEVICE_PTRS
            import torch
            L = labels
            if not (_is_torch(L) and L.is_cuda):
                raise ValueError("with device points, labels must be a device tensor")
            B = L.shape[0]
            lp = L.data_ptr()
            nums = torch.empty(B, dtype=torch.int64, device=kz.device)
            nptr = nums.data_ptr()
        else:
            L = np.ascontiguousarray(labels, dtype=np.uint32)
            B = L.shape[0]
            if B and L.shape[1] != (n + 31) // 32:
                raise ValueError("label rows must have ceil(n/32) words")
            lp = L.ctypes.data
            nums = np.empty(B, dtype=np.uint64)
            nptr = nums.ctypes.data
        r = _Result()
        sm = _PermSummary()
        st = self._lib.ddks_permutation_batch(self._h, zp, n, d, n_p, lp, B, flags, nptr,
                                              ctypes.byref(r), ctypes.byref(sm))
        self._check(st, "ddks_permutation_batch")
        summary = {"B": sm.B, "n_ge": sm.n_ge, "p_value": sm.p_value, "fraction": sm.fraction}
        return nums, Result._from(r), summary

    def vdks(self, P, Q, voxels_per_dim: int, *, flags: int = 0):
        """vdKS (Alg. 1) of P and Q on a voxels_per_dim^d grid: (Result,
        number of filled voxels); Result.argmax_origin is the voxel key."""
        pp, n_p, d, kp, dev_p = _points(P)
        qp, n_q, dq, kq, dev_q = _points(Q)
        if d != dq:
            raise ValueError("P and Q must have the same number of columns")
        if dev_p != dev_q:
            raise ValueError("P and Q must both be host arrays or both device tensors")
        if dev_p:
            flags |= DDKS_DEVICE_PTRS
        r = _Result()
        nf = ctypes.c_int64()
        st = self._lib.ddks_vdks(self._h, pp, n_p, qp, n_q, d, voxels_per_dim, flags, ctypes.byref(r),
                                 ctypes.byref(nf))
        self._check(st, "ddks_vdks")
        return Result._from(r), nf.value

    def rdks(self, P, Q, *, flags: int = 0):
        """rdKS (Alg. 2) of P and Q: (Result, per-corner numerators[d + 1]);
        Result.argmax_origin is the lowest maximising corner."""
        pp, n_p, d, kp, dev_p = _points(P)
        qp, n_q, dq, kq, dev_q = _points(Q)
        if d != dq:
            raise ValueError("P and Q must have the same number of columns")
        if dev_p != dev_q:
            raise ValueError("P and Q must both be host arrays or both device tensors")
        if dev_p:
            flags |= DDKS_DEVICE_PTRS
        r = _Result()
        per = np.zeros(d + 1, dtype=np.uint64)
        st = self._lib.ddks_rdks(self._h, pp, n_p, qp, n_q, d, flags, ctypes.byref(r), per.ctypes.data)
        self._check(st, "ddks_rdks")
        return Result._from(r), per

    def significance(self, counts, n_p: int, n_q: int, d: int, num: int, *, flags: int = 0):
        if _is_torch(counts) and counts.is_cuda:
            flags |= DDKS_DEVICE_PTRS
            cp = counts.data_ptr()
            keep = counts
        else:
            keep = np.ascontiguousarray(counts, dtype=np.uint32)
            cp = keep.ctypes.data
        S = ctypes.c_double()
        st = self._lib.ddks_significance(self._h, cp, n_p, n_q, d, num, flags, ctypes.byref(S))
        self._check(st, "ddks_significance")
        return S.value

    def serve_submit(self, P, Q, flags: int = 0) -> int:
        """Submits one test (host arrays); flags: DDKS_WITH_SIGNIFICANCE
        (and DDKS_SIG_POISSON) for the analytic significance in the result.
        Returns the ticket, or -1 when the queue is full."""
        pp, n_p, d, kp, dev_p = _points(P)
        qp, n_q, dq, kq, dev_q = _points(Q)
        if dev_p or dev_q:
            raise ValueError("serving takes host arrays")
        if d != dq:
            raise ValueError("P and Q must have the same number of columns")
        req = _Request(pp, n_p, qp, n_q, d, flags)
        t = ctypes.c_uint64()
        st = self._lib.ddks_serve_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if st == DDKS_E_AGAIN:
            return -1
        self._check(st, "ddks_serve_submit")
        return t.value

    def serve_poll(self, ticket: int, timeout_us: int = -1):
        """Result, or None if still pending after timeout_us."""
        r = _Result()
        st = self._lib.ddks_serve_poll(self._h, ticket, timeout_us, ctypes.byref(r))
        if st == DDKS_E_PENDING:
            return None
        self._check(st, "ddks_serve_poll")
        return Result._from(r)

    def profile(self, reset: bool = False) -> dict:
        """Device-time counters (needs flags=DDKS_PROFILE_KERNELS at creation)."""
        p = _Profile()
        self._check(self._lib.ddks_profile_get(self._h, ctypes.byref(p), 1 if reset else 0),
                    "ddks_profile_get")
        return {k: getattr(p, k) for k, _ in _Profile._fields_}

    def serve_stats(self, reset: bool = False) -> dict:
        s = _ServeStats()
        st = self._lib.ddks_serve_stats_get(self._h, ctypes.byref(s), 1 if reset else 0)
        self._check(st, "ddks_serve_stats_get")
        return {k: getattr(s, k) for k, _ in _ServeStats._fields_}


def perm_summary(nums, num_obs: int) -> dict:
    """Permutation p-value of num_obs among the relabelling numerators nums
    (ddks_perm_summary_of): {B, n_ge, p_value, fraction}."""
    a = np.ascontiguousarray(nums, dtype=np.uint64)
    sm = _PermSummary()
    st = load().ddks_perm_summary_of(a.ctypes.data if a.size else None, a.size, int(num_obs),
                                     ctypes.byref(sm))
    if st != DDKS_OK:
        raise DDKSError(st, "ddks_perm_summary_of")
    return {"B": sm.B, "n_ge": sm.n_ge, "p_value": sm.p_value, "fraction": sm.fraction}


def version() -> str:
    return load().ddks_version().decode()
