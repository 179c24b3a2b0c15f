"""CPU oracle for the exact ddKS statistic -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and
its Python binding) never does, and this package never imports the product.

Functions follow the paper (arXiv:2106.13706):
  distance      -- Sec. 2.1 Eq. (ddks_tensor_definition) with Eq. (g)'s '>='
                   convention and Eq. (membership)/(d1), normalised as in
                   Sec. 3 Eq. (abs_difference); exact integers num/den.
  permutation   -- the permutation test of Sec. 3 / Sec. 4.2, every
                   relabelling re-run through the definition.
  pvalue        -- permutation p-value (add-one estimator; the paper gives
                   no formula, see the readings in the design notes).
  significance  -- analytic significance S, Sec. 3 Eq. (ddks_significance)
                   with the Bayes rate estimator (M_T + 1)/(N_T + 2).
  tail          -- 1 - P(delta <= D | n_P, n_T, lambda) for one entry.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None



# rate models of the analytic significance (Sec. 3)
_MODELS = {"binomial": 0, "poisson": 1}

def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32, u64p = ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)
    vp = ctypes.c_void_p
    lib.ddks_oracle_distance.argtypes = [vp, i64, vp, i64, i32, i32, vp, vp, vp, u64p,
                                         ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int32)]
    lib.ddks_oracle_distance.restype = ctypes.c_int
    lib.ddks_oracle_permutation.argtypes = [vp, i64, i32, i64, vp, i32, i32, vp]
    lib.ddks_oracle_permutation.restype = ctypes.c_int
    lib.ddks_oracle_tail.argtypes = [i64, i64, ctypes.c_double, ctypes.c_uint64]
    lib.ddks_oracle_tail.restype = ctypes.c_double
    lib.ddks_oracle_tail_model.argtypes = [i64, i64, ctypes.c_double, ctypes.c_uint64, ctypes.c_int]
    lib.ddks_oracle_tail_model.restype = ctypes.c_double
    lib.ddks_oracle_significance_model.argtypes = [vp, i64, i64, i32, ctypes.c_uint64, ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_double)]
    lib.ddks_oracle_significance_model.restype = ctypes.c_int
    lib.ddks_oracle_significance.argtypes = [vp, i64, i64, i32, ctypes.c_uint64,
                                             ctypes.POINTER(ctypes.c_double)]
    lib.ddks_oracle_significance.restype = ctypes.c_int
    lib.ddks_oracle_vdks.argtypes = [vp, i64, vp, i64, i32, i32, u64p, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.ddks_oracle_vdks.restype = ctypes.c_int
    lib.ddks_oracle_rdks.argtypes = [vp, i64, vp, i64, i32, u64p, ctypes.POINTER(ctypes.c_int32), vp]
    lib.ddks_oracle_rdks.restype = ctypes.c_int
    lib.ddks_oracle_origin_counts.argtypes = [vp, i64, vp, i64, i32, vp, i64, vp]
    lib.ddks_oracle_origin_counts.restype = ctypes.c_int
    _lib = lib
    return lib


@dataclass
class OracleResult:
    num: int
    den: int
    D: float
    argmax_origin: int
    argmax_orthant: int
    counts: np.ndarray | None = None       # [N, 2^d, 2] uint32, sample 0 = P
    origin_num: np.ndarray | None = None   # [N] uint64
    origin_code: np.ndarray | None = None  # [N] int32


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return a


def distance(P, Q, *, threads: int = 1, counts: bool = False,
             per_origin: bool = False) -> OracleResult:
    """Exact ddKS of two fp32 samples (rows are points)."""
    lib = _load()
    P, Q = _f32(P), _f32(Q)
    if P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must have the same dimension")
    n_p, d = P.shape
    n_q = Q.shape[0]
    N = n_p + n_q
    c = np.zeros((N, 1 << d, 2), dtype=np.uint32) if counts else None
    on = np.zeros(N, dtype=np.uint64) if per_origin else None
    oc = np.zeros(N, dtype=np.int32) if per_origin else None
    num = ctypes.c_uint64()
    ko = ctypes.c_int64()
    jo = ctypes.c_int32()
    st = lib.ddks_oracle_distance(
        P.ctypes.data, n_p, Q.ctypes.data, n_q, d, threads,
        c.ctypes.data if c is not None else None,
        on.ctypes.data if on is not None else None,
        oc.ctypes.data if oc is not None else None,
        ctypes.byref(num), ctypes.byref(ko), ctypes.byref(jo))
    if st != 0:
        raise ValueError(f"oracle distance failed with status {st}")
    den = n_p * n_q
    return OracleResult(num.value, den, num.value / den, ko.value, jo.value, c, on, oc)


def origin_counts(P, Q, idx) -> np.ndarray:
    """[len(idx), 2^d, 2] counts of the chosen origins (P-then-Q indices)."""
    lib = _load()
    P, Q = _f32(P), _f32(Q)
    d = P.shape[1]
    ix = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((ix.size, 1 << d, 2), dtype=np.uint32)
    st = lib.ddks_oracle_origin_counts(P.ctypes.data, P.shape[0], Q.ctypes.data, Q.shape[0], d,
                                       ix.ctypes.data, ix.size, out.ctypes.data)
    if st != 0:
        raise ValueError(f"oracle origin_counts failed with status {st}")
    return out


def labels_to_words(mask_rows) -> np.ndarray:
    """Pack a [B, n] boolean matrix (True = first sample) into [B, ceil(n/32)]
    uint32 words, bit i%32 of word i/32."""
    m = np.asarray(mask_rows, dtype=bool)
    B, n = m.shape
    w = (n + 31) // 32
    out = np.zeros((B, w), dtype=np.uint32)
    for i in range(n):
        out[:, i // 32] |= (m[:, i].astype(np.uint32) << np.uint32(i % 32))
    return out


def permutation(Z, n_p: int, labels_words, *, threads: int = 1) -> np.ndarray:
    """Numerators of the statistic for each relabelling row."""
    lib = _load()
    Z = _f32(Z)
    n, d = Z.shape
    L = np.ascontiguousarray(labels_words, dtype=np.uint32)
    B = L.shape[0]
    if L.shape[1] != (n + 31) // 32:
        raise ValueError("label rows must have ceil(n/32) words")
    nums = np.zeros(B, dtype=np.uint64)
    st = lib.ddks_oracle_permutation(Z.ctypes.data, n, d, n_p, L.ctypes.data, B, threads,
                                     nums.ctypes.data)
    if st != 0:
        raise ValueError(f"oracle permutation failed with status {st}")
    return nums


def pvalue(nums, num_obs: int) -> tuple[float, float]:
    """Permutation p-value: (1 + #{num_b >= num_obs}) / (1 + B), and the raw
    fraction #{num_b >= num_obs} / B.  All statistics share one denominator,
    so the comparison is exact on the numerators."""
    nums = np.asarray(nums, dtype=np.uint64)
    hits = int(np.count_nonzero(nums >= np.uint64(num_obs)))
    B = nums.size
    return (1 + hits) / (1 + B), (hits / B if B else float("nan"))


def tail(n_p: int, n_q: int, lam: float, num: int, model: str = "binomial") -> float:
    """1 - P(|a/n_p - b/n_q| <= num/(n_p n_q)), a~Bi(n_p,lam), b~Bi(n_q,lam); with
    model="poisson" the pmfs are Poisson of the same means on the same supports."""
    return float(_load().ddks_oracle_tail_model(n_p, n_q, lam, num, _MODELS[model]))


def significance(counts, n_p: int, n_q: int, d: int, num: int, model: str = "binomial") -> float:
    """Analytic significance S of num/(n_p n_q) from the [N, 2^d, 2] counts."""
    lib = _load()
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    if c.shape != (n_p + n_q, 1 << d, 2):
        raise ValueError("counts must be [n_p+n_q, 2^d, 2]")
    S = ctypes.c_double()
    st = lib.ddks_oracle_significance_model(c.ctypes.data, n_p, n_q, d, num, _MODELS[model],
                                            ctypes.byref(S))
    if st != 0:
        raise ValueError(f"oracle significance failed with status {st}")
    return S.value


@dataclass
class VdksResult:
    num: int
    den: int
    D: float
    argmax_voxel: int    # sum_m v_m V^m of the maximising voxel (lowest)
    argmax_orthant: int
    n_filled: int        # voxels holding at least one point


def vdks(P, Q, V: int) -> VdksResult:
    """vdKS (Alg. 1) with V voxels per dimension."""
    lib = _load()
    P, Q = _f32(P), _f32(Q)
    if P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must have the same dimension")
    n_p, d = P.shape
    n_q = Q.shape[0]
    num = ctypes.c_uint64()
    kv = ctypes.c_int64()
    jo = ctypes.c_int32()
    nf = ctypes.c_int64()
    st = lib.ddks_oracle_vdks(P.ctypes.data, n_p, Q.ctypes.data, n_q, d, V, ctypes.byref(num),
                              ctypes.byref(kv), ctypes.byref(jo), ctypes.byref(nf))
    if st != 0:
        raise ValueError(f"oracle vdks failed with status {st}")
    den = n_p * n_q
    return VdksResult(num.value, den, num.value / den, kv.value, jo.value, nf.value)


@dataclass
class RdksResult:
    num: int
    den: int
    D: float
    argmax_corner: int   # 0 = the origin, m + 1 = the unit point e_m (lowest maximising)
    per_corner: np.ndarray  # numerator of each corner


def rdks(P, Q) -> RdksResult:
    """rdKS (Alg. 2): the two-sample KS statistic of the distances from each of
    the d + 1 corners of the normalised space, maximised over the corners."""
    lib = _load()
    P, Q = _f32(P), _f32(Q)
    if P.shape[1] != Q.shape[1]:
        raise ValueError("P and Q must have the same dimension")
    n_p, d = P.shape
    n_q = Q.shape[0]
    num = ctypes.c_uint64()
    corner = ctypes.c_int32()
    per = np.zeros(d + 1, dtype=np.uint64)
    st = lib.ddks_oracle_rdks(P.ctypes.data, n_p, Q.ctypes.data, n_q, d, ctypes.byref(num),
                              ctypes.byref(corner), per.ctypes.data)
    if st != 0:
        raise ValueError(f"oracle rdks failed with status {st}")
    den = n_p * n_q
    return RdksResult(num.value, den, num.value / den, corner.value, per)
