"""Power study of Sec. 4.2: the smallest sample size, and the smallest
parameter difference at a fixed sample size, at which a two-sample test built
on the exact statistic (or on vdKS / rdKS) rejects H0 at level alpha, each
found by bisection.

Each test is the permutation test the paper uses for every method (Sec. 4.2,
100 permutations): the p-value is the add-one estimator
(1 + #{relabellings at least as extreme}) / (1 + B).  For the exact statistic
all B relabellings run in one batched launch (ddks_permutation_batch); vdKS
and rdKS re-run the statistic on every relabelled pair and take the p-value
from ddks_perm_summary_of.  Reading of the bisection target (the paper aims
at a significance within a thousandth of alpha, finer than the 1/101 grid of
100 permutations can resolve): the smallest n in [n_lo, n_hi] (or delta in
[lo, hi], to a tolerance) whose test rejects, by bisection on the rejection
indicator, each point with its own seeded draw.  Everything here is
host-side orchestration; the statistics and p-values come from the library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import native, workloads


@dataclass
class PowerPoint:
    n: int
    p_value: float
    D: float
    rejected: bool
    # what reproduces the point: workloads.power_dataset(dataset, n_points,
    # d=d, delta=delta, seed=data_seed) and workloads.relabel_rows(2 n_points,
    # n_points, B, label_seed)
    n_points: int = 0
    delta: float | None = None
    data_seed: int = 0
    label_seed: int = 0


def _unpack_rows(words: np.ndarray, n_total: int) -> np.ndarray:
    bits = np.unpackbits(words.view(np.uint8), axis=1, bitorder="little")[:, :n_total]
    return bits.astype(bool)


def permutation_test(ctx: native.Context, P: np.ndarray, Q: np.ndarray, B: int = 100,
                     method: str = "ddks", seed: int = 0, voxels_per_dim: int = 8) -> tuple:
    """(p-value, observed D) of the permutation test of P against Q."""
    Z = np.concatenate([P, Q]).astype(np.float32)
    n_p, n = len(P), len(P) + len(Q)
    labels = workloads.relabel_rows(n, n_p, B, seed)
    if method == "ddks":
        _, obs, summ = ctx.permutation_batch(Z, n_p, labels)
        return summ["p_value"], obs.D
    stat = {"vdks": lambda a, b: ctx.vdks(a, b, voxels_per_dim)[0].num,
            "rdks": lambda a, b: ctx.rdks(a, b)[0].num}[method]
    obs = stat(P, Q)
    nums = [stat(Z[m], Z[~m]) for m in _unpack_rows(labels, n)]
    return native.perm_summary(nums, obs)["p_value"], obs / (n_p * (n - n_p))


def min_sample_size(ctx: native.Context, dataset: str, method: str = "ddks", alpha: float = 0.05,
                    B: int = 100, n_lo: int = 4, n_hi: int = 2048, d: int = 3,
                    delta: float | None = None, seed: int = workloads.SEED_BASE + 60,
                    voxels_per_dim: int = 8):
    """Smallest n (points per sample) in [n_lo, n_hi] whose permutation test
    rejects H0 at alpha (bisection; None if even n_hi does not reject), and the
    points evaluated."""
    cache = {}

    def rejects(n):
        if n not in cache:
            P, Q = workloads.power_dataset(dataset, n, d=d, delta=delta, seed=seed + n)
            p, D = permutation_test(ctx, P, Q, B, method, seed=seed + 7919 * n,
                                    voxels_per_dim=voxels_per_dim)
            cache[n] = PowerPoint(n, p, D, p <= alpha, n, delta, seed + n, seed + 7919 * n)
        return cache[n].rejected

    if not rejects(n_hi):
        return None, sorted(cache.values(), key=lambda x: x.n)
    lo, hi = n_lo, n_hi
    if rejects(lo):
        return lo, sorted(cache.values(), key=lambda x: x.n)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if rejects(mid):
            hi = mid
        else:
            lo = mid
    return hi, sorted(cache.values(), key=lambda x: x.n)


def min_parameter_gap(ctx: native.Context, dataset: str, method: str = "ddks", n: int = 50,
                      alpha: float = 0.05, B: int = 100, lo: float = 0.0, hi: float = 4.0,
                      tol: float = 1.0 / 64, d: int = 3, seed: int = workloads.SEED_BASE + 61,
                      voxels_per_dim: int = 8):
    """Smallest delta in [lo, hi] (to tol) at which the permutation test of n
    points per sample rejects H0 at alpha (bisection; None if delta = hi does
    not reject), and the points evaluated (PowerPoint.n holds the step index)."""
    if workloads.POWER_DEFAULT_DELTA[dataset] is None:
        raise ValueError(f"{dataset} has no parameter to vary")
    pts = []

    def rejects(delta):
        k = len(pts)
        P, Q = workloads.power_dataset(dataset, n, d=d, delta=delta, seed=seed + k)
        p, D = permutation_test(ctx, P, Q, B, method, seed=seed + 7919 * (k + 1),
                                voxels_per_dim=voxels_per_dim)
        pts.append((delta, PowerPoint(k, p, D, p <= alpha, n, delta, seed + k, seed + 7919 * (k + 1))))
        return p <= alpha

    if not rejects(hi):
        return None, pts
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if rejects(mid):
            hi = mid
        else:
            lo = mid
    return hi, pts
