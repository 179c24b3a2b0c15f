"""Seeded synthetic inputs for the ddKS workloads.

This module only draws random numbers and lays them out; it holds none of
the statistic's arithmetic, so both the GPU path and the CPU oracle can be
fed from it without sharing any part of the method.

The paper's datasets (Sec. 4.1) come without their parameters, so these
stand in for them with the same structure:
  gaussian_shift  ~ GVM  (two Gaussians, shifted means)
  gaussian_scale  ~ GVS  (two Gaussians, one wider coordinate)
  mixture_grid    ~ MM-like 3-component mixture on a 1/64 grid (forces ties
                    and produces -0.0)
  permutation     Gaussian vs unit-variance Laplace, pooled, plus seeded
                    relabelling rows (Sec. 3's permutation test)
  serving_stream  a GVM-like stream of tests of mixed d and sizes with
                    Poisson arrivals

All draws use numpy's PCG64 ``default_rng(seed)`` in float64 and are then
rounded to float32 (round-to-nearest).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2106137060


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def gaussian_shift(n_p: int = 500, n_q: int = 500, d: int = 3, shift: float = 0.1,
                   seed: int = SEED_BASE + 1):
    """P ~ N(0, I_d); Q ~ N(shift*1, I_d), Q drawn after P."""
    g = _rng(seed)
    P = g.standard_normal((n_p, d))
    Q = g.standard_normal((n_q, d)) + shift
    return P.astype(np.float32), Q.astype(np.float32)


def gaussian_scale(n_p: int = 20000, n_q: int = 20000, d: int = 4, last_sd: float = 1.2,
                   seed: int = SEED_BASE + 2):
    """P ~ N(0, I_d); Q ~ N(0, diag(1, .., 1, last_sd^2))."""
    g = _rng(seed)
    P = g.standard_normal((n_p, d))
    scale = np.ones(d)
    scale[-1] = last_sd
    Q = g.standard_normal((n_q, d)) * scale
    return P.astype(np.float32), Q.astype(np.float32)


def mixture_grid(n_p: int = 100000, n_q: int = 100000, d: int = 6, shift: float = 0.2,
                 grid: int = 64, seed: int = SEED_BASE + 3):
    """3-component Gaussian mixture, unit covariance, equal weights.  Component
    c has mean s_c * e_{a_c} (a_c uniform axis, s_c uniform sign); Q is the
    same mixture with component 0's mean moved by shift along its own axis.
    Every value is rounded to a 1/grid lattice (exact in fp32), which creates
    ties and keeps negative zeros."""
    g = _rng(seed)
    axes = g.integers(0, d, size=3)
    signs = g.choice(np.array([-1.0, 1.0]), size=3)
    mu = np.zeros((3, d))
    mu[np.arange(3), axes] = signs
    mu_q = mu.copy()
    mu_q[0, axes[0]] += shift * signs[0]

    def draw(n, means):
        z = g.integers(0, 3, size=n)
        x = means[z] + g.standard_normal((n, d))
        return np.rint(x * grid) / grid

    P = draw(n_p, mu)
    Q = draw(n_q, mu_q)
    return P.astype(np.float32), Q.astype(np.float32)


def label_rows(n: int, n_p: int, B: int, seed: int) -> np.ndarray:
    """B seeded relabelling rows packed as [B, ceil(n/32)] uint32 words: row b
    uses default_rng(seed + 1000 + b).permutation(n); its first n_p entries
    are marked (bit i%32 of word i/32 set) as the first sample."""
    w = (n + 31) // 32
    out = np.zeros((B, w), dtype=np.uint32)
    for b in range(B):
        idx = _rng(seed + 1000 + b).permutation(n)[:n_p]
        mask = np.zeros(n, dtype=bool)
        mask[idx] = True
        bits = np.zeros(w * 32, dtype=np.uint32)
        bits[:n] = mask
        out[b] = (bits.reshape(w, 32) << np.arange(32, dtype=np.uint32)).sum(axis=1,
                                                                              dtype=np.uint32)
    return out


def permutation(n_each: int = 4096, d: int = 5, B: int = 1024, seed: int = SEED_BASE + 4):
    """Pooled Z: rows [0, n_each) ~ N(0, I_d), rows [n_each, 2 n_each) ~
    Laplace(0, 1/sqrt(2)) per coordinate (unit variance).  The observed split
    is 'first n_each rows are the first sample'.  Returns (Z, n_p, labels)."""
    g = _rng(seed)
    A = g.standard_normal((n_each, d))
    Bl = g.laplace(0.0, 1.0 / np.sqrt(2.0), size=(n_each, d))
    Z = np.concatenate([A, Bl]).astype(np.float32)
    return Z, n_each, label_rows(2 * n_each, n_each, B, seed)


@dataclass
class Request:
    t_arrival: float
    P: np.ndarray
    Q: np.ndarray
    d: int
    delta: float
    seed: int = 0  # generator seed of P and Q (see materialize)


@dataclass
class Stream:
    requests: list = field(default_factory=list)


def serving_stream(n_requests: int = 10000, rate: float = 1000.0, d_range=(2, 8),
                   n_range=(64, 65536), delta_max: float = 0.3, seed: int = SEED_BASE + 5,
                   materialize: bool = True) -> Stream:
    """Poisson-arrival stream of tests: d uniform in d_range (inclusive),
    n_P and n_Q independently log-uniform in n_range (rounded), delta uniform
    in [0, delta_max], P ~ N(0, I_d), Q ~ N(delta*1, I_d).  Arrival gaps are
    exponential with the given rate (tests per second)."""
    g = _rng(seed)
    t = 0.0
    reqs = []
    lo, hi = np.log(n_range[0]), np.log(n_range[1])
    for _ in range(n_requests):
        t += g.exponential(1.0 / rate)
        d = int(g.integers(d_range[0], d_range[1] + 1))
        n_p = int(np.rint(np.exp(g.uniform(lo, hi))))
        n_q = int(np.rint(np.exp(g.uniform(lo, hi))))
        delta = float(g.uniform(0.0, delta_max))
        sub = int(g.integers(0, 2**63 - 1))
        if materialize:
            h = _rng(sub)
            P = h.standard_normal((n_p, d)).astype(np.float32)
            Q = (h.standard_normal((n_q, d)) + delta).astype(np.float32)
        else:
            P = np.empty((n_p, d), np.float32)
            Q = np.empty((n_q, d), np.float32)
        reqs.append(Request(t, P, Q, d, delta, sub))
    return Stream(reqs)


def materialize(r: Request):
    """(P, Q) of a request from serving_stream(materialize=False): the same
    arrays the materialized stream holds."""
    h = _rng(r.seed)
    P = h.standard_normal((r.P.shape[0], r.d)).astype(np.float32)
    Q = (h.standard_normal((r.Q.shape[0], r.d)) + r.delta).astype(np.float32)
    return P, Q


# ---------------------------------------------------------------- power-study datasets
# Sec. 4.1's synthetic datasets (LS needs a trained network and images, so it
# is left out).  The paper gives no parameters; these are the stated ones,
# with sigma = 1 and the means placed symmetrically about the origin:
#   GVM   P ~ N(-delta/2 1, I), Q ~ N(+delta/2 1, I)                 (delta 0.5)
#   GVS   P ~ N(0, I), Q ~ N(0, (1 + delta)^2 I)                      (delta 0.5)
#   DVU   P uniform on the diagonal from 0 to 1, Q uniform on [0, 1]^d (no parameter)
#   Skew  P ~ Exp(1)^d, Q ~ Exp(1 + delta)^d (rates)                 (delta 0.5)
#   MM    GVM with the first round(noise n) points of each sample replaced by
#         draws uniform on [-3 sigma, 3 sigma]^d                      (delta 0.5, noise 0.5)
POWER_DATASETS = ("GVM", "GVS", "DVU", "Skew", "MM")
POWER_DEFAULT_DELTA = {"GVM": 0.5, "GVS": 0.5, "DVU": None, "Skew": 0.5, "MM": 0.5}


def power_dataset(name: str, n: int, d: int = 3, delta: float | None = None, noise: float = 0.5,
                  seed: int = SEED_BASE + 6):
    """Two samples of n points each from one of the power-study datasets."""
    g = _rng(seed)
    if name not in POWER_DEFAULT_DELTA:
        raise ValueError(f"unknown dataset {name}")
    delta = POWER_DEFAULT_DELTA[name] if delta is None else delta
    if name == "GVM" or name == "MM":
        P = g.standard_normal((n, d)) - delta / 2
        Q = g.standard_normal((n, d)) + delta / 2
        if name == "MM":
            k = int(round(noise * n))
            for X in (P, Q):
                X[:k] = g.uniform(-3.0, 3.0, size=(k, d))
    elif name == "GVS":
        P = g.standard_normal((n, d))
        Q = g.standard_normal((n, d)) * (1.0 + delta)
    elif name == "DVU":
        t = g.uniform(0.0, 1.0, size=(n, 1))
        P = np.repeat(t, d, axis=1)
        Q = g.uniform(0.0, 1.0, size=(n, d))
    else:  # Skew
        P = g.exponential(1.0, size=(n, d))
        Q = g.exponential(1.0 / (1.0 + delta), size=(n, d))
    return P.astype(np.float32), Q.astype(np.float32)


def relabel_rows(n_total: int, n_p: int, B: int, seed: int) -> np.ndarray:
    """B seeded relabellings of a pooled sample (label_rows with its own seed)."""
    return label_rows(n_total, n_p, B, seed)


# The five workloads by name, as (callable, description).
WORKLOADS = {
    "gaussian_shift_d3_500": (gaussian_shift,
                              "d=3, n_P=n_Q=500, P~N(0,I), Q~N(0.1*1,I)"),
    "gaussian_scale_d4_20000": (gaussian_scale,
                                "d=4, n_P=n_Q=20000, P~N(0,I), Q~N(0,diag(1,1,1,1.44))"),
    "mixture_grid_d6_100000": (mixture_grid,
                               "d=6, n_P=n_Q=100000, 3-component mixture on a 1/64 grid"),
    "permutation_d5_8192x1024": (permutation,
                                 "d=5, pooled 2x4096 (Gaussian vs Laplace), 1024 relabellings"),
    "serving_10000": (serving_stream,
                      "10^4 Poisson-arrival tests, d in 2..8, n log-uniform in [64, 65536]"),
}
