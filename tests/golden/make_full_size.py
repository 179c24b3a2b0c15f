#!/usr/bin/env python3
"""Writes the full-size expected values of the five workloads from the CPU
oracle alone (test infrastructure: nothing here touches the GPU library).

Each output file under tests/golden/ records what the oracle computes on the
seeded inputs of ``paper_2106_13706_amd.workloads`` at the workload's full
size, plus a SHA-256 of those inputs so that a change of the generators is
caught before any comparison:

  full_gaussian_shift_d3_500.json      exact statistic + counts digest
  full_gaussian_scale_d4_20000.json    exact statistic + counts digest +
                                       analytic significance (both models)
  full_mixture_grid_d6_100000.json     exact statistic + counts digest
  full_permutation_d5_8192x1024.json   all 1024 relabelling numerators, the
                                       observed split and its significance
  serving_10000_sample.json            every stream request with at most
                                       8192 points, and a seeded stratified
                                       sample of the larger ones per d

The counts digest is SHA-256 over the [N][2^d][2] little-endian uint32
membership counts (origin-major, P then Q, sample 0 = P).

Usage: python tests/golden/make_full_size.py [--threads T] [name ...]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2106_13706_amd import workloads  # noqa: E402


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def counts_sha(c):
    return sha(np.ascontiguousarray(c, dtype="<u4"))


def _write(name, obj):
    p = os.path.join(HERE, name)
    with open(p, "w") as f:
        json.dump(obj, f, indent=1)
        f.write("\n")
    print(f"wrote {p}", flush=True)


def exact(name, P, Q, threads, significance=False):
    t0 = time.perf_counter()
    o = oracle.distance(P, Q, counts=True, threads=threads)
    sec = time.perf_counter() - t0
    out = {"workload": name, "d": int(P.shape[1]), "n_p": len(P), "n_q": len(Q),
           "inputs_sha256": sha(P, Q), "num": o.num, "den": o.den, "D": o.D,
           "argmax_origin": o.argmax_origin, "argmax_orthant": o.argmax_orthant,
           "counts_sha256": counts_sha(o.counts),
           "oracle_seconds": round(sec, 1), "oracle_threads": threads}
    if significance:
        for model in ("binomial", "poisson"):
            out[f"S_{model}"] = oracle.significance(o.counts, len(P), len(Q), P.shape[1], o.num,
                                                    model=model)
    print(f"{name}: num {o.num} argmax ({o.argmax_origin},{o.argmax_orthant}) in {sec:.1f} s",
          flush=True)
    return out


def make_shift(threads):
    P, Q = workloads.gaussian_shift()
    _write("full_gaussian_shift_d3_500.json", exact("gaussian_shift_d3_500", P, Q, threads, True))


def make_scale(threads):
    P, Q = workloads.gaussian_scale()
    _write("full_gaussian_scale_d4_20000.json",
           exact("gaussian_scale_d4_20000", P, Q, threads, True))


def make_mixture(threads):
    P, Q = workloads.mixture_grid()
    _write("full_mixture_grid_d6_100000.json", exact("mixture_grid_d6_100000", P, Q, threads))


def make_permutation(threads):
    Z, n_p, labels = workloads.permutation()
    t0 = time.perf_counter()
    nums = oracle.permutation(Z, n_p, labels, threads=threads)
    sec = time.perf_counter() - t0
    obs = exact("permutation_d5_8192x1024 observed split", Z[:n_p], Z[n_p:], threads, True)
    p, frac = oracle.pvalue(nums, obs["num"])
    out = {"workload": "permutation_d5_8192x1024", "n": len(Z), "n_p": n_p, "d": int(Z.shape[1]),
           "B": int(labels.shape[0]), "inputs_sha256": sha(Z, labels),
           "nums": [int(x) for x in nums], "observed": obs, "p_value": p, "fraction": frac,
           "oracle_seconds": round(sec, 1), "oracle_threads": threads}
    print(f"permutation: {len(nums)} rows in {sec:.1f} s, p = {p}", flush=True)
    _write("full_permutation_d5_8192x1024.json", out)


# Stratified sample of the larger serving requests: per d, this many requests
# from each point-count band (the first ones of the band in a seeded shuffle).
SERVE_BANDS = ((8192, 16384, 3), (16384, 32768, 3), (32768, 65536, 3), (65536, 131072, 4))
SERVE_SAMPLE_SEED = workloads.SEED_BASE + 505


def serving_selection(stream):
    """Indices of the checked requests: all with n_p + n_q <= 8192, then per
    d and band the first k of a seeded shuffle."""
    N = np.array([r.P.shape[0] + r.Q.shape[0] for r in stream.requests])
    d = np.array([r.d for r in stream.requests])
    small = [int(i) for i in np.nonzero(N <= 8192)[0]]
    order = np.random.default_rng(SERVE_SAMPLE_SEED).permutation(len(N))
    large = []
    for dd in range(2, 9):
        for lo, hi, k in SERVE_BANDS:
            pick = [int(i) for i in order if d[i] == dd and lo < N[i] <= hi][:k]
            large += pick
    return small, sorted(large)


def make_serving(threads):
    stream = workloads.serving_stream(materialize=False)
    small, large = serving_selection(stream)
    rows = []
    h = hashlib.sha256()
    t0 = time.perf_counter()
    for k, i in enumerate(small + large):
        P, Q = workloads.materialize(stream.requests[i])
        h.update(P.tobytes())
        h.update(Q.tobytes())
        o = oracle.distance(P, Q, threads=threads)
        rows.append([i, o.num, o.argmax_origin, o.argmax_orthant])
        if k % 500 == 0 or i in large:
            print(f"  request {i}: d={P.shape[1]} N={len(P) + len(Q)} num {o.num} "
                  f"({time.perf_counter() - t0:.0f} s)", flush=True)
    out = {"workload": "serving_10000",
           "selection": "every request with n_p + n_q <= 8192, then per d in 2..8 the first "
                        "requests of a seeded shuffle (seed %d) in each band (lo, hi, count) %s"
                        % (SERVE_SAMPLE_SEED, [list(b) for b in SERVE_BANDS]),
           "n_small": len(small), "n_large": len(large), "inputs_sha256": h.hexdigest(),
           "columns": ["request", "num", "argmax_origin", "argmax_orthant"], "rows": rows,
           "oracle_seconds": round(time.perf_counter() - t0, 1), "oracle_threads": threads}
    _write("serving_10000_sample.json", out)


MAKERS = {"shift": make_shift, "scale": make_scale, "mixture": make_mixture,
          "permutation": make_permutation, "serving": make_serving}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("names", nargs="*", default=list(MAKERS))
    a = ap.parse_args()
    for n in a.names:
        MAKERS[n](a.threads)


if __name__ == "__main__":
    main()
