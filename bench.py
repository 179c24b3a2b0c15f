#!/usr/bin/env python3
"""Benchmark of the exact ddKS orthant-counting sweep on one MI355X.

Prints ONE JSON line.  The headline is origin*point*dim compares per second
of a whole ddks_distance step (ingest, sweep, scoring, reduction, result
read-back) on the d=4, 20000+20000 Gaussian workload with inputs already
resident in HBM.  The same line carries:
  roofline      the sweep kernel's device time (HIP events recorded by the
                library on the stream it launches on) against the VALU
                compare peak;
  cpu_baseline  the CPU oracle timed on this host on the same workload;
  extras        the d=6 100000+100000 mixture, the permutation batch and the
                serving loop, when their entry points are available.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 2.4 GHz, one 32-bit VALU lane-op per compare.
VALU_COMPARE_PEAK = 256 * 64 * 2.4e9
PROFILES = os.path.join(ROOT, "profiles")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, or None if
    the kernel source changed since the counters were taken."""
    p = os.path.join(PROFILES, f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(p):
        return None
    t = json.load(open(p))
    src = os.path.join(ROOT, t["source"])
    if not os.path.exists(src) or _sha(src) != t["source_sha256"]:
        return None
    return t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]


def _time_distance(ctx, P, Q, steps, warmup, torch):
    for _ in range(warmup):
        r = ctx.distance(P, Q)
    torch.cuda.synchronize()
    ctx.profile(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        r = ctx.distance(P, Q)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return r, (t1 - t0) / steps, ctx.profile(reset=True)


def cpu_baseline(P, Q, compares):
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        o = oracle.distance(P, Q, threads=cores)
        times.append(time.perf_counter() - t0)
        if sum(times) > 20.0:
            break
    times.sort()
    med = times[len(times) // 2]
    return o, {"value": compares / med, "unit": "compares/s", "cores": cores, "kind": "oracle",
               "sample": f"the full workload ({len(P) + len(Q)} origins x "
                         f"{len(P) + len(Q)} points x {P.shape[1]} dims), median of "
                         f"{len(times)} run(s), {med:.2f} s each"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one device copy of this size (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on a single device).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2106_13706_amd import native, workloads

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ctx = native.Context(stream=stream, flags=native.DDKS_PROFILE_KERNELS)

    workload = "gaussian_scale_d4_20000"
    P, Q = workloads.gaussian_scale()
    n_p, n_q, d = len(P), len(Q), P.shape[1]
    N = n_p + n_q
    compares = N * N * d
    Pt = torch.from_numpy(P).to(dev)
    Qt = torch.from_numpy(Q).to(dev)
    _log(f"[bench] {workload}: warmup {args.warmup}, steps {args.steps}")
    r, sec, prof = _time_distance(ctx, Pt, Qt, args.steps, args.warmup, torch)
    ms_per_step = sec * 1e3
    value = compares / sec
    sweep_s = prof["sweep_ms"] / max(1, prof["sweeps"]) / 1e3
    achieved = compares / sweep_s if sweep_s > 0 else 0.0
    traffic = _traffic("k_sweep", workload)
    line = {
        "metric": "origin*point*dim compares/s",
        "value": value,
        "unit": "compares/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "d": d, "n_p": n_p, "n_q": n_q,
                   "inputs": "device-resident fp32", "result": {"num": r.num, "den": r.den}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_COMPARE_PEAK,
                     "unit": "compares/s", "frac": achieved / VALU_COMPARE_PEAK,
                     "traffic": traffic,
                     "kernel": "k_sweep", "kernel_avg_ms": sweep_s * 1e3,
                     "score_avg_ms": prof["score_ms"] / max(1, prof["sweeps"])},
    }
    _log(f"[bench] step {ms_per_step:.4f} ms, sweep {sweep_s * 1e3:.4f} ms, "
         f"frac {achieved / VALU_COMPARE_PEAK:.3f}")

    if not args.no_cpu_baseline:
        _log("[bench] cpu baseline (oracle)")
        o, cb = cpu_baseline(P, Q, compares)
        if o.num != r.num:
            raise SystemExit(f"GPU/oracle mismatch: {r.num} vs {o.num}")
        line["cpu_baseline"] = cb

    extras = {}
    if not args.no_extras:
        _log("[bench] extra: mixture_grid_d6_100000")
        P3, Q3 = workloads.mixture_grid()
        P3t = torch.from_numpy(P3).to(dev)
        Q3t = torch.from_numpy(Q3).to(dev)
        N3 = len(P3) + len(Q3)
        c3 = N3 * N3 * P3.shape[1]
        r3, s3, p3 = _time_distance(ctx, P3t, Q3t, 5, 2, torch)
        k3 = p3["sweep_ms"] / max(1, p3["sweeps"]) / 1e3
        extras["mixture_grid_d6_100000"] = {
            "value": c3 / s3, "unit": "compares/s", "ms_per_step": s3 * 1e3,
            "kernel_avg_ms": k3 * 1e3, "frac": (c3 / k3) / VALU_COMPARE_PEAK,
            "num": r3.num, "den": r3.den}
        del P3t, Q3t
    if extras:
        line["extras"] = extras

    if args.copy_mib:
        a = torch.empty(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        _log(f"[bench] copy calibration: {args.copy_mib} MiB")

    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
