"""GPU serving loop (continuous batching): every result equals the oracle's
and the single-test path's for the same inputs, alone or in a mix of
dimensions and sizes; admission under a memory budget, queue limits and
error paths.  Integer results, tolerance 0."""
import os
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


def _mix(seed, count, nmax=3000):
    g = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        d = int(g.integers(1, 9))
        n_p = int(np.rint(np.exp(g.uniform(np.log(1), np.log(nmax)))))
        n_q = int(np.rint(np.exp(g.uniform(np.log(1), np.log(nmax)))))
        P = g.standard_normal((n_p, d)).astype(np.float32)
        Q = (g.standard_normal((n_q, d)) + g.uniform(0, 0.3)).astype(np.float32)
        if g.random() < 0.3:
            P = np.rint(P * 2) / 2
            Q = np.rint(Q * 2) / 2
            P[P == 0] = -0.0
        reqs.append((P.astype(np.float32), Q.astype(np.float32)))
    return reqs


def _ctx_env(env, **kw):
    """A context created with the environment overrides in env (restored after)."""
    import os
    from paper_2106_13706_amd import native
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return native.Context(**kw)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _key(r):
    return (r.num, r.den, r.argmax_origin, r.argmax_orthant)


def test_mix_matches_oracle_and_single_path(oracle_mod):
    from paper_2106_13706_amd import native
    reqs = _mix(1, 120)
    with native.Context() as ctx:
        tickets = [ctx.serve_submit(P, Q) for P, Q in reqs]
        assert all(t > 0 for t in tickets)
        got = [ctx.serve_poll(t) for t in tickets]
        alone = []
        for P, Q in reqs:
            t = ctx.serve_submit(P, Q)
            alone.append(ctx.serve_poll(t))
        single = [ctx.distance(P, Q) for P, Q in reqs]
        st = ctx.serve_stats()
    for (P, Q), a, b, s in zip(reqs, got, alone, single):
        o = oracle_mod.distance(P, Q, threads=THREADS)
        assert _key(a) == _key(b) == _key(s) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)
        assert a.D == o.D
    assert st["completed"] == 240 and st["submitted"] == 240
    assert st["launches"] >= 2 and st["p99_latency_us"] >= st["p50_latency_us"] > 0
    assert 0 < st["busy_us"] <= st["p99_latency_us"] * st["launches"]


def test_concurrent_submitters(oracle_mod):
    from paper_2106_13706_amd import native
    reqs = _mix(2, 64, nmax=5000)
    out = {}
    with native.Context(serve_streams=3) as ctx:
        def worker(idx):
            for i in idx:
                P, Q = reqs[i]
                out[i] = ctx.serve_poll(ctx.serve_submit(P, Q))
        ts = [threading.Thread(target=worker, args=(range(k, len(reqs), 4),)) for k in range(4)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    for i, (P, Q) in enumerate(reqs):
        o = oracle_mod.distance(P, Q, threads=THREADS)
        assert _key(out[i]) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)


def test_memory_budget_admission(oracle_mod):
    """A budget that holds only a few requests at once: all still complete
    (admitted as memory frees up); one that can never fit is refused."""
    from paper_2106_13706_amd import native
    g = np.random.default_rng(3)
    reqs = [(g.standard_normal((10000, 8)).astype(np.float32),
             g.standard_normal((10000, 8)).astype(np.float32)) for _ in range(6)]
    with native.Context() as ref:
        expected = [_key(ref.distance(P, Q)) for P, Q in reqs]
    # 2 MiB of budget: each request needs 0.64 MB, so at most three are resident
    with native.Context(mem_budget=2 << 20) as ctx:
        tickets = [ctx.serve_submit(P, Q) for P, Q in reqs]
        res = [ctx.serve_poll(t) for t in tickets]
        assert [_key(r) for r in res] == expected
        big = g.standard_normal((130000, 8)).astype(np.float32)
        with pytest.raises(native.DDKSError) as e:
            ctx.serve_submit(big[:65000], big[65000:])
        assert e.value.status == native.DDKS_E_NOMEM
        assert ctx.serve_stats()["rejected_nomem"] == 1


def test_workload_serving_stratified(oracle_mod):
    """The 10^4-test serving stream: a seeded stratified subset served
    together and checked against the oracle -- every test with N <= 8192 among
    the first 1200 of the stream, plus for each d the first four tests with
    8192 < N <= 32768 (these take the rank-encoded path from N = 16384)."""
    from paper_2106_13706_amd import native, workloads
    stream = workloads.serving_stream(materialize=False)
    reqs = stream.requests
    N = [r.P.shape[0] + r.Q.shape[0] for r in reqs]
    pick = [i for i in range(1200) if N[i] <= 8192]
    for d in range(2, 9):
        pick += [i for i in range(len(reqs)) if reqs[i].d == d and 8192 < N[i] <= 32768][:4]
    assert len(pick) >= 400
    data = [workloads.materialize(reqs[i]) for i in pick]
    with native.Context() as ctx:
        tickets = [ctx.serve_submit(P, Q) for P, Q in data]
        got = [ctx.serve_poll(t) for t in tickets]
    for i, (P, Q), r in zip(pick, data, got):
        o = oracle_mod.distance(P, Q, counts=False, threads=THREADS)
        assert _key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant), (i, P.shape, Q.shape)


def test_queue_full_and_errors():
    from paper_2106_13706_amd import native
    g = np.random.default_rng(4)
    with native.Context(serve_queue_depth=3) as ctx:
        P = g.standard_normal((50, 3)).astype(np.float32)
        tickets = [ctx.serve_submit(P, P + 1) for _ in range(3)]
        assert ctx.serve_submit(P, P + 1) == -1  # DDKS_E_AGAIN
        assert ctx.serve_stats()["rejected_again"] == 1
        for t in tickets:
            assert ctx.serve_poll(t) is not None
        assert ctx.serve_submit(P, P + 1) > 0  # room again after collection
        with pytest.raises(native.DDKSError) as e:
            ctx.serve_poll(987654)
        assert e.value.status == native.DDKS_E_UNKNOWN_TICKET
        bad = P.copy()
        bad[3, 1] = np.nan
        with pytest.raises(native.DDKSError) as e:
            ctx.serve_submit(bad, P)
        assert e.value.status == native.DDKS_E_NONFINITE
        with pytest.raises(native.DDKSError) as e:
            ctx.serve_submit(np.zeros((3, 9), np.float32), np.zeros((3, 9), np.float32))
        assert e.value.status == native.DDKS_E_INVALID_ARG


def test_rank_encoded_requests(oracle_mod):
    """Mid-size tests (16384 <= N <= 65536) are rank encoded on the device
    and swept with 16-bit compares, larger ones up to 131072 points on
    shifted codes; smaller ones keep fp32.  A mix of all three, with ties and
    signed zeros in some, against the oracle."""
    from paper_2106_13706_amd import native
    g = np.random.default_rng(21)
    shapes = [(9000, 8000, 3), (20000, 15000, 5), (30000, 35000, 2), (12000, 5000, 8),
              (3000, 2000, 3), (70000, 100, 4), (16384, 16384, 1), (8192, 8193, 6)]
    reqs = []
    for i, (n_p, n_q, d) in enumerate(shapes):
        P = g.standard_normal((n_p, d)).astype(np.float32)
        Q = (g.standard_normal((n_q, d)) + 0.2).astype(np.float32)
        if i % 2:
            P = (np.rint(P * 3) / 3).astype(np.float32)
            Q = (np.rint(Q * 3) / 3).astype(np.float32)
            P[P == 0] = -0.0
        reqs.append((P, Q))
    with native.Context() as ctx:
        tickets = [ctx.serve_submit(P, Q) for P, Q in reqs]
        for (P, Q), t in zip(reqs, tickets):
            print(f"  served n_p={len(P)} n_q={len(Q)} d={P.shape[1]}", flush=True)
            r = ctx.serve_poll(t, timeout_us=-1)
            o = oracle_mod.distance(P, Q, counts=False, threads=THREADS)
            assert _key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)


def test_sample_size_bounds(oracle_mod):
    """d = 8 with a 70000-point first sample needs two LDS histograms per
    block of the packed sweep; it is served and matches the oracle.  Twice that
    cannot be held by any admissible block shape and is refused with
    DDKS_E_NOT_SUPPORTED before anything is queued."""
    from paper_2106_13706_amd import native
    g = np.random.default_rng(8)
    with native.Context() as ctx:
        P = g.standard_normal((70000, 8)).astype(np.float32)
        Q = (g.standard_normal((100, 8)) + 0.5).astype(np.float32)
        t = ctx.serve_submit(P, Q)
        r = ctx.serve_poll(t, timeout_us=-1)
        o = oracle_mod.distance(P, Q, counts=False, threads=THREADS)
        assert _key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)
        big = np.zeros((140000, 8), np.float32)
        with pytest.raises(native.DDKSError) as e:
            ctx.serve_submit(big, Q)
        assert e.value.status == native.DDKS_E_NOT_SUPPORTED
        assert ctx.serve_stats()["submitted"] == 1


def test_poll_timeout_reports_pending():
    from paper_2106_13706_amd import native
    g = np.random.default_rng(5)
    with native.Context() as ctx:
        P = g.standard_normal((60000, 8)).astype(np.float32)
        Q = g.standard_normal((60000, 8)).astype(np.float32)
        t = ctx.serve_submit(P, Q)
        assert ctx.serve_poll(t, timeout_us=0) is None
        r = ctx.serve_poll(t, timeout_us=-1)
        assert r is not None and r.den == 60000 * 60000
        assert _key(r) == _key(ctx.distance(P, Q))


def test_destroy_with_outstanding_requests():
    from paper_2106_13706_amd import native
    g = np.random.default_rng(6)
    ctx = native.Context()
    for _ in range(20):
        ctx.serve_submit(g.standard_normal((3000, 4)).astype(np.float32),
                         g.standard_normal((2000, 4)).astype(np.float32))
    ctx.close()  # drains the serving loop and frees everything


def test_significance_in_serving(oracle_mod):
    """Served tests that ask for the analytic significance (Sec. 3), binomial
    and Poisson, mixed with tests that do not: num and argmax equal the
    oracle's; S equals the plain call's S exactly (same counts, same kernels,
    fixed-order reduction) and the oracle's within the relative bound of the
    significance tests; S = -1 where it was not asked for."""
    import math
    from paper_2106_13706_amd import native
    g = np.random.default_rng(31)
    cases = []
    for k in range(24):
        d = int(g.integers(2, 7))
        n_p, n_q = int(g.integers(20, 2500)), int(g.integers(20, 2500))
        if k == 5:
            n_p, n_q = 12000, 9000  # a size served on the rank-16 path
        P = g.standard_normal((n_p, d)).astype(np.float32)
        Q = (g.standard_normal((n_q, d)) + g.uniform(0, 0.3)).astype(np.float32)
        flags = [0, native.DDKS_WITH_SIGNIFICANCE,
                 native.DDKS_WITH_SIGNIFICANCE | native.DDKS_SIG_POISSON][k % 3]
        cases.append((P, Q, flags))
    with native.Context() as ctx:
        tickets = [ctx.serve_submit(P, Q, flags) for P, Q, flags in cases]
        got = [ctx.serve_poll(t) for t in tickets]
        plain = [ctx.distance(P, Q, flags=flags) for P, Q, flags in cases]
        with pytest.raises(native.DDKSError) as e:
            ctx.serve_submit(cases[0][0], cases[0][1], native.DDKS_FORCE_F32)
        assert e.value.status == native.DDKS_E_INVALID_ARG
    U = 2.0 ** -53
    for (P, Q, flags), r, p in zip(cases, got, plain):
        n_p, n_q, d = len(P), len(Q), P.shape[1]
        o = oracle_mod.distance(P, Q, counts=True, threads=THREADS)
        assert _key(r) == _key(p) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)
        if not flags:
            assert r.S == -1.0
            continue
        model = "poisson" if flags & native.DDKS_SIG_POISSON else "binomial"
        So = oracle_mod.significance(o.counts, n_p, n_q, d, o.num, model)
        print(f"  {model} d={d} n=({n_p},{n_q}): served S={r.S!r} plain={p.S!r} oracle={So!r}",
              flush=True)
        assert r.S == p.S
        rtol = 128 * U * math.lgamma(max(n_p, n_q) + 1.0) + 1e-12
        assert abs(r.S - So) <= rtol * So + o.counts.size * 1e-304


@pytest.mark.parametrize("waves", ["4", "16"])
def test_forced_packed_waves(oracle_mod, waves):
    """The packed sweep under each admissible block shape (the tuner picks
    among 4, 8 and 16 waves): a mix of dimensions and sizes against the
    oracle."""
    from paper_2106_13706_amd import native
    reqs = _mix(50 + int(waves), 80)
    old = os.environ.get("DDKS_FORCE_PACKED_WAVES")
    os.environ["DDKS_FORCE_PACKED_WAVES"] = waves
    try:
        ctx = native.Context()
    finally:
        if old is None:
            os.environ.pop("DDKS_FORCE_PACKED_WAVES")
        else:
            os.environ["DDKS_FORCE_PACKED_WAVES"] = old
    try:
        tickets = [ctx.serve_submit(P, Q) for P, Q in reqs]
        got = [ctx.serve_poll(t) for t in tickets]
    finally:
        ctx.close()
    for (P, Q), r in zip(reqs, got):
        o = oracle_mod.distance(P, Q, threads=THREADS)
        assert _key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)


def test_packed_waves_tuned_and_cached(oracle_mod, tmp_path):
    """A burst of small tests of one dimension fills packed launches large
    enough to tune their block shape, which lands in the cache file (kind
    20 + path); results match the oracle."""
    from paper_2106_13706_amd import native
    g = np.random.default_rng(91)
    reqs = []
    for _ in range(300):
        n_p, n_q = int(g.integers(1500, 4000)), int(g.integers(1500, 4000))
        reqs.append((g.standard_normal((n_p, 3)).astype(np.float32),
                     (g.standard_normal((n_q, 3)) + 0.1).astype(np.float32)))
    cache = tmp_path / "tune.txt"
    # the first launch waits for the whole burst, so that one packed run holds
    # enough work to be tuned (whatever the pace of the submissions)
    with _ctx_env({"DDKS_SERVE_HOLD": str(len(reqs))}, tune_cache=str(cache)) as ctx:
        tickets = [ctx.serve_submit(P, Q) for P, Q in reqs]
        got = [ctx.serve_poll(t) for t in tickets]
        assert ctx.serve_stats()["launches"] >= 1
    for (P, Q), r in zip(reqs[::10], got[::10]):
        o = oracle_mod.distance(P, Q, threads=THREADS)
        assert _key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)
    lines = [list(map(int, l.split())) for l in cache.read_text().split("\n") if l.strip()]
    print(f"  cache: {lines}", flush=True)
    packed = [l for l in lines if l[0] in (20, 21) and l[1] == 3]
    assert packed and all(l[3] in (4, 8, 16) for l in packed)
