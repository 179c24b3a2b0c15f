"""GPU parity of ddks_distance against the CPU oracle: counts, num, den, D
and argmax bit-for-bit (integer results; tolerance 0).  Needs an MI355X."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
THREADS = max(1, min(16, os.cpu_count() or 1))


def _ctx(**env):
    from paper_2106_13706_amd import native
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return native.Context()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.fixture(scope="module")
def ctx():
    c = _ctx()
    yield c
    c.close()


def check(ctx, oracle_mod, P, Q, counts=True, flags=0):
    print(f"  case n_p={len(P)} n_q={len(Q)} d={P.shape[1]}", flush=True)
    if counts:
        r, c = ctx.distance(P, Q, counts=True, flags=flags)
    else:
        r = ctx.distance(P, Q, flags=flags)
    o = oracle_mod.distance(P, Q, counts=counts, threads=THREADS)
    assert (r.num, r.den, r.argmax_origin, r.argmax_orthant) == (
        o.num, o.den, o.argmax_origin, o.argmax_orthant)
    assert r.D == o.D
    if counts:
        np.testing.assert_array_equal(c, o.counts)
    return r


@pytest.mark.parametrize("name", ["example_a.json", "example_b.json", "example_c.json"])
def test_worked_examples(ctx, oracle_mod, name):
    g = json.load(open(os.path.join(GOLDEN, name)))
    P = np.array(g["P"], np.float32)
    Q = np.array(g["Q"], np.float32)
    r = check(ctx, oracle_mod, P, Q)
    assert (r.num, r.den) == (g["num"], g["den"])


SIZES = [(1, 1), (1, 2), (3, 5), (63, 1), (64, 64), (65, 63), (100, 37), (300, 211),
         (1000, 1), (777, 1234)]


PATHS = {"f32": 0x2, "rank16": 0x10}  # DDKS_FORCE_F32, DDKS_FORCE_RANK16


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("d", range(1, 9))
def test_random_sizes_all_d(ctx, oracle_mod, d, path):
    g = np.random.default_rng(1000 + d)
    for n_p, n_q in SIZES:
        P = g.standard_normal((n_p, d)).astype(np.float32)
        Q = (g.standard_normal((n_q, d)) * 1.1 + 0.2).astype(np.float32)
        check(ctx, oracle_mod, P, Q, flags=PATHS[path])


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
def test_ties_and_signed_zero(ctx, oracle_mod, d, path):
    g = np.random.default_rng(77 + d)
    P = g.integers(-2, 3, size=(301, d)).astype(np.float32)
    Q = g.integers(-1, 3, size=(257, d)).astype(np.float32)
    P[g.random(P.shape) < 0.3] = -0.0
    Q[g.random(Q.shape) < 0.2] = -0.0
    assert np.signbit(P).any() and np.signbit(Q).any()
    check(ctx, oracle_mod, P, Q, flags=PATHS[path])


@pytest.mark.parametrize("path", sorted(PATHS))
def test_subnormals_and_extremes(ctx, oracle_mod, path):
    tiny = np.float32(1e-45)
    vals = np.array([0.0, -0.0, tiny, -tiny, 2 * tiny, 1e-40, -1e-40, 1.1754942e-38,
                     1.1754944e-38, 3.4028235e38, -3.4028235e38, 1.0, -1.0], np.float32)
    g = np.random.default_rng(5)
    for d in (1, 2, 4, 7):
        P = g.choice(vals, size=(150, d)).astype(np.float32)
        Q = g.choice(vals, size=(170, d)).astype(np.float32)
        check(ctx, oracle_mod, P, Q, flags=PATHS[path])


@pytest.mark.parametrize("waves,chunks", [(1, 1), (2, 3), (4, 1), (4, 7), (8, 2), (8, 1),
                                          (12, 1), (12, 3), (16, 1), (16, 3)])
def test_launch_shapes(oracle_mod, waves, chunks):
    c = _ctx(DDKS_FORCE_WAVES=waves, DDKS_FORCE_CHUNKS=chunks)
    try:
        g = np.random.default_rng(waves * 10 + chunks)
        for d in (2, 4, 6, 8):
            P = np.rint(g.standard_normal((2345, d)) * 4).astype(np.float32)
            Q = np.rint(g.standard_normal((1999, d)) * 4 + 0.5).astype(np.float32)
            for flags in PATHS.values():
                check(c, oracle_mod, P, Q, flags=flags)
    finally:
        c.close()


@pytest.mark.parametrize("chunks", [2, 3])
def test_partial_count_formats(oracle_mod, chunks):
    """Chunked plans store each chunk's counts as one 32-bit word per bin and
    lane (16-bit halves) when a chunk holds at most 65535 points, else as two
    words.  140000 points in 2 chunks take the wide form, in 3 chunks the
    packed one; each with dense ranks (a 1/8 grid) and with shifted codes
    (continuous values, whose corrections go to the chunk of the moved point),
    against the oracle."""
    from paper_2106_13706_amd import native
    c = _ctx(DDKS_FORCE_CHUNKS=chunks)
    try:
        g = np.random.default_rng(chunks)
        for grid in (True, False):
            P = g.standard_normal((71000, 2)).astype(np.float32)
            Q = (g.standard_normal((69000, 2)) * 1.1 + 0.03).astype(np.float32)
            if grid:
                P, Q = (np.rint(P * 8) / 8).astype(np.float32), (np.rint(Q * 8) / 8).astype(np.float32)
            before = c.profile()["shifted_calls"]
            check(c, oracle_mod, P, Q, counts=False, flags=native.DDKS_FORCE_RANK16)
            assert c.profile()["shifted_calls"] == before + (0 if grid else 1)
    finally:
        c.close()


def test_wide_partial_counts_d8_shifted(oracle_mod):
    """d = 8, 140000 points in 2 chunks (70000 per chunk: the two-word partial
    counts) on shifted codes: sampled origins' 256 orthant counts against the
    oracle, the maximum against the returned counts, and the same result on
    fp32 compares."""
    from paper_2106_13706_amd import native
    c = _ctx(DDKS_FORCE_CHUNKS=2)
    try:
        g = np.random.default_rng(808)
        P = g.standard_normal((70000, 8)).astype(np.float32)
        Q = (g.standard_normal((70000, 8)) + 0.05).astype(np.float32)
        before = c.profile()["shifted_calls"]
        r, cnt = c.distance(P, Q, counts=True, flags=native.DDKS_FORCE_RANK16)
        assert c.profile()["shifted_calls"] == before + 1
        _check_sampled(oracle_mod, r, cnt, P, Q, seed=8)
        rf = c.distance(P, Q, flags=native.DDKS_FORCE_F32)
        assert (rf.num, rf.argmax_origin, rf.argmax_orthant) == (r.num, r.argmax_origin, r.argmax_orthant)
    finally:
        c.close()


def _check_sampled(oracle_mod, r, c, P, Q, seed):
    """Counts at sampled origins against the oracle; at every origin the
    counts partition both samples and the reported maximum is the maximum of
    the returned counts."""
    n_p, n_q = len(P), len(Q)
    N = n_p + n_q
    g = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([g.integers(0, N, 40), [0, n_p - 1, n_p, N - 1,
                                                            r.argmax_origin]]))
    np.testing.assert_array_equal(c[idx], oracle_mod.origin_counts(P, Q, idx))
    assert (c[:, :, 0].sum(axis=1, dtype=np.int64) == n_p).all()
    assert (c[:, :, 1].sum(axis=1, dtype=np.int64) == n_q).all()
    s = np.abs(c[:, :, 0].astype(np.int64) * n_q - c[:, :, 1].astype(np.int64) * n_p)
    flat = int(np.argmax(s.reshape(-1)))
    assert int(s.reshape(-1)[flat]) == r.num
    assert divmod(flat, s.shape[1]) == (r.argmax_origin, r.argmax_orthant)


@pytest.mark.parametrize("waves,chunks", [(16, 1), (12, 1), (8, 1), (1, 1), (0, 0)])
def test_counter_bound_shapes(oracle_mod, waves, chunks):
    """A first sample of 70000 points in one chunk: 16, 12 or 8 waves need two
    LDS histograms per block so that no 16-bit counter overflows (12 waves:
    waves 0, 2, .. and 1, 3, .. share one each, 6 x 5834 points); one wave
    per block cannot hold it in one chunk, so the planner splits the points.
    (0, 0): the library's own choice.  Every shape must give the same exact
    result."""
    env = {} if waves == 0 else dict(DDKS_FORCE_WAVES=waves, DDKS_FORCE_CHUNKS=chunks)
    c = _ctx(**env)
    try:
        g = np.random.default_rng(31)
        d = 3
        P = g.standard_normal((70000, d)).astype(np.float32)
        Q = (g.standard_normal((3001, d)) * 1.2).astype(np.float32)
        for flags in PATHS.values():
            print(f"  counter-bound waves={waves} chunks={chunks} flags={flags}", flush=True)
            r, cnt = c.distance(P, Q, counts=True, flags=flags)
            _check_sampled(oracle_mod, r, cnt, P, Q, seed=waves + flags)
            r2 = c.distance(Q, P, flags=flags)
            assert r2.num == r.num
    finally:
        c.close()


def test_nonfinite_rejected(ctx):
    from paper_2106_13706_amd import native
    P = np.zeros((10, 3), np.float32)
    Q = np.ones((10, 3), np.float32)
    for bad in (np.nan, np.inf, -np.inf):
        P2 = P.copy()
        P2[4, 1] = bad
        with pytest.raises(native.DDKSError) as e:
            ctx.distance(P2, Q)
        assert e.value.status == native.DDKS_E_NONFINITE
    # the context keeps working after a rejected call
    assert ctx.distance(P, Q).num == 100


def test_nonfinite_rejected_on_the_graph_path(oracle_mod):
    """Device inputs of 8192..65536 points replay as a graph whose rank
    encoding reads P and Q itself (no ingested copy): a NaN or infinity in
    either sample, in the first or last point, is still rejected, a -0 still
    ties with +0, and the replays before and after stay exact."""
    import torch
    from paper_2106_13706_amd import native
    g = np.random.default_rng(9)
    P = np.rint(g.standard_normal((6000, 3)) * 4).astype(np.float32)
    Q = np.rint(g.standard_normal((5000, 3)) * 4 + 1).astype(np.float32)
    P[P == 0] = -0.0
    o = oracle_mod.distance(P, Q, threads=THREADS)
    Pd, Qd = torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda()
    with native.Context() as c:
        key = lambda r: (r.num, r.argmax_origin, r.argmax_orthant)
        assert key(c.distance(Pd, Qd)) == (o.num, o.argmax_origin, o.argmax_orthant)
        for which, at in (("P", (0, 0)), ("Q", (4999, 2)), ("P", (5999, 1))):
            for bad in (np.nan, np.inf, -np.inf):
                X = Pd if which == "P" else Qd
                keep = X[at].item()
                X[at] = float(bad)
                torch.cuda.synchronize()  # the library runs on its own stream
                with pytest.raises(native.DDKSError) as e:
                    c.distance(Pd, Qd)
                assert e.value.status == native.DDKS_E_NONFINITE
                X[at] = keep
                torch.cuda.synchronize()
        assert key(c.distance(Pd, Qd)) == (o.num, o.argmax_origin, o.argmax_orthant)


def test_invalid_arguments(ctx):
    from paper_2106_13706_amd import native
    with pytest.raises(native.DDKSError) as e:
        ctx.distance(np.zeros((3, 9), np.float32), np.zeros((3, 9), np.float32))
    assert e.value.status == native.DDKS_E_INVALID_ARG
    with pytest.raises(native.DDKSError) as e:
        ctx.distance(np.zeros((0, 2), np.float32), np.zeros((3, 2), np.float32))
    assert e.value.status == native.DDKS_E_INVALID_ARG


def test_device_pointers(oracle_mod):
    import torch
    from paper_2106_13706_amd import native
    s = torch.cuda.current_stream()
    c = native.Context(stream=s)
    try:
        g = np.random.default_rng(3)
        P = g.standard_normal((1500, 4)).astype(np.float32)
        Q = g.standard_normal((1700, 4)).astype(np.float32)
        Pt = torch.from_numpy(P).cuda()
        Qt = torch.from_numpy(Q).cuda()
        r, cnt = c.distance(Pt, Qt, counts=True)
        o = oracle_mod.distance(P, Q, counts=True, threads=THREADS)
        assert (r.num, r.argmax_origin, r.argmax_orthant) == (o.num, o.argmax_origin,
                                                              o.argmax_orthant)
        np.testing.assert_array_equal(cnt.cpu().numpy().view(np.uint32), o.counts)
    finally:
        c.close()


@pytest.mark.parametrize("n_p,n_q", [(2600, 2200), (5000, 4000)])
def test_result_wait_with_device_counts(oracle_mod, n_p, n_q):
    """A call whose only host output is the result returns once the final
    kernel has written it, which can be just before that kernel ends on the
    library's own stream.  Counts written to device memory by the earlier
    kernels must be complete by then: each call's counts are read on torch's
    stream (not the library's) right after it returns, over captured and
    replayed calls with the inputs rewritten in place (fp32 path at 4800
    points, 16-bit codes at 9000), against the oracle."""
    import torch
    from paper_2106_13706_amd import native
    c = native.Context()  # library-owned stream
    try:
        g = np.random.default_rng(91 + n_p)
        d = 4
        Pt = torch.empty((n_p, d), dtype=torch.float32, device="cuda")
        Qt = torch.empty((n_q, d), dtype=torch.float32, device="cuda")
        for rep in range(4):
            P = np.rint(g.standard_normal((n_p, d)) * 6).astype(np.float32)
            Q = np.rint(g.standard_normal((n_q, d)) * 6 + 1).astype(np.float32)
            Pt.copy_(torch.from_numpy(P))
            Qt.copy_(torch.from_numpy(Q))
            torch.cuda.synchronize()  # the library's stream does not follow torch's
            print(f"  result wait n_p={n_p} n_q={n_q} rep={rep}", flush=True)
            r, cnt = c.distance(Pt, Qt, counts=True)
            got = cnt.cpu().numpy().view(np.uint32)
            o = oracle_mod.distance(P, Q, counts=True, threads=THREADS)
            assert (r.num, r.argmax_origin, r.argmax_orthant) == (o.num, o.argmax_origin,
                                                                  o.argmax_orthant)
            np.testing.assert_array_equal(got, o.counts)
    finally:
        c.close()


@pytest.mark.parametrize("flags", [0x0, 0x2, 0x10])
def test_graph_replays(oracle_mod, flags):
    """Device-resident inputs: the call is captured once and then replayed.
    Replays see data rewritten in place, eager calls in between do not
    disturb them, and a new size is captured again; every result against the
    oracle."""
    import torch
    from paper_2106_13706_amd import native
    c = native.Context(stream=torch.cuda.current_stream(), flags=native.DDKS_PROFILE_KERNELS)
    try:
        g = np.random.default_rng(40 + flags)
        d = 3
        Pt = torch.empty((3000, d), dtype=torch.float32, device="cuda")
        Qt = torch.empty((2500, d), dtype=torch.float32, device="cuda")
        key = lambda r: (r.num, r.den, r.argmax_origin, r.argmax_orthant)
        for rep in range(4):
            P = (np.rint(g.standard_normal((3000, d)) * 4) / 4).astype(np.float32)
            Q = (np.rint(g.standard_normal((2500, d)) * 4 + 1) / 4).astype(np.float32)
            Pt.copy_(torch.from_numpy(P))
            Qt.copy_(torch.from_numpy(Q))
            print(f"  replay {rep} flags={flags}", flush=True)
            r = c.distance(Pt, Qt, flags=flags)
            assert key(r) == key(oracle_mod.distance(P, Q, counts=False, threads=THREADS))
            if rep == 1:
                r2 = c.distance(P[:100], Q[:50], flags=flags)  # eager: host inputs
                assert key(r2) == key(oracle_mod.distance(P[:100], Q[:50], counts=False))
        r = c.distance(Pt[:2000], Qt[:1000], flags=flags)  # new key: captured again
        assert key(r) == key(oracle_mod.distance(P[:2000], Q[:1000], counts=False,
                                                 threads=THREADS))
        prof = c.profile()
        assert prof["sweeps"] == 6
        assert prof["graph_calls"] == 5
    finally:
        c.close()


# ------------------------------------------------------------- the workloads

def test_workload_gaussian_shift_d3_500(ctx, oracle_mod):
    from paper_2106_13706_amd import workloads
    P, Q = workloads.gaussian_shift()
    check(ctx, oracle_mod, P, Q)


def test_workload_gaussian_scale_d4_20000(ctx, oracle_mod):
    from paper_2106_13706_amd import workloads
    P, Q = workloads.gaussian_scale()
    check(ctx, oracle_mod, P, Q)


@pytest.mark.parametrize("path", sorted(PATHS))
def test_workload_gaussian_scale_d4_20000_paths(ctx, oracle_mod, path):
    from paper_2106_13706_amd import workloads
    P, Q = workloads.gaussian_scale()
    check(ctx, oracle_mod, P, Q, counts=False, flags=PATHS[path])


def test_workload_mixture_grid_d6_scaled(ctx, oracle_mod):
    """Same recipe as the 100000-point workload at 1/10 the size: full parity."""
    from paper_2106_13706_amd import workloads
    P, Q = workloads.mixture_grid(n_p=10000, n_q=10000)
    assert np.signbit(P).any()
    check(ctx, oracle_mod, P, Q)
    check(ctx, oracle_mod, P, Q, counts=False, flags=PATHS["f32"])


@pytest.mark.parametrize("n_p,n_q,d", [(4095, 0, 2), (2048, 2048, 3), (4000, 97, 2),
                                       (4097, 4096, 1), (32768, 32768, 2), (2047, 1, 2),
                                       (2049, 1, 5), (6143, 1, 3), (3000, 3145, 4)])
def test_rank16_tile_edges(ctx, oracle_mod, n_p, n_q, d):
    """Rank encoding at tile boundaries (4096 keys per sorted tile up to 65536
    points; also the multiples of 2048) up to the largest size whose ranks
    always fit 16 bits (65536 points); ties and signed zeros so that equal
    values span tiles."""
    g = np.random.default_rng(n_p + n_q)
    n_q = max(n_q, 1)
    P = (np.rint(g.standard_normal((n_p, d)) * 40) / 8).astype(np.float32)
    Q = (np.rint(g.standard_normal((n_q, d)) * 40 + 3) / 8).astype(np.float32)
    P[P == 0] = -0.0
    check(ctx, oracle_mod, P, Q, counts=n_p + n_q < 20000, flags=PATHS["rank16"])


def test_rank16_dense_path_and_fallback(ctx, oracle_mod):
    """More than 65536 points: with few distinct values the dense ranks fit
    16 bits; with more than 65536 distinct values in a dimension that
    dimension is coded by shifted sorted positions and corrected after the
    sweep.  Both must match the oracle."""
    g = np.random.default_rng(44)
    P = np.rint(g.standard_normal((40000, 2)) * 30).astype(np.float32)
    Q = np.rint(g.standard_normal((30001, 2)) * 30 + 3).astype(np.float32)
    check(ctx, oracle_mod, P, Q, counts=False, flags=PATHS["rank16"])
    P = g.standard_normal((36000, 2)).astype(np.float32)
    Q = g.standard_normal((34000, 2)).astype(np.float32)
    assert len(np.unique(np.concatenate([P, Q])[:, 0])) > 65536
    check(ctx, oracle_mod, P, Q, counts=False, flags=PATHS["rank16"])


def test_workload_mixture_grid_d6_100000_sampled(ctx, oracle_mod):
    """Full size: counts at sampled origins against the oracle, and properties
    that hold at any size for the rest (count partition, self-count, the
    reported maximum is the maximum of the returned counts, symmetry)."""
    from paper_2106_13706_amd import workloads
    P, Q = workloads.mixture_grid()
    n_p, n_q = len(P), len(Q)
    N = n_p + n_q
    r, c = ctx.distance(P, Q, counts=True)
    g = np.random.default_rng(0)
    idx = np.unique(np.concatenate([g.integers(0, N, 48), [0, n_p - 1, n_p, N - 1,
                                                            r.argmax_origin]]))
    np.testing.assert_array_equal(c[idx], oracle_mod.origin_counts(P, Q, idx))
    assert (c[:, :, 0].sum(axis=1, dtype=np.int64) == n_p).all()
    assert (c[:, :, 1].sum(axis=1, dtype=np.int64) == n_q).all()
    assert (c[:n_p, -1, 0] >= 1).all() and (c[n_p:, -1, 1] >= 1).all()
    s = np.abs(c[:, :, 0].astype(np.int64) * n_q - c[:, :, 1].astype(np.int64) * n_p)
    flat = int(np.argmax(s.reshape(-1)))
    assert int(s.reshape(-1)[flat]) == r.num
    assert divmod(flat, s.shape[1]) == (r.argmax_origin, r.argmax_orthant)
    r2 = ctx.distance(Q, P)
    assert r2.num == r.num and r2.den == r.den
