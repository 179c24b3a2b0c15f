"""More than 65536 distinct values in a dimension: the 16-bit code there is
the first sorted position of the point's value shifted right, and the points
that share an origin's code with a smaller value (fewer than 2^shift of them,
ties or not) are moved to their exact orthant after the sweep.  Counts and D
against the oracle, exactly; the profile counter shows that the shifted path
ran."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


def key(r):
    return (r.num, r.den, r.argmax_origin, r.argmax_orthant)


@pytest.fixture(scope="module")
def ctx():
    from paper_2106_13706_amd import native
    c = native.Context(flags=native.DDKS_NO_AUTOTUNE)
    yield c
    c.close()


@pytest.mark.parametrize("n_p,n_q,d,shift", [(40000, 30000, 8, 1), (70000, 60000, 3, 1),
                                             (90000, 50000, 4, 2), (100000, 100001, 2, 2),
                                             (66000, 1, 1, 1)])
def test_matches_oracle(ctx, oracle_mod, n_p, n_q, d, shift):
    g = np.random.default_rng(n_p + d)
    P = g.standard_normal((n_p, d)).astype(np.float32)
    Q = (g.standard_normal((n_q, d)) * 1.1 + 0.05).astype(np.float32)
    if d > 1:
        P[:, 0] = np.rint(P[:, 0] * 4) / 4  # one dimension with few values (no shift there)
    print(f"  shifted n=({n_p},{n_q}) d={d}", flush=True)
    before = ctx.profile()
    r = ctx.distance(P, Q)
    after = ctx.profile()
    assert after["shifted_calls"] == before["shifted_calls"] + 1
    o = oracle_mod.distance(P, Q, counts=False, threads=THREADS)
    assert key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)


def test_counts_exact(ctx, oracle_mod):
    g = np.random.default_rng(77)
    P = g.standard_normal((36000, 3)).astype(np.float32)
    Q = (g.standard_normal((34000, 3)) + 0.1).astype(np.float32)
    Q[:2000] = P[:2000]  # shared points: ties across the samples
    r, counts = ctx.distance(P, Q, counts=True)
    o = oracle_mod.distance(P, Q, counts=True, threads=THREADS)
    assert key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)
    np.testing.assert_array_equal(counts, o.counts)


def test_counts_exact_d8(ctx, oracle_mod):
    """d = 8, where bit 7 of a bin index is stored flipped: every one of the
    256 orthant counts of every origin after the corrections, against the
    oracle (70000 points, shifted codes in the continuous dimensions, dense
    ranks in a rounded one)."""
    g = np.random.default_rng(88)
    P = g.standard_normal((40000, 8)).astype(np.float32)
    Q = (g.standard_normal((30000, 8)) * 1.1).astype(np.float32)
    P[:, 3] = np.rint(P[:, 3] * 2) / 2
    Q[:, 3] = np.rint(Q[:, 3] * 2) / 2
    before = ctx.profile()
    r, counts = ctx.distance(P, Q, counts=True)
    assert ctx.profile()["shifted_calls"] == before["shifted_calls"] + 1
    o = oracle_mod.distance(P, Q, counts=True, threads=THREADS)
    assert key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)
    np.testing.assert_array_equal(counts, o.counts)


def test_heavy_ties_in_a_shifted_dimension(ctx, oracle_mod):
    """66000 distinct values plus 4000 more copies of 10.0 and 3000 of 500.5
    (shift 1 on 73000 points): the tied runs cross code boundaries and sit
    just below other values' origins, and every compare stays exact."""
    g = np.random.default_rng(5)
    x = np.concatenate([np.arange(66000, dtype=np.float32), np.full(4000, 10.0, np.float32),
                        np.full(3000, 500.5, np.float32)])
    x = x[g.permutation(len(x))]
    P, Q = x[:36000, None].copy(), x[36000:, None].copy()
    before = ctx.profile()
    r, counts = ctx.distance(P, Q, counts=True)
    after = ctx.profile()
    assert after["shifted_calls"] == before["shifted_calls"] + 1
    o = oracle_mod.distance(P, Q, counts=True, threads=THREADS)
    assert key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)
    np.testing.assert_array_equal(counts, o.counts)


def test_two_shifted_dimensions_with_shared_groups(ctx, oracle_mod):
    """d = 2, both dimensions shifted, the second a tied copy of the first
    plus 0, 1 or 2, so many points share an origin's code in both dimensions
    at once (each is corrected once)."""
    g = np.random.default_rng(11)
    n = 140000
    Z = np.empty((n, 2), np.float32)
    Z[:, 0] = g.permutation(n).astype(np.float32)           # all distinct
    Z[:, 1] = (Z[:, 0] + g.integers(0, 3, n)).astype(np.float32)  # close to the first
    P, Q = Z[:70000].copy(), Z[70000:].copy()
    before = ctx.profile()
    r, counts = ctx.distance(P, Q, counts=True)
    after = ctx.profile()
    assert after["shifted_calls"] == before["shifted_calls"] + 1
    o = oracle_mod.distance(P, Q, counts=True, threads=THREADS)
    assert key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)
    np.testing.assert_array_equal(counts, o.counts)


def _num_from_counts(counts, n_p, n_q):
    """(num, lowest origin, lowest code) of the per-origin counts."""
    c = counts.astype(np.int64)
    v = np.abs(c[:, :, 0] * n_q - c[:, :, 1] * n_p)
    flat = int(np.argmax(v))  # first maximum: lowest origin, then lowest code
    return int(v.max()), flat // v.shape[1], flat % v.shape[1]


def test_largest_shift(ctx, oracle_mod):
    """N = 2^22 points needs shift 6 in both dimensions, the largest the
    16-bit path takes; one point more and the call runs on fp32 compares.
    Too large for the full oracle: the counts of sampled origins (the argmax,
    the origins next to two heavy ties, random ones) against the oracle's,
    D against the counts and against the fp32 path."""
    n = 1 << 21
    g = np.random.default_rng(22)
    P = g.standard_normal((n, 2)).astype(np.float32)
    Q = (g.standard_normal((n, 2)) * 1.05).astype(np.float32)
    P[:5000, 0] = np.float32(0.25)   # heavy ties inside a shifted dimension
    Q[:3000, 1] = np.float32(-0.5)
    print("  largest shift N=2^22 d=2", flush=True)
    before = ctx.profile()
    r, counts = ctx.distance(P, Q, counts=True)
    after = ctx.profile()
    assert after["shifted_calls"] == before["shifted_calls"] + 1
    assert (r.num, r.argmax_origin, r.argmax_orthant) == _num_from_counts(counts, n, n)
    from paper_2106_13706_amd.native import DDKS_FORCE_F32
    rf = ctx.distance(P, Q, flags=DDKS_FORCE_F32)
    assert key(rf) == key(r)
    Z = np.concatenate([P, Q])
    near = [int(np.argmin(np.where(Z[:, 0] > 0.25, Z[:, 0], np.inf))),
            int(np.argmin(np.where(Z[:, 1] > -0.5, Z[:, 1], np.inf))), 0, n]
    idx = np.unique(np.concatenate([[r.argmax_origin], near, g.integers(0, 2 * n, 120)]))
    np.testing.assert_array_equal(counts[idx], oracle_mod.origin_counts(P, Q, idx))

    # one point more: past the 16-bit codes, the fp32 path (same answer)
    P1, Q1 = P[:, :1].copy(), np.concatenate([Q[:, :1], [[0.125]]]).astype(np.float32)
    before = ctx.profile()
    r1 = ctx.distance(P1, Q1)
    assert ctx.profile()["shifted_calls"] == before["shifted_calls"]
    assert key(ctx.distance(P1, Q1, flags=DDKS_FORCE_F32)) == key(r1)


def test_graph_replays_shifted_codes(oracle_mod):
    """Device-resident inputs past 65536 points run as a captured graph that
    codes every dimension by shifted positions (no host read of the distinct
    counts).  Replays over new contents of the same buffers, with eager calls
    between them, each against the oracle; ties in every dimension included
    (there an eager call would keep the dense ranks)."""
    import torch
    from paper_2106_13706_amd import native
    g = np.random.default_rng(31)
    n_p, n_q, d = 40000, 36000, 3
    P = torch.empty((n_p, d), dtype=torch.float32, device="cuda")
    Q = torch.empty((n_q, d), dtype=torch.float32, device="cuda")
    with native.Context(flags=native.DDKS_NO_AUTOTUNE) as ctx:
        for rep in range(3):
            Ph = g.standard_normal((n_p, d)).astype(np.float32)
            Qh = (g.standard_normal((n_q, d)) * 1.1).astype(np.float32)
            if rep == 1:  # few distinct values in every dimension
                Ph = (np.rint(Ph * 8) / 8).astype(np.float32)
                Qh = (np.rint(Qh * 8) / 8).astype(np.float32)
            P.copy_(torch.from_numpy(Ph))
            Q.copy_(torch.from_numpy(Qh))
            print(f"  graph replay {rep}", flush=True)
            before = ctx.profile()["shifted_calls"]
            r = ctx.distance(P, Q)
            assert ctx.profile()["shifted_calls"] == before + 1
            eager = ctx.distance(Ph, Qh)  # host inputs: the eager path
            o = oracle_mod.distance(Ph, Qh, counts=False, threads=THREADS)
            assert key(r) == key(eager) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)


def test_serving_large_tests_on_shifted_codes(oracle_mod):
    """Serving sweeps solo tests of 65537..131072 points on shifted codes
    (encoded, swept and corrected back to back on the slot's stream), mixed
    with packed and mid-size tests in the same batches, and a larger test on
    fp32 compares; every result against the oracle, and the stats count the
    shifted ones."""
    from paper_2106_13706_amd import native
    g = np.random.default_rng(41)
    shapes = [(40000, 30000, 8), (50000, 50001, 2), (3000, 2000, 3), (45000, 40000, 5),
              (20000, 20000, 4), (65537, 1, 1), (70000, 61072, 3), (70000, 70000, 2)]
    big = sum(1 for a, b, _ in shapes if 65536 < a + b <= 131072)
    reqs = []
    for i, (n_p, n_q, d) in enumerate(shapes):
        P = g.standard_normal((n_p, d)).astype(np.float32)
        Q = (g.standard_normal((n_q, d)) * 1.05 + 0.02).astype(np.float32)
        if i % 3 == 1:
            P[:, 0] = np.rint(P[:, 0] * 4) / 4  # heavy ties in one dimension
        reqs.append((P, Q))
    with native.Context(serve_streams=2) as ctx:
        tickets = [ctx.serve_submit(P, Q) for P, Q in reqs]
        got = [ctx.serve_poll(t, timeout_us=-1) for t in tickets]
        st = ctx.serve_stats()
    assert st["shifted_tests"] == big
    for (P, Q), r in zip(reqs, got):
        print(f"  served n_p={len(P)} n_q={len(Q)} d={P.shape[1]}", flush=True)
        o = oracle_mod.distance(P, Q, counts=False, threads=THREADS)
        assert key(r) == (o.num, o.den, o.argmax_origin, o.argmax_orthant)
