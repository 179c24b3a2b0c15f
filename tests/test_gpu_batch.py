"""GPU parity of ddks_permutation_batch (the permutation test of Sec. 3 and
Sec. 4.2) against the CPU oracle, which rebuilds every relabelled pair of
samples and re-runs the definition.  Integer results, tolerance 0."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))
PATHS = {"f32": 0x2, "rank16": 0x10}


@pytest.fixture(scope="module")
def ctx():
    from paper_2106_13706_amd import native
    c = native.Context()
    yield c
    c.close()


def _rows(g, n, n_p, B):
    m = np.zeros((B, n), bool)
    for b in range(B):
        m[b, g.permutation(n)[:n_p]] = True
    return m


@pytest.mark.parametrize("path", sorted(PATHS))
@pytest.mark.parametrize("d,n,n_p,B", [(1, 40, 17, 9), (2, 130, 64, 37), (3, 257, 100, 41),
                                       (5, 300, 150, 33), (6, 200, 73, 8), (7, 129, 64, 5),
                                       (8, 100, 50, 6)])
def test_all_rows_small(ctx, oracle_mod, path, d, n, n_p, B):
    g = np.random.default_rng(d * 1000 + n)
    Z = np.rint(g.standard_normal((n, d)) * 3).astype(np.float32)
    Z[g.random(Z.shape) < 0.1] = -0.0
    masks = _rows(g, n, n_p, B)
    words = oracle_mod.labels_to_words(masks)
    print(f"  batch d={d} n={n} n_p={n_p} B={B} path={path}", flush=True)
    nums, obs, summ = ctx.permutation_batch(Z, n_p, words, flags=PATHS[path])
    exp = oracle_mod.permutation(Z, n_p, words, threads=THREADS)
    np.testing.assert_array_equal(nums, exp)
    o = oracle_mod.distance(Z[:n_p], Z[n_p:], threads=THREADS)
    assert (obs.num, obs.den, obs.argmax_origin, obs.argmax_orthant) == (
        o.num, o.den, o.argmax_origin, o.argmax_orthant)
    p, frac = oracle_mod.pvalue(exp, o.num)
    assert summ["B"] == B and summ["p_value"] == p and summ["fraction"] == frac


def test_malformed_rows_rejected(ctx, oracle_mod):
    from paper_2106_13706_amd import native
    g = np.random.default_rng(2)
    n, n_p = 70, 30
    Z = g.standard_normal((n, 2)).astype(np.float32)
    good = oracle_mod.labels_to_words(_rows(g, n, n_p, 3))
    bad = good.copy()
    bad[1, 0] ^= 1  # one bit too many or too few
    with pytest.raises(native.DDKSError) as e:
        ctx.permutation_batch(Z, n_p, bad)
    assert e.value.status == native.DDKS_E_INVALID_ARG
    stray = good.copy()
    first = int(np.flatnonzero(_unpack(stray[2], n))[0])
    stray[2, first // 32] &= ~np.uint32(1 << (first % 32))
    stray[2, -1] |= np.uint32(1 << 31)  # a bit beyond n (n = 70 -> word 2 bit 31 is point 95)
    with pytest.raises(native.DDKSError):
        ctx.permutation_batch(Z, n_p, stray)
    nums, _, _ = ctx.permutation_batch(Z, n_p, good)  # the context still works
    np.testing.assert_array_equal(nums, oracle_mod.permutation(Z, n_p, good))


def _unpack(row, n):
    bits = np.zeros(len(row) * 32, bool)
    for w, v in enumerate(row):
        for t in range(32):
            bits[w * 32 + t] = (int(v) >> t) & 1
    return bits[:n]


def test_observed_only(ctx, oracle_mod):
    g = np.random.default_rng(4)
    Z = g.standard_normal((90, 3)).astype(np.float32)
    nums, obs, summ = ctx.permutation_batch(Z, 40, np.zeros((0, 3), np.uint32))
    assert nums.size == 0 and summ["B"] == 0
    assert obs.num == oracle_mod.distance(Z[:40], Z[40:]).num


def test_workload_permutation_d5_8192x1024(ctx, oracle_mod):
    """Full workload: every relabelling row on the GPU, sampled rows and the
    observed split on the oracle; a second call replays the captured graph and
    must give identical numerators, also with other work in between."""
    from paper_2106_13706_amd import workloads
    Z, n_p, labels = workloads.permutation()
    nums, obs, summ = ctx.permutation_batch(Z, n_p, labels)
    rows = [0, 1, 511, 1023] + list(np.random.default_rng(9).integers(0, 1024, 8))
    exp = oracle_mod.permutation(Z, n_p, labels[rows], threads=THREADS)
    np.testing.assert_array_equal(nums[rows], exp)
    o = oracle_mod.distance(Z[:n_p], Z[n_p:], threads=THREADS)
    assert obs.num == o.num and obs.argmax_origin == o.argmax_origin
    assert summ["n_ge"] == int(np.count_nonzero(nums >= o.num))
    for rep in range(3):
        ctx.distance(Z[:1000], Z[1000:2100])  # eager work between replays
        nums2, obs2, summ2 = ctx.permutation_batch(Z, n_p, labels)
        np.testing.assert_array_equal(nums2, nums)
        assert obs2.num == obs.num and summ2 == summ


def test_device_pointers(oracle_mod):
    import torch
    from paper_2106_13706_amd import native
    c = native.Context(stream=torch.cuda.current_stream())
    try:
        g = np.random.default_rng(12)
        n, n_p, d, B = 500, 211, 4, 23
        Z = g.standard_normal((n, d)).astype(np.float32)
        words = oracle_mod.labels_to_words(_rows(g, n, n_p, B))
        Zt = torch.from_numpy(Z).cuda()
        Lt = torch.from_numpy(words.view(np.int32)).cuda()
        nums, obs, _ = c.permutation_batch(Zt, n_p, Lt)
        np.testing.assert_array_equal(nums.cpu().numpy().view(np.uint64),
                                      oracle_mod.permutation(Z, n_p, words, threads=THREADS))
    finally:
        c.close()


def _ctx_env(env, **kw):
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


@pytest.mark.parametrize("shape", ["4:4", "16:4", "4:8", "16:8"])  # waves:relabellings per block
@pytest.mark.parametrize("d", [3, 5, 7])
def test_forced_permutation_shapes(oracle_mod, shape, d):
    """Every relabelling row against the oracle under each admissible shape of
    the permutation kernel (the tuner picks among these); shapes a dimension
    does not admit (8 relabellings per block past d = 6) fall back to the
    default and must still be right."""
    g = np.random.default_rng(70 + d)
    n, n_p, B = 1500, 700, 45
    Z = np.rint(g.standard_normal((n, d)) * 6).astype(np.float32)
    words = oracle_mod.labels_to_words(_rows(g, n, n_p, B))
    ctx = _ctx_env({"DDKS_FORCE_PERM": shape})
    try:
        print(f"  shape {shape} d={d}", flush=True)
        for path in sorted(PATHS):
            nums, obs, _ = ctx.permutation_batch(Z, n_p, words, flags=PATHS[path])
            np.testing.assert_array_equal(nums, oracle_mod.permutation(Z, n_p, words, threads=THREADS))
            assert obs.num == oracle_mod.distance(Z[:n_p], Z[n_p:], threads=THREADS).num
    finally:
        ctx.close()


def test_permutation_shape_tuned_and_cached(oracle_mod, tmp_path):
    """A sizeable batch tunes the permutation kernel's shape once and records
    it in the cache file (kind 10 + path: waves, relabellings per block); the
    tuned call and a replay still match the oracle."""
    from paper_2106_13706_amd import native
    g = np.random.default_rng(81)
    n, n_p, B, d = 6000, 3000, 96, 4
    Z = g.standard_normal((n, d)).astype(np.float32)
    words = oracle_mod.labels_to_words(_rows(g, n, n_p, B))
    cache = tmp_path / "tune.txt"
    exp = oracle_mod.permutation(Z, n_p, words, threads=THREADS)
    with native.Context(tune_cache=str(cache)) as ctx:
        for _ in range(2):
            nums, _, _ = ctx.permutation_batch(Z, n_p, words)
            np.testing.assert_array_equal(nums, exp)
    lines = [list(map(int, l.split())) for l in cache.read_text().split("\n") if l.strip()]
    perm = [l for l in lines if l[0] in (10, 11) and l[1] == d]
    print(f"  cache: {lines}", flush=True)
    assert len(perm) == 1 and perm[0][3] in (4, 8, 16) and perm[0][4] in (4, 8)
