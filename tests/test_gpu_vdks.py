"""GPU vdKS (Sec. 2.2.2, Alg. 1) against the CPU oracle: the statistic, the
lowest maximising voxel key and orthant, and the number of filled voxels,
all exactly (integer results, tolerance 0)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2106_13706_amd import native
    c = native.Context()
    yield c
    c.close()


def check(ctx, oracle_mod, P, Q, V, **kw):
    print(f"  vdks n=({len(P)},{len(Q)}) d={P.shape[1]} V={V}", flush=True)
    r, nf = ctx.vdks(P, Q, V, **kw)
    o = oracle_mod.vdks(P, Q, V)
    assert (r.num, r.den, r.argmax_origin, r.argmax_orthant, nf) == (
        o.num, o.den, o.argmax_voxel, o.argmax_orthant, o.n_filled)
    assert r.D == o.D and r.S == -1.0
    return r


@pytest.mark.parametrize("d", range(1, 9))
def test_random_all_d(ctx, oracle_mod, d):
    g = np.random.default_rng(300 + d)
    for V, n_p, n_q in [(2, 50, 70), (4, 333, 280), (7, 1000, 1200), (64, 900, 100)]:
        P = g.standard_normal((n_p, d)).astype(np.float32)
        Q = (g.standard_normal((n_q, d)) * 1.2 + 0.3).astype(np.float32)
        check(ctx, oracle_mod, P, Q, V)


def test_ties_signed_zero_and_constant_dimension(ctx, oracle_mod):
    g = np.random.default_rng(5)
    P = np.rint(g.standard_normal((400, 3)) * 2).astype(np.float32)
    Q = np.rint(g.standard_normal((350, 3)) * 2 + 1).astype(np.float32)
    P[P == 0] = -0.0
    P[:, 2] = 1.5
    Q[:, 2] = 1.5
    for V in (1, 3, 5, 8):
        check(ctx, oracle_mod, P, Q, V)


def test_lattice_equals_exact(ctx, oracle_mod):
    g = np.random.default_rng(8)
    V = 6
    P = g.integers(0, V, size=(500, 3)).astype(np.float32)
    Q = g.integers(0, V, size=(450, 3)).astype(np.float32)
    P[0], P[1] = 0, V - 1
    r = check(ctx, oracle_mod, P, Q, V)
    assert r.num == oracle_mod.distance(P, Q).num


def test_workload_scale_and_fine_grid(ctx, oracle_mod):
    """The d = 4, 20000 + 20000 workload on a 16^4 grid, and a grid so fine that
    most points have a voxel of their own."""
    from paper_2106_13706_amd import workloads
    P, Q = workloads.gaussian_scale()
    check(ctx, oracle_mod, P, Q, 16)
    check(ctx, oracle_mod, P[:3000], Q[:3000], 4096)


@pytest.mark.parametrize("d", [1, 3, 4, 7, 8])
def test_byte_and_int16_encodings(ctx, oracle_mod, d):
    """Up to 128 voxels per dimension (and d <= 7) the sweep codes voxel
    coordinates one byte each, from 129 on (and at d = 8) as int16: both sides
    of the boundary, with coordinates at both ends of the grid."""
    g = np.random.default_rng(700 + d)
    for V in (127, 128, 129, 200):
        P = g.uniform(-1, 1, size=(900, d)).astype(np.float32)
        Q = (g.uniform(-1, 1, size=(800, d)) * 0.9 + 0.05).astype(np.float32)
        P[0], P[1] = -1.0, 1.0  # the extents: voxels 0 and V - 1 in every dimension
        check(ctx, oracle_mod, P, Q, V)


@pytest.mark.parametrize("V", [4, 5])
def test_dense_and_hashed_voxel_tables(ctx, oracle_mod, V):
    """The voxel table takes the key as its slot when the grid has no more
    voxels than the table has slots (at least twice the points, a power of
    two): 60 + 40 points get 256 slots, so a 4^4 grid (256 voxels) is counted
    directly and a 5^4 grid (625) through the hash."""
    g = np.random.default_rng(900 + V)
    P = g.uniform(0, 1, size=(60, 4)).astype(np.float32)
    Q = g.uniform(0, 1, size=(40, 4)).astype(np.float32) ** 2
    P[0], P[1] = 0.0, 1.0
    check(ctx, oracle_mod, P, Q, V)


def test_device_pointers_and_errors(ctx, oracle_mod):
    import torch
    from paper_2106_13706_amd import native
    g = np.random.default_rng(9)
    P = g.standard_normal((700, 5)).astype(np.float32)
    Q = (g.standard_normal((800, 5)) + 0.2).astype(np.float32)
    c = native.Context(stream=torch.cuda.current_stream())
    try:
        r, nf = c.vdks(torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda(), 5)
        o = oracle_mod.vdks(P, Q, 5)
        assert (r.num, r.argmax_origin, r.argmax_orthant, nf) == (o.num, o.argmax_voxel,
                                                                  o.argmax_orthant, o.n_filled)
    finally:
        c.close()
    for bad_v in (0, 65536):
        with pytest.raises(native.DDKSError) as e:
            ctx.vdks(P, Q, bad_v)
        assert e.value.status == native.DDKS_E_INVALID_ARG
    with pytest.raises(native.DDKSError) as e:
        ctx.vdks(np.zeros((5, 8), np.float32), np.ones((5, 8), np.float32), 300)  # 300^8 > 4e18
    assert e.value.status == native.DDKS_E_INVALID_ARG
    bad = P.copy()
    bad[3, 2] = np.inf
    with pytest.raises(native.DDKSError) as e:
        ctx.vdks(bad, Q, 5)
    assert e.value.status == native.DDKS_E_NONFINITE
    assert ctx.vdks(P, Q, 5)[0].num == o.num  # the context keeps working


def _ctx_env(env, **kw):
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


def _heavy_and_light(seed, d, n_heavy):
    """A sample whose points mostly share one voxel (so the chunk holding it
    has more than 65535 points: 64-bit bins) beside spread-out points (other
    chunks stay under 65536: 32-bit bins)."""
    g = np.random.default_rng(seed)
    P = np.concatenate([np.full((n_heavy, d), 0.25, np.float32),
                        g.uniform(-1, 1, size=(3000, d)).astype(np.float32)])
    Q = np.concatenate([np.full((n_heavy // 2, d), -0.5, np.float32),
                        g.uniform(-1, 1, size=(2500, d)).astype(np.float32)])
    return P, Q


@pytest.mark.parametrize("shape", ["4:1", "16:3", "8:6", "4:16", "4:1:2", "8:6:2", "16:3:2"])  # waves:chunks[:groups]
def test_forced_vsweep_shapes(oracle_mod, shape):
    """Every admissible shape of the weighted sweep (one or two origin groups
    per block) gives the oracle's result, with 32-bit bins (chunks under 65536
    points of each sample), with 64-bit bins, and with both kinds of chunk in
    one launch; a shape the dimension does not admit (two groups of 64-bit
    bins at d = 8 exceed the LDS) falls back to the default."""
    from paper_2106_13706_amd import workloads
    ctx = _ctx_env({"DDKS_FORCE_VSWEEP": shape})
    try:
        P, Q = workloads.gaussian_scale()
        check(ctx, oracle_mod, P, Q, 8)
        for d, V in [(3, 7), (6, 4)]:
            check(ctx, oracle_mod, *_heavy_and_light(d, d, 70000), V)
        g = np.random.default_rng(44)
        P = g.standard_normal((90000, 2)).astype(np.float32)
        Q = (g.standard_normal((80000, 2)) + 0.1).astype(np.float32)
        check(ctx, oracle_mod, P, Q, 3)  # 9 voxels: every chunk far over 65535 points
        check(ctx, oracle_mod, *_heavy_and_light(8, 8, 70000), 3)
        P = g.standard_normal((3000, 5)).astype(np.float32)
        Q = (g.standard_normal((2900, 5)) + 0.2).astype(np.float32)
        check(ctx, oracle_mod, P, Q, 6)  # an odd number of origin groups
    finally:
        ctx.close()


def test_vsweep_shape_tuned_and_cached(oracle_mod, tmp_path):
    """Enough filled voxels to tune the weighted sweep's shape: one entry lands
    in the cache file, kind 31 for the byte encoding of a 16^4 grid (30 for
    int16 coordinates), and the result is the oracle's."""
    from paper_2106_13706_amd import native, workloads
    P, Q = workloads.gaussian_scale()
    cache = tmp_path / "tune.txt"
    with native.Context(tune_cache=str(cache)) as ctx:
        r = check(ctx, oracle_mod, P, Q, 16)
        r2 = check(ctx, oracle_mod, P, Q, 16)
        assert r2.num == r.num
    lines = [list(map(int, l.split())) for l in cache.read_text().split("\n") if l.strip()]
    print(f"  cache: {lines}", flush=True)
    vs = [l for l in lines if l[0] == 31 and l[1] == 4]
    assert len(vs) == 1 and vs[0][3] in (4, 8, 16) and 1 <= vs[0][4] % 256 <= 16 and vs[0][4] // 256 in (0, 1)
