"""GPU rdKS (Sec. 2.2.3, Alg. 2) against the CPU oracle: the statistic, the
lowest maximising corner and every corner's numerator, exactly (integer
results, tolerance 0; both sides compute the fp32 distances with the same
rounded operations in the same order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2106_13706_amd import native
    c = native.Context()
    yield c
    c.close()


def check(ctx, oracle_mod, P, Q, **kw):
    print(f"  rdks n=({len(P)},{len(Q)}) d={P.shape[1]}", flush=True)
    r, per = ctx.rdks(P, Q, **kw)
    o = oracle_mod.rdks(P, Q)
    assert (r.num, r.den, r.argmax_origin) == (o.num, o.den, o.argmax_corner)
    np.testing.assert_array_equal(per, o.per_corner)
    assert r.D == o.D and r.S == -1.0
    return r


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8, 16, 64])
def test_random(ctx, oracle_mod, d):
    g = np.random.default_rng(500 + d)
    for n_p, n_q in [(1, 1), (3, 7), (200, 150), (3000, 2500)]:
        P = g.standard_normal((n_p, d)).astype(np.float32)
        Q = (g.standard_normal((n_q, d)) * 1.1 + 0.2).astype(np.float32)
        check(ctx, oracle_mod, P, Q)


def test_ties_shared_points_signed_zero(ctx, oracle_mod):
    g = np.random.default_rng(6)
    P = np.rint(g.standard_normal((700, 3)) * 2).astype(np.float32)
    Q = np.rint(g.standard_normal((650, 3)) * 2 + 0.5).astype(np.float32)
    Q[:100] = P[:100]
    P[P == 0] = -0.0
    Q[:, 1] = 2.0
    P[:, 1] = 2.0  # a constant dimension
    check(ctx, oracle_mod, P, Q)


@pytest.mark.parametrize("n_p,n_q,d", [(4096, 1, 2), (20000, 20000, 4), (70000, 60000, 3)])
def test_many_tiles_and_segments(ctx, oracle_mod, n_p, n_q, d):
    g = np.random.default_rng(n_p + d)
    P = g.standard_normal((n_p, d)).astype(np.float32)
    Q = (g.standard_normal((n_q, d)) + 0.05).astype(np.float32)
    check(ctx, oracle_mod, P, Q)


@pytest.mark.parametrize("N", [64, 255, 256, 257, 1023, 1024, 1025, 3500, 4095, 4096, 4097, 8192])
def test_sort_tile_boundaries(ctx, oracle_mod, N):
    """Column sorts of one 256-, 1024- or 4096-pair tile (written straight to
    the sorted columns) and of several tiles, around each size limit, with
    ties (values on a coarse grid)."""
    g = np.random.default_rng(N)
    n_p = N // 3 + 1
    Z = (np.rint(g.standard_normal((N, 3)) * 8) / 8).astype(np.float32)
    check(ctx, oracle_mod, Z[:n_p], Z[n_p:])


@pytest.mark.parametrize("d,n", [(31, 300), (32, 300), (257, 150), (4096, 12)])
def test_distance_kernel_paths(ctx, oracle_mod, d, n):
    """Both distance kernels (one thread per point and corner below 32
    dimensions, the point's row staged in LDS from 32 on, up to the 4096 limit)."""
    g = np.random.default_rng(d)
    P = g.standard_normal((n, d)).astype(np.float32)
    Q = (g.standard_normal((n + 3, d)) * 1.3).astype(np.float32)
    check(ctx, oracle_mod, P, Q)


def test_high_dimension(ctx, oracle_mod):
    """The paper's latent-space case: 100 points per sample in 1000 dimensions."""
    g = np.random.default_rng(1000)
    P = g.standard_normal((100, 1000)).astype(np.float32)
    Q = g.uniform(-1.7, 1.7, size=(100, 1000)).astype(np.float32)
    check(ctx, oracle_mod, P, Q)


def test_device_pointers_and_errors(ctx, oracle_mod):
    import torch
    from paper_2106_13706_amd import native
    g = np.random.default_rng(10)
    P = g.standard_normal((900, 6)).astype(np.float32)
    Q = (g.standard_normal((800, 6)) * 0.9).astype(np.float32)
    c = native.Context(stream=torch.cuda.current_stream())
    try:
        r, per = c.rdks(torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda())
        o = oracle_mod.rdks(P, Q)
        assert (r.num, r.argmax_origin) == (o.num, o.argmax_corner)
        np.testing.assert_array_equal(per, o.per_corner)
    finally:
        c.close()
    bad = P.copy()
    bad[7, 3] = np.nan
    with pytest.raises(native.DDKSError) as e:
        ctx.rdks(bad, Q)
    assert e.value.status == native.DDKS_E_NONFINITE
    with pytest.raises(native.DDKSError) as e:
        ctx.rdks(np.zeros((3, 4097), np.float32), np.zeros((3, 4097), np.float32))
    assert e.value.status == native.DDKS_E_INVALID_ARG
    assert ctx.rdks(P, Q)[0].num == o.num  # the context keeps working
