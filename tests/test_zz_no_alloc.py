"""ddks_distance_noalloc (the entry point for callers that cannot allocate
device memory) against ddks_distance, through the C ABI: the same result and
the same counts, bit for bit (integer results, tolerance 0), on two calls in a
row whose second input is smaller, on both compare paths and on a chunked
launch shape; oversized inputs are refused before anything is launched."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _key(r):
    return (r.num, r.den, r.D, r.argmax_origin, r.argmax_orthant, r.d, r.n_p, r.n_q)


def _pair(seed, n_p, n_q, d, grid=None):
    g = np.random.default_rng(seed)
    P = g.standard_normal((n_p, d))
    Q = g.standard_normal((n_q, d)) * 1.1 + 0.1
    if grid:
        P, Q = np.rint(P * grid) / grid, np.rint(Q * grid) / grid
    return P.astype(np.float32), Q.astype(np.float32)


def _check(ctx, P, Q, flags=0):
    import torch
    from paper_2106_13706_amd import native
    N, d = len(P) + len(Q), P.shape[1]
    Pt, Qt = torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda()
    counts = torch.empty((N, 1 << d, 2), dtype=torch.int32, device="cuda")
    print(f"  case n_p={len(P)} n_q={len(Q)} d={d} flags={flags:#x}", flush=True)
    r = ctx.distance_noalloc(Pt, Qt, flags=flags)
    rc = ctx.distance_noalloc(Pt, Qt, counts=counts, flags=flags)
    ref, ref_counts = ctx.distance(Pt, Qt, counts=True, flags=flags)
    assert _key(r) == _key(rc) == _key(ref)
    assert r.S == -1.0
    assert torch.equal(counts, ref_counts)
    return r


@pytest.mark.parametrize("flags", [0, 0x2, 0x10])  # default, DDKS_FORCE_F32, DDKS_FORCE_RANK16
def test_two_calls_second_smaller(flags):
    from paper_2106_13706_amd import native
    with native.Context() as ctx:
        # the d = 4, 20000 + 20000 workload (rank codes, two point chunks), then smaller
        from paper_2106_13706_amd import workloads
        _check(ctx, *workloads.gaussian_scale(), flags=flags)
        _check(ctx, *_pair(2, 3001, 2750, 4, grid=8), flags=flags)
        _check(ctx, *_pair(3, 70, 45, 3), flags=flags)


def test_paths_and_shapes():
    """Sizes spanning several origin groups and a ragged tail, every d, and
    more than 65536 points (fp32 compares in the no-allocation call)."""
    from paper_2106_13706_amd import native
    with native.Context() as ctx:
        for d in range(1, 9):
            _check(ctx, *_pair(10 + d, 1000 + 37 * d, 777, d, grid=4 if d % 2 else None))
        _check(ctx, *_pair(30, 40000, 30001, 3))


def test_no_device_allocation_and_limits():
    """After a first call has loaded the kernels, further calls leave the
    device's free memory unchanged; an input beyond the scratch is refused
    with DDKS_E_NOMEM and the context keeps working."""
    import torch
    from paper_2106_13706_amd import native
    P, Q = _pair(40, 9000, 8000, 5)
    Pt, Qt = torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda()
    big = torch.zeros((2_000_000, 8), dtype=torch.float32, device="cuda")
    with native.Context() as ctx:
        first = ctx.distance_noalloc(Pt, Qt)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for _ in range(3):
            assert _key(ctx.distance_noalloc(Pt, Qt)) == _key(first)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        with pytest.raises(native.DDKSError) as e:
            ctx.distance_noalloc(big, big)
        assert e.value.status == native.DDKS_E_NOMEM
        with pytest.raises(native.DDKSError) as e:
            ctx.distance_noalloc(Pt, Qt, flags=native.DDKS_WITH_SIGNIFICANCE)
        assert e.value.status == native.DDKS_E_NOT_SUPPORTED
        assert _key(ctx.distance_noalloc(Pt, Qt)) == _key(ctx.distance(P, Q))
