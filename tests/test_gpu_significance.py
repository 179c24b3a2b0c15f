"""GPU analytic significance (Sec. 3, Eq. ddks_significance) against the CPU
oracle.  Both evaluate the same sums in fp64 in different orders, so they
agree to |S_gpu - S_oracle| <= 1e-9 * |S_oracle| + 1e-12 (each tail is a sum
of at most n_P + n_T + 2 non-negative terms, and the log-sum has N * 2^d
terms; the bound leaves several orders of magnitude of margin over the
accumulated rounding).  The device sums only windows around each mean outside
which the left-out mass is below ~1e-304 (Bernstein's inequality).  Binomial
model: S = 0 exactly when D = 1; the Poisson model (Sec. 3's large-sample
replacement) keeps the mass beyond the sample sizes."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


def close(a, b):
    return abs(a - b) <= 1e-9 * abs(b) + 1e-12


@pytest.fixture(scope="module")
def ctx():
    from paper_2106_13706_amd import native
    c = native.Context()
    yield c
    c.close()


MODELS = {"binomial": 0x0, "poisson": 0x40}  # DDKS_SIG_POISSON


@pytest.mark.parametrize("model", sorted(MODELS))
@pytest.mark.parametrize("d,n_p,n_q,shift", [(1, 20, 25, 0.0), (2, 60, 45, 0.5), (3, 150, 200, 0.1),
                                             (4, 300, 280, 0.0), (2, 7, 300, 1.0)])
def test_matches_oracle(ctx, oracle_mod, d, n_p, n_q, shift, model):
    g = np.random.default_rng(d * 100 + n_p)
    P = g.standard_normal((n_p, d)).astype(np.float32)
    Q = (g.standard_normal((n_q, d)) + shift).astype(np.float32)
    r, counts = ctx.distance(P, Q, counts=True)
    for num in (r.num, 0, r.den // 3, r.den):
        S = ctx.significance(counts, n_p, n_q, d, num, flags=MODELS[model])
        So = oracle_mod.significance(counts, n_p, n_q, d, num, model)
        print(f"  {model} d={d} n=({n_p},{n_q}) num={num}: S={S!r} oracle={So!r}", flush=True)
        assert close(S, So)
        assert 0.0 <= S <= 1.0
    if model == "binomial":
        assert ctx.significance(counts, n_p, n_q, d, r.den) == 0.0


@pytest.mark.parametrize("model", sorted(MODELS))
@pytest.mark.parametrize("n_p,n_q", [(50000, 50000), (3000, 60000), (60000, 700)])
def test_large_samples_windows(ctx, oracle_mod, n_p, n_q, model):
    """Large samples, where the device sums only a window around each mean:
    counts holding a few distinct second-sample
    values (the statistic only needs c_Q), so that the oracle's full sums
    stay cheap."""
    N = n_p + n_q
    vals = np.array([0, 1, 7, n_q // 50, n_q // 3, n_q // 2, n_q - 3, n_q], np.uint32)
    g = np.random.default_rng(n_p + n_q)
    counts = np.zeros((N, 2, 2), np.uint32)
    counts[:, :, 1] = vals[g.integers(0, len(vals), size=(N, 2))]
    den = n_p * n_q
    for num in (0, den // 5000, den // 1000, den // 100, den // 10):
        S = ctx.significance(counts, n_p, n_q, 1, num, flags=MODELS[model])
        So = oracle_mod.significance(counts, n_p, n_q, 1, num, model)
        print(f"  {model} n=({n_p},{n_q}) num={num}: S={S!r} oracle={So!r}", flush=True)
        assert close(S, So)


@pytest.mark.parametrize("model", sorted(MODELS))
@pytest.mark.parametrize("device", [False, True])
def test_distance_with_significance(oracle_mod, model, device):
    """ddks_distance with DDKS_WITH_SIGNIFICANCE: S of the statistic it finds,
    computed on the device from counts that stay there."""
    import torch
    from paper_2106_13706_amd import native
    flags = native.DDKS_WITH_SIGNIFICANCE | MODELS[model]
    c = native.Context(stream=torch.cuda.current_stream() if device else None)
    try:
        g = np.random.default_rng(17)
        for d, n_p, n_q in [(3, 900, 700), (5, 2000, 2500), (2, 40, 9000)]:
            P = g.standard_normal((n_p, d)).astype(np.float32)
            Q = (g.standard_normal((n_q, d)) + 0.15).astype(np.float32)
            o = oracle_mod.distance(P, Q, counts=True, threads=THREADS)
            So = oracle_mod.significance(o.counts, n_p, n_q, d, o.num, model)
            args = (torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda()) if device else (P, Q)
            r = c.distance(*args, flags=flags)
            r2, cnt = c.distance(*args, counts=True, flags=flags)
            print(f"  {model} dev={device} d={d} n=({n_p},{n_q}): S={r.S!r} oracle={So!r}", flush=True)
            assert (r.num, r.argmax_origin, r.argmax_orthant) == (o.num, o.argmax_origin,
                                                                  o.argmax_orthant)
            assert close(r.S, So) and r2.S == r.S
            cnt = cnt.cpu().numpy().view(np.uint32) if device else cnt
            np.testing.assert_array_equal(cnt, o.counts)
            assert c.distance(*args).S == -1.0  # not asked for
    finally:
        c.close()


def test_workload_permutation_observed(ctx, oracle_mod):
    from paper_2106_13706_amd import workloads
    Z, n_p, _ = workloads.permutation(B=1)
    P, Q = Z[:n_p], Z[n_p:]
    r, counts = ctx.distance(P, Q, counts=True)
    S = ctx.significance(counts, n_p, len(Q), P.shape[1], r.num)
    So = oracle_mod.significance(counts, n_p, len(Q), P.shape[1], r.num)
    print(f"  S={S!r} oracle={So!r}", flush=True)
    assert close(S, So)


def test_rejects_bad_counts(ctx):
    from paper_2106_13706_amd import native
    c = np.zeros((5, 4, 2), np.uint32)
    c[:, 0, 0] = 2
    c[:, 0, 1] = 3
    c[1, 1, 1] = 9  # exceeds n_q = 3
    with pytest.raises(native.DDKSError) as e:
        ctx.significance(c, 2, 3, 2, 1)
    assert e.value.status == native.DDKS_E_INVALID_ARG
    c[1, 1, 1] = 0
    assert 0.0 <= ctx.significance(c, 2, 3, 2, 1) <= 1.0
