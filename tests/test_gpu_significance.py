"""GPU analytic significance (Sec. 3, Eq. ddks_significance) against the CPU
oracle.  Both evaluate the same sums in fp64 in different orders, so they
agree to |S_gpu - S_oracle| <= 1e-9 * |S_oracle| + 1e-12 (each tail is a sum
of at most n_P + n_T + 2 non-negative terms, and the log-sum has N * 2^d
terms; the bound leaves several orders of magnitude of margin over the
accumulated rounding).  S = 0 exactly when D = 1."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def close(a, b):
    return abs(a - b) <= 1e-9 * abs(b) + 1e-12


@pytest.fixture(scope="module")
def ctx():
    from paper_2106_13706_amd import native
    c = native.Context()
    yield c
    c.close()


@pytest.mark.parametrize("d,n_p,n_q,shift", [(1, 20, 25, 0.0), (2, 60, 45, 0.5), (3, 150, 200, 0.1),
                                             (4, 300, 280, 0.0), (2, 7, 300, 1.0)])
def test_matches_oracle(ctx, oracle_mod, d, n_p, n_q, shift):
    g = np.random.default_rng(d * 100 + n_p)
    P = g.standard_normal((n_p, d)).astype(np.float32)
    Q = (g.standard_normal((n_q, d)) + shift).astype(np.float32)
    r, counts = ctx.distance(P, Q, counts=True)
    for num in (r.num, 0, r.den // 3, r.den):
        S = ctx.significance(counts, n_p, n_q, d, num)
        So = oracle_mod.significance(counts, n_p, n_q, d, num)
        print(f"  d={d} n=({n_p},{n_q}) num={num}: S={S!r} oracle={So!r}", flush=True)
        assert close(S, So)
        assert 0.0 <= S <= 1.0
    assert ctx.significance(counts, n_p, n_q, d, r.den) == 0.0


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
