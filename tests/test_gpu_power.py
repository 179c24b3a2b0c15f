"""The power-study harness of Sec. 4.2 on the GPU: its permutation p-values
against a per-relabelling recomputation with plain calls, and a bisection
run."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2106_13706_amd import native
    c = native.Context()
    yield c
    c.close()


def test_batched_p_value_equals_recomputation(ctx):
    from paper_2106_13706_amd import power, workloads
    P, Q = workloads.power_dataset("GVS", 150, seed=3)
    p, D = power.permutation_test(ctx, P, Q, B=40, method="ddks", seed=11)
    Z = np.concatenate([P, Q])
    masks = power._unpack_rows(workloads.relabel_rows(300, 150, 40, 11), 300)
    assert all(m.sum() == 150 for m in masks)
    obs = ctx.distance(P, Q)
    ge = sum(1 for m in masks if ctx.distance(Z[m], Z[~m]).num >= obs.num)
    assert p == (1 + ge) / 41 and D == obs.D


@pytest.mark.parametrize("method", ["vdks", "rdks"])
def test_approximate_methods_p_values(ctx, method):
    from paper_2106_13706_amd import power, workloads
    P, Q = workloads.power_dataset("DVU", 60, seed=4)
    p, D = power.permutation_test(ctx, P, Q, B=30, method=method, seed=2)
    assert 0 < p <= 1 and 0 <= D <= 1
    assert p == power.permutation_test(ctx, P, Q, B=30, method=method, seed=2)[0]  # seeded


def test_bisection_dvu(ctx):
    """The paper rejects DVU at alpha = 0.05 from about ten points per sample."""
    from paper_2106_13706_amd import power
    n, pts = power.min_sample_size(ctx, "DVU", B=100, n_hi=256)
    print(f"  DVU min n = {n}: {[(x.n, x.p_value) for x in pts]}", flush=True)
    assert n is not None and n <= 128
    assert all(x.rejected == (x.p_value <= 0.05) for x in pts)


def test_parameter_gap_gvm(ctx):
    """At n = 50 the exact statistic separates GVM means well below one sigma."""
    from paper_2106_13706_amd import power
    gap, pts = power.min_parameter_gap(ctx, "GVM", n=50)
    print(f"  GVM gap at n=50: {gap}: {[(round(x, 4), p.p_value) for x, p in pts]}", flush=True)
    assert gap is not None and 0 < gap < 2.0
    assert all(p.rejected == (p.p_value <= 0.05) for _, p in pts)
    with pytest.raises(ValueError):
        power.min_parameter_gap(ctx, "DVU")
