"""GPU analytic significance (Sec. 3, Eq. ddks_significance) against the CPU
oracle, compared relatively.

Both sides evaluate the same sums in fp64 in different orders, and from
log-factorials of different libraries (the device's lgamma, glibc's):
  - every pmf is exp of at most three log-factorials plus two log-rate
    terms, each of magnitude at most ln(n_max!); two libraries each within a
    few ulp of the true value differ by at most ~8u of that magnitude
    (u = 2^-53) per term, so a pmf, and any sum or product of two of them,
    moves by at most 6 * 8u * ln(n_max!) relative; the sums themselves add
    ~n u, far less;
  - the device sums each tail over windows around the means outside which
    the left-out mass is at most e^-700 (Bernstein's inequality), so S can
    differ by at most entries * 1e-304 in absolute terms.
Hence |S - S_oracle| <= rtol(n_max) * S_oracle + entries * 1e-304 with
rtol(n) = 128 u ln(n!) + 1e-12 (no absolute floor above the windows' own
bound).  The large-sample cases pick the statistic so that the oracle's S
lies in (1e-300, 0.5) and so that each of the device's three ways of
bounding a tail is taken: narrow windows kept, narrow windows summed and
redone wide because the tail came out below their threshold, and wide
windows first because a normal estimate puts D far out.  Binomial model:
S = 0 exactly when D = 1; the Poisson model (Sec. 3's large-sample
replacement) keeps the mass beyond the sample sizes."""
import json
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

THREADS = max(1, len(os.sched_getaffinity(0)))
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


def rtol(n_max):
    return 128 * U * math.lgamma(n_max + 1.0) + 1e-12


def close(S, So, n_max, entries):
    return abs(S - So) <= rtol(n_max) * So + entries * 1e-304


# The device's window policy (the kernel's documented constants): a normal
# estimate z of how far D lies out picks wide windows first when z > 12;
# otherwise narrow windows are summed and kept when the tail is >= 1e-30.
Z_WIDE_FIRST = 12.0
NARROW_MIN_TAIL = 1e-30


def _var(n_p, n_q, t, model):
    lam = (t + 1.0) / (n_q + 2.0)
    return (lam if model == "poisson" else lam * (1.0 - lam)) * (1.0 / n_p + 1.0 / n_q)


def z_of(n_p, n_q, t, num, model):
    return (num / (n_p * n_q)) / math.sqrt(_var(n_p, n_q, t, model))


def num_for_z(n_p, n_q, t, z, model):
    return int(z * math.sqrt(_var(n_p, n_q, t, model)) * n_p * n_q)


def regime(z, tail):
    if z > Z_WIDE_FIRST:
        return "wide_first"
    return "narrow_kept" if tail >= NARROW_MIN_TAIL else "narrow_then_wide"


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
        assert close(S, So, max(n_p, n_q), counts.size // 2)
        assert 0.0 <= S <= 1.0
    if model == "binomial":
        assert ctx.significance(counts, n_p, n_q, d, r.den) == 0.0


SIZES = [(50000, 50000), (3000, 60000), (60000, 700)]
Z_GRID = (6.0, 9.0, 11.5, 11.8, 11.95, 12.5, 16.0, 25.0, 35.0, 45.0)


def _single_value_counts(n_p, n_q, t):
    """d = 1 counts whose second-sample entries all equal t (S only reads c_Q)."""
    c = np.zeros((n_p + n_q, 2, 2), np.uint32)
    c[:, :, 1] = t
    return c


@pytest.mark.parametrize("model", sorted(MODELS))
def test_large_samples_windows(ctx, oracle_mod, model):
    """Large samples, where the device sums only windows around the means.
    One value of c_Q per case, so that S = 1 - (1 - tail)^entries checks that
    value's tail on its own; the statistic is placed z normal deviations out
    for z on a grid, and the cases whose oracle S lies in (1e-300, 0.5) are
    compared.  Every window regime must be among them."""
    seen = {}
    worst = 0.0
    for n_p, n_q in SIZES:
        for t in (0, 7, n_q // 50, n_q // 2, n_q - 3):
            counts = _single_value_counts(n_p, n_q, t)
            entries = counts.size // 2
            lam = (t + 1.0) / (n_q + 2.0)
            for z in Z_GRID:
                num = num_for_z(n_p, n_q, t, z, model)
                if num >= n_p * n_q:
                    continue
                So = oracle_mod.significance(counts, n_p, n_q, 1, num, model)
                S = ctx.significance(counts, n_p, n_q, 1, num, flags=MODELS[model])
                tail = oracle_mod.tail(n_p, n_q, lam, num, model)
                reg = regime(z_of(n_p, n_q, t, num, model), tail)
                rel = abs(S - So) / So if So > 0 else abs(S)
                print(f"  {model} n=({n_p},{n_q}) c_Q={t} z={z} num={num} [{reg}]: "
                      f"S={S!r} oracle={So!r} rel={rel:.2e}", flush=True)
                assert close(S, So, max(n_p, n_q), entries)
                if 1e-300 < So < 0.5:
                    seen[reg] = seen.get(reg, 0) + 1
                    worst = max(worst, rel / rtol(max(n_p, n_q)))
    print(f"  informative cases per regime: {seen}; worst error / rtol = {worst:.3f}", flush=True)
    assert set(seen) == {"narrow_kept", "narrow_then_wide", "wide_first"}
    assert min(seen.values()) >= 3


@pytest.mark.parametrize("model", sorted(MODELS))
def test_large_samples_mixed_values(ctx, oracle_mod, model):
    """Many distinct values of c_Q at once (the product over origins and
    orthants), with the statistic chosen so that S stays below 0.5: the
    value with the widest spread sits 7 deviations out, the others further
    (no value near n_q: under the Poisson model its mass beyond the sample
    size alone would saturate S)."""
    n_p, n_q = 50000, 50000
    vals = np.array([3, 7, 400, 1000, 9000, 25000, 31000, 40000, 47000], np.int64)
    g = np.random.default_rng(5)
    counts = np.zeros((n_p + n_q, 4, 2), np.uint32)
    counts[:, :, 1] = vals[g.integers(0, len(vals), size=(n_p + n_q, 4))]
    num = max(num_for_z(n_p, n_q, int(t), 7.0, model) for t in vals)
    So = oracle_mod.significance(counts, n_p, n_q, 2, num, model)
    S = ctx.significance(counts, n_p, n_q, 2, num, flags=MODELS[model])
    print(f"  {model}: num={num} S={S!r} oracle={So!r}", flush=True)
    assert 1e-300 < So < 0.5
    assert close(S, So, n_q, counts.size // 2)


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
            assert close(r.S, So, max(n_p, n_q), o.counts.size // 2) and r2.S == r.S
            cnt = cnt.cpu().numpy().view(np.uint32) if device else cnt
            np.testing.assert_array_equal(cnt, o.counts)
            assert c.distance(*args).S == -1.0  # not asked for
    finally:
        c.close()


@pytest.mark.parametrize("model", sorted(MODELS))
def test_workload_gaussian_scale_d4_20000(ctx, model):
    """The d = 4, 20000 + 20000 workload's S in one ddks_distance call, against
    the oracle's value stored by tests/golden/make_full_size.py."""
    from paper_2106_13706_amd import native, workloads
    g = json.load(open(os.path.join(GOLDEN, "full_gaussian_scale_d4_20000.json")))
    P, Q = workloads.gaussian_scale()
    r = ctx.distance(P, Q, flags=native.DDKS_WITH_SIGNIFICANCE | MODELS[model])
    So = g[f"S_{model}"]
    print(f"  {model}: S={r.S!r} oracle={So!r} rel={abs(r.S - So) / So:.2e}", flush=True)
    assert r.num == g["num"]
    assert 1e-300 < So < 0.5
    assert close(r.S, So, 20000, 40000 * 16)


@pytest.mark.parametrize("model", sorted(MODELS))
def test_workload_permutation_observed(ctx, model):
    """The permutation workload's observed split (d = 5, 4096 + 4096): its S
    against the oracle's stored value, beside the permutation p-value."""
    from paper_2106_13706_amd import native, workloads
    g = json.load(open(os.path.join(GOLDEN, "full_permutation_d5_8192x1024.json")))["observed"]
    Z, n_p, _ = workloads.permutation(B=1)
    P, Q = Z[:n_p], Z[n_p:]
    r = ctx.distance(P, Q, flags=native.DDKS_WITH_SIGNIFICANCE | MODELS[model])
    So = g[f"S_{model}"]
    print(f"  {model}: S={r.S!r} oracle={So!r}", flush=True)
    assert r.num == g["num"]
    assert 1e-300 < So < 0.5
    assert close(r.S, So, n_p, 8192 * 32)


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
