"""Pins for the oracle's inference pieces: the analytic significance of
Sec. 3 and the permutation test / p-value.  CPU only."""
import math

import numpy as np
import pytest
from scipy.stats import binom, poisson

from tests.tensor_reference import ddks_tensor


# ---------------------------------------------------------------- tail / S

@pytest.mark.parametrize("lam", [0.05, 0.3, 0.5, 0.9])
def test_tail_closed_form_single_trials(oracle_mod, lam):
    # n_P = n_T = 1: delta in {0, 1}; P(delta > 0) = 2 lam (1 - lam)
    assert math.isclose(oracle_mod.tail(1, 1, lam, 0), 2 * lam * (1 - lam), rel_tol=1e-12)
    assert oracle_mod.tail(1, 1, lam, 1) == 0.0


@pytest.mark.parametrize("n", [1, 2, 5, 17, 40])
def test_tail_closed_form_equal_sizes_half_rate(oracle_mod, n):
    # P(a == b) for a, b ~ Bi(n, 1/2) is C(2n, n) / 4^n (Vandermonde)
    exp = 1.0 - math.comb(2 * n, n) / 4.0 ** n
    assert math.isclose(oracle_mod.tail(n, n, 0.5, 0), exp, rel_tol=1e-10, abs_tol=1e-15)


@pytest.mark.parametrize("n_p,n_q", [(3, 5), (7, 4), (12, 12), (20, 9)])
def test_tail_vs_double_sum(oracle_mod, n_p, n_q):
    """Direct sum over every (a, b) with the library binomial pmf."""
    for lam in (0.1, 0.37, 0.8):
        pa = binom.pmf(np.arange(n_p + 1), n_p, lam)
        pb = binom.pmf(np.arange(n_q + 1), n_q, lam)
        for num in (0, 1, n_p, n_q, (n_p * n_q) // 3, n_p * n_q - 1, n_p * n_q):
            far = 0.0
            for a in range(n_p + 1):
                for b in range(n_q + 1):
                    if abs(a * n_q - b * n_p) > num:
                        far += pa[a] * pb[b]
            assert math.isclose(oracle_mod.tail(n_p, n_q, lam, num), far,
                                rel_tol=1e-9, abs_tol=1e-14)


# ---------------------------------------------------------------- Poisson model
# Sec. 3: for large samples and small rates each binomial pmf may be replaced
# by the Poisson pmf of the same mean; read with the sums over the same
# supports 0..m, so P(delta <= D) = sum over (a, b) in the window of
# Pois(a; n_p lam) Pois(b; n_q lam), a <= n_p, b <= n_q.

@pytest.mark.parametrize("n_p,n_q", [(3, 5), (7, 4), (12, 12), (20, 9)])
def test_poisson_tail_vs_direct_window_sum(oracle_mod, n_p, n_q):
    """The oracle computes the complement as (mass beyond the supports) +
    (excluded mass inside); here 1 - (the included mass), summed directly
    with the library Poisson pmf."""
    for lam in (0.02, 0.1, 0.37, 0.8):
        pa = poisson.pmf(np.arange(n_p + 1), n_p * lam)
        pb = poisson.pmf(np.arange(n_q + 1), n_q * lam)
        for num in (0, 1, n_p, n_q, (n_p * n_q) // 3, n_p * n_q - 1, n_p * n_q):
            inside = 0.0
            for a in range(n_p + 1):
                for b in range(n_q + 1):
                    if abs(a * n_q - b * n_p) <= num:
                        inside += pa[a] * pb[b]
            assert math.isclose(oracle_mod.tail(n_p, n_q, lam, num, "poisson"), 1.0 - inside,
                                rel_tol=1e-9, abs_tol=1e-14)


@pytest.mark.parametrize("lam", [0.01, 0.2, 0.7])
def test_poisson_tail_single_trials(oracle_mod, lam):
    # n_P = n_T = 1, num = 0: included iff a == b, a, b in {0, 1}, each ~ Pois(lam)
    inside = math.exp(-2 * lam) * (1 + lam * lam)
    assert math.isclose(oracle_mod.tail(1, 1, lam, 0, "poisson"), 1 - inside, rel_tol=1e-12)


@pytest.mark.parametrize("n_p,n_q", [(200, 300), (1000, 800), (5000, 5000)])
def test_poisson_close_to_binomial_le_cam(oracle_mod, n_p, n_q):
    """Le Cam: TV(Bi(m, lam), Pois(m lam)) <= m lam^2.  The included event
    then differs between the models by at most (n_p + n_q) lam^2 plus the
    Poisson mass beyond the supports (negligible here)."""
    for lam in (0.0005, 0.002, 0.01):
        bound = (n_p + n_q) * lam * lam + 1e-12
        for num in (0, n_p, n_q, (n_p * n_q) // 100, (n_p * n_q) // 20):
            tb = oracle_mod.tail(n_p, n_q, lam, num)
            tp = oracle_mod.tail(n_p, n_q, lam, num, "poisson")
            assert abs(tb - tp) <= bound, (lam, num, tb, tp, bound)


def test_poisson_significance_properties(oracle_mod):
    g = np.random.default_rng(5)
    P = g.standard_normal((25, 3)).astype(np.float32)
    Q = (g.standard_normal((30, 3)) + 0.4).astype(np.float32)
    r = oracle_mod.distance(P, Q, counts=True)
    den = r.den
    prev = 1.0
    for num in [0, den // 10, den // 5, r.num, den // 2, den - 1, den]:
        S = oracle_mod.significance(r.counts, 25, 30, 3, num, "poisson")
        assert 0.0 <= S <= 1.0
        assert S <= prev + 1e-15  # non-increasing in D
        prev = S
    # product structure, as for the binomial model
    keep = 1.0
    for k in range(55):
        for j in range(8):
            lam = (int(r.counts[k, j, 1]) + 1) / (30 + 2)
            keep *= 1.0 - oracle_mod.tail(25, 30, lam, r.num, "poisson")
    assert math.isclose(oracle_mod.significance(r.counts, 25, 30, 3, r.num, "poisson"),
                        1.0 - keep, rel_tol=1e-10, abs_tol=1e-15)


def test_significance_properties(oracle_mod):
    g = np.random.default_rng(3)
    P = g.standard_normal((25, 2)).astype(np.float32)
    Q = (g.standard_normal((30, 2)) + 0.4).astype(np.float32)
    r = oracle_mod.distance(P, Q, counts=True)
    den = r.den
    prev = 1.0
    for num in [0, den // 10, den // 5, r.num, den // 2, den - 1, den]:
        S = oracle_mod.significance(r.counts, 25, 30, 2, num)
        assert 0.0 <= S <= 1.0
        assert S <= prev + 1e-15  # non-increasing in D
        prev = S
    assert oracle_mod.significance(r.counts, 25, 30, 2, den) == 0.0


def test_significance_product_structure(oracle_mod):
    """S = 1 - prod over (origin, orthant) of (1 - tail) with lambda from the
    second sample's count (Bayes estimator (M_T + 1)/(N_T + 2))."""
    P = np.array([[0, 0], [1, 2], [2, 1]], np.float32)
    Q = np.array([[1, 1], [2, 2]], np.float32)
    r = oracle_mod.distance(P, Q, counts=True)
    keep = 1.0
    for k in range(5):
        for j in range(4):
            lam = (int(r.counts[k, j, 1]) + 1) / (2 + 2)
            keep *= 1.0 - oracle_mod.tail(3, 2, lam, r.num)
    assert math.isclose(oracle_mod.significance(r.counts, 3, 2, 2, r.num), 1.0 - keep,
                        rel_tol=1e-12, abs_tol=1e-15)


# ---------------------------------------------------------------- permutation

def test_permutation_rows(oracle_mod):
    g = np.random.default_rng(1)
    n, n_p, d = 23, 11, 3
    Z = np.rint(g.standard_normal((n, d)) * 2).astype(np.float32)
    masks = []
    for b in range(9):
        m = np.zeros(n, bool)
        m[g.permutation(n)[:n_p]] = True
        masks.append(m)
    m0 = np.zeros(n, bool)
    m0[:n_p] = True
    masks.append(m0)
    words = oracle_mod.labels_to_words(np.array(masks))
    nums = oracle_mod.permutation(Z, n_p, words, threads=2)
    for m, num in zip(masks, nums):
        assert int(num) == ddks_tensor(Z[m], Z[~m])[0]
    assert int(nums[-1]) == oracle_mod.distance(Z[:n_p], Z[n_p:]).num


def test_permutation_rejects_bad_row(oracle_mod):
    Z = np.zeros((10, 2), np.float32)
    m = np.zeros((1, 10), bool)
    m[0, :3] = True  # 3 ones, n_p = 4
    with pytest.raises(ValueError):
        oracle_mod.permutation(Z, 4, oracle_mod.labels_to_words(m))


def test_pvalue():
    import oracle
    nums = np.array([5, 9, 9, 1, 12, 9], np.uint64)
    p, frac = oracle.pvalue(nums, 9)
    assert p == (1 + 4) / 7 and frac == 4 / 6
    p, frac = oracle.pvalue(nums, 13)
    assert p == 1 / 7 and frac == 0.0
