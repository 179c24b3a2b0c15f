"""Pins for the CPU oracle: worked examples, the d=1 reduction to the
two-sample KS test, an independent tensor formulation, and invariants that
the definition implies (Sec. 2.1, Appendix proofs).  CPU only."""
import json
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from tests.tensor_reference import ddks_tensor, ks_1d_sortmerge

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- examples

@pytest.mark.parametrize("name", ["example_a.json", "example_b.json", "example_c.json"])
def test_worked_examples(oracle_mod, name):
    g = _golden(name)
    r = oracle_mod.distance(np.array(g["P"], np.float32), np.array(g["Q"], np.float32),
                            counts=True)
    assert (r.num, r.den) == (g["num"], g["den"])
    assert (r.argmax_origin, r.argmax_orthant) == (g["argmax_origin"], g["argmax_orthant"])
    if "counts" in g:
        exp = np.array(g["counts"], dtype=np.uint32)  # [N][sample][orthant]
        np.testing.assert_array_equal(r.counts, exp.transpose(0, 2, 1))


def test_example_b_strict_convention_differs(oracle_mod):
    """The tie rule matters: under strict '>' the same data gives D = 1."""
    g = _golden("example_b.json")
    P = np.array(g["P"], np.float32)
    Q = np.array(g["Q"], np.float32)
    # A strict '>' comparison equals '>=' after moving every point down by an
    # infinitesimal relative to the origins; emulate it with the tensor form.
    S = np.concatenate([P, Q]).astype(np.float64)
    n_p, n_q = len(P), len(Q)
    best = 0
    for o in S:
        cP = np.bincount([int(sum(int(x[m] > o[m]) << m for m in range(2))) for x in P],
                         minlength=4)
        cQ = np.bincount([int(sum(int(x[m] > o[m]) << m for m in range(2))) for x in Q],
                         minlength=4)
        best = max(best, int(np.abs(cP * n_q - cQ * n_p).max()))
    assert best == g["strict_greater_num"]
    assert oracle_mod.distance(P, Q).num == g["num"]


def test_example_c_decreasing_map(oracle_mod):
    g = _golden("example_c.json")
    P = np.array(g["P"], np.float32)
    Q = np.array(g["Q"], np.float32)
    P2, Q2 = P.copy(), Q.copy()
    P2[:, 0] *= -1
    Q2[:, 0] *= -1
    r = oracle_mod.distance(P2, Q2)
    e = g["negated_axis0"]
    assert (r.num, r.den, r.argmax_origin, r.argmax_orthant) == (
        e["num"], e["den"], e["argmax_origin"], e["argmax_orthant"])


def test_triangle_inequality_fails_with_sample_origins(oracle_mod):
    """The appendix proof assumes a common evaluation grid; with origins drawn
    from the samples themselves the triangle inequality can fail."""
    X = np.array([[0, 1], [0, 0]], np.float32)
    Y = np.array([[1, 1], [1, 0]], np.float32)
    Z = np.array([[0, 0], [2, 0], [1, 1]], np.float32)
    dxy = oracle_mod.distance(X, Y).D
    dxz = oracle_mod.distance(X, Z).D
    dzy = oracle_mod.distance(Z, Y).D
    for A, B in ((X, Y), (X, Z), (Z, Y)):
        num, den, _, _ = ddks_tensor(A, B)
        assert oracle_mod.distance(A, B).num == num
    assert dxy == 1.0
    assert dxy > dxz + dzy


# ---------------------------------------------------------------- d = 1

@pytest.mark.parametrize("seed", range(6))
def test_d1_equals_two_sample_ks(oracle_mod, seed):
    from scipy.stats import ks_2samp
    g = np.random.default_rng(seed)
    a = g.integers(-5, 6, size=int(g.integers(1, 40))).astype(np.float32)
    b = g.integers(-4, 8, size=int(g.integers(1, 40))).astype(np.float32)
    r = oracle_mod.distance(a[:, None], b[:, None])
    num, den = ks_1d_sortmerge(a, b)
    assert (r.num, r.den) == (num, den)
    assert math.isclose(r.D, ks_2samp(a, b).statistic, rel_tol=0, abs_tol=1e-12)


def test_d1_continuous_large(oracle_mod):
    from scipy.stats import ks_2samp
    g = np.random.default_rng(7)
    a = g.standard_normal(700).astype(np.float32)
    b = (g.standard_normal(900) * 1.3).astype(np.float32)
    r = oracle_mod.distance(a[:, None], b[:, None], threads=4)
    assert (r.num, r.den) == ks_1d_sortmerge(a, b)
    assert math.isclose(r.D, ks_2samp(a, b).statistic, abs_tol=1e-12)


# ---------------------------------------------------------------- tensor form

small_sets = st.integers(1, 4).flatmap(lambda d: st.tuples(
    st.just(d),
    st.lists(st.lists(st.integers(-2, 2), min_size=d, max_size=d), min_size=1, max_size=9),
    st.lists(st.lists(st.integers(-2, 2), min_size=d, max_size=d), min_size=1, max_size=9)))


@settings(max_examples=150, deadline=None)
@given(small_sets)
def test_matches_tensor_formulation(oracle_mod, case):
    d, P, Q = case
    P = np.array(P, np.float32).reshape(-1, d)
    Q = np.array(Q, np.float32).reshape(-1, d)
    r = oracle_mod.distance(P, Q, counts=True)
    num, den, MP, MQ = ddks_tensor(P, Q)
    assert (r.num, r.den) == (num, den)
    np.testing.assert_array_equal(r.counts[:, :, 0], MP)
    np.testing.assert_array_equal(r.counts[:, :, 1], MQ)


def test_matches_tensor_formulation_random_real(oracle_mod):
    g = np.random.default_rng(11)
    for d in range(1, 6):
        P = g.standard_normal((23, d)).astype(np.float32)
        Q = (g.standard_normal((17, d)) + 0.3).astype(np.float32)
        r = oracle_mod.distance(P, Q, counts=True, threads=3)
        num, den, MP, MQ = ddks_tensor(P, Q)
        assert (r.num, r.den) == (num, den)
        np.testing.assert_array_equal(r.counts[:, :, 0], MP)


def test_exhaustive_tiny_binary_grid(oracle_mod):
    """Every pair of 2-point samples on {0,1}^2 (with repetition)."""
    pts = [np.array([a, b], np.float32) for a in (0, 1) for b in (0, 1)]
    for i in range(4):
        for j in range(4):
            for k in range(4):
                for l in range(4):
                    P = np.stack([pts[i], pts[j]])
                    Q = np.stack([pts[k], pts[l]])
                    assert oracle_mod.distance(P, Q).num == ddks_tensor(P, Q)[0]


# ---------------------------------------------------------------- invariants

def _rand_case(seed, d=None, lo=-3, hi=3):
    g = np.random.default_rng(seed)
    d = d or int(g.integers(1, 5))
    P = g.integers(lo, hi + 1, size=(int(g.integers(1, 15)), d)).astype(np.float32)
    Q = g.integers(lo, hi + 1, size=(int(g.integers(1, 15)), d)).astype(np.float32)
    return g, P, Q


@pytest.mark.parametrize("seed", range(10))
def test_identity_and_row_permutation(oracle_mod, seed):
    g, P, _ = _rand_case(seed)
    assert oracle_mod.distance(P, P).num == 0
    assert oracle_mod.distance(P, P[g.permutation(len(P))]).num == 0


@pytest.mark.parametrize("seed", range(10))
def test_symmetry_and_count_swap(oracle_mod, seed):
    _, P, Q = _rand_case(seed)
    a = oracle_mod.distance(P, Q, counts=True)
    b = oracle_mod.distance(Q, P, counts=True)
    assert a.num == b.num and a.den == b.den
    n_p = len(P)
    # origins swap blocks, samples swap
    sw = np.concatenate([b.counts[len(Q):], b.counts[:len(Q)]])[:, :, ::-1]
    np.testing.assert_array_equal(a.counts, sw)
    assert 0 <= a.num <= a.den
    assert n_p * len(Q) == a.den


@pytest.mark.parametrize("seed", range(10))
def test_count_partition_and_self_count(oracle_mod, seed):
    _, P, Q = _rand_case(seed)
    r = oracle_mod.distance(P, Q, counts=True)
    assert (r.counts[:, :, 0].sum(axis=1) == len(P)).all()
    assert (r.counts[:, :, 1].sum(axis=1) == len(Q)).all()
    top = r.counts.shape[1] - 1
    assert (r.counts[:len(P), top, 0] >= 1).all()
    assert (r.counts[len(P):, top, 1] >= 1).all()


@pytest.mark.parametrize("seed", range(8))
def test_row_order_replication_constant_dim_axis_perm(oracle_mod, seed):
    g, P, Q = _rand_case(seed)
    base = oracle_mod.distance(P, Q)
    r = oracle_mod.distance(P[g.permutation(len(P))], Q[g.permutation(len(Q))])
    assert r.num == base.num
    r = oracle_mod.distance(np.concatenate([P, P]), np.concatenate([Q, Q]))
    assert r.D == base.D and r.num == 4 * base.num
    c = np.float32(g.integers(-3, 4))
    r = oracle_mod.distance(np.hstack([P, np.full((len(P), 1), c, np.float32)]),
                            np.hstack([Q, np.full((len(Q), 1), c, np.float32)]))
    assert r.num == base.num
    perm = g.permutation(P.shape[1])
    assert oracle_mod.distance(P[:, perm], Q[:, perm]).num == base.num


@pytest.mark.parametrize("seed", range(8))
def test_strictly_increasing_maps(oracle_mod, seed):
    g = np.random.default_rng(100 + seed)
    d = int(g.integers(1, 5))
    P = g.standard_normal((int(g.integers(2, 30)), d)).astype(np.float32)
    Q = (g.standard_normal((int(g.integers(2, 30)), d)) * 1.5).astype(np.float32)
    base = oracle_mod.distance(P, Q)
    # exact power-of-two scaling
    assert oracle_mod.distance(P * np.float32(8), Q * np.float32(8)).num == base.num
    # per-dimension dense rank (strictly increasing, exact in fp32)
    Z = np.concatenate([P, Q])
    R = np.empty_like(Z)
    for m in range(d):
        _, inv = np.unique(Z[:, m], return_inverse=True)
        R[:, m] = inv.astype(np.float32)
    assert oracle_mod.distance(R[:len(P)], R[len(P):]).num == base.num
    # monotone cubic on values where it stays exact order-wise
    C = np.cbrt(Z.astype(np.float64)).astype(np.float32)
    if len(np.unique(C, axis=0)) == len(np.unique(Z, axis=0)):
        ok = all(len(np.unique(C[:, m])) == len(np.unique(Z[:, m])) for m in range(d))
        if ok:
            assert oracle_mod.distance(C[:len(P)], C[len(P):]).num == base.num


def test_signed_zero_and_denormals(oracle_mod):
    """-0 compares equal to +0; denormals are ordered exactly."""
    P = np.array([[0.0, 1e-45], [-0.0, 2e-45]], np.float32)
    Q = np.array([[-0.0, 0.0], [0.0, -1e-45]], np.float32)
    a = oracle_mod.distance(P, Q)
    Pc, Qc = P.copy(), Q.copy()
    Pc[Pc == 0] = 0.0
    Qc[Qc == 0] = 0.0
    assert oracle_mod.distance(Pc, Qc).num == a.num
    assert a.num == ddks_tensor(P, Q)[0]
    # scaling denormals up by 2^60 is exact and strictly increasing
    s = np.float32(2.0 ** 60)
    assert oracle_mod.distance(P * s, Q * s).num == a.num


def test_threads_do_not_change_result(oracle_mod):
    g = np.random.default_rng(5)
    P = np.rint(g.standard_normal((150, 3)) * 2).astype(np.float32)
    Q = np.rint(g.standard_normal((130, 3)) * 2).astype(np.float32)
    a = oracle_mod.distance(P, Q, counts=True, per_origin=True)
    for t in (2, 3, 7, 64):
        b = oracle_mod.distance(P, Q, counts=True, per_origin=True, threads=t)
        assert (a.num, a.argmax_origin, a.argmax_orthant) == (b.num, b.argmax_origin,
                                                              b.argmax_orthant)
        np.testing.assert_array_equal(a.counts, b.counts)
        np.testing.assert_array_equal(a.origin_num, b.origin_num)


def test_argmax_is_first_maximiser(oracle_mod):
    g = np.random.default_rng(9)
    P = g.integers(0, 3, size=(12, 2)).astype(np.float32)
    Q = g.integers(1, 4, size=(9, 2)).astype(np.float32)
    r = oracle_mod.distance(P, Q, counts=True, per_origin=True)
    n_p, n_q = len(P), len(Q)
    s = np.abs(r.counts[:, :, 0].astype(np.int64) * n_q - r.counts[:, :, 1].astype(np.int64) * n_p)
    flat = int(np.argmax(s.reshape(-1)))  # numpy argmax returns the first maximiser
    assert (r.argmax_origin, r.argmax_orthant) == divmod(flat, s.shape[1])
    np.testing.assert_array_equal(r.origin_num, s.max(axis=1).astype(np.uint64))


def test_origin_counts_subset_matches_full(oracle_mod):
    g = np.random.default_rng(21)
    P = np.rint(g.standard_normal((40, 3)) * 3).astype(np.float32)
    Q = np.rint(g.standard_normal((31, 3)) * 3).astype(np.float32)
    full = oracle_mod.distance(P, Q, counts=True).counts
    idx = np.array([0, 5, 39, 40, 70, 12])
    np.testing.assert_array_equal(oracle_mod.origin_counts(P, Q, idx), full[idx])
    num, _, MP, MQ = ddks_tensor(P, Q)
    np.testing.assert_array_equal(oracle_mod.origin_counts(P, Q, idx)[:, :, 1], MQ[idx])
