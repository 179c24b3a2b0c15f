"""Pins for the oracle's rdKS (Sec. 2.2.3, Alg. 2, radial approximation).
Readings: d + 1 corners of the pooled-normalised space (origin and unit
points), squared Euclidean distances in fp32 with every operation rounded on
its own, and per corner the two-sample KS statistic of the distance lists
(thresholds at distinct distances, absolute difference).  CPU only."""
import numpy as np
import pytest
from scipy.stats import ks_2samp


def distances_f32(P, Q):
    """[corner, point] squared distances, the same fp32 steps as the reading."""
    Z = np.concatenate([P, Q]).astype(np.float32)
    lo, hi = Z.min(axis=0), Z.max(axis=0)
    span = (hi - lo).astype(np.float32)
    diff = (Z - lo).astype(np.float32)
    with np.errstate(invalid="ignore", divide="ignore"):
        u = np.where(hi > lo, diff / np.where(hi > lo, span, np.float32(1)), np.float32(0)).astype(np.float32)
    d = Z.shape[1]
    out = np.zeros((d + 1, len(Z)), np.float32)
    for c in range(d + 1):
        acc = np.zeros(len(Z), np.float32)
        for m in range(d):
            t = (u[:, m] - np.float32(1.0 if c == m + 1 else 0.0)).astype(np.float32)
            acc = (acc + (t * t).astype(np.float32)).astype(np.float32)
        out[c] = acc
    return out


def ks_numerators_brute(P, Q):
    """Per corner: max over every pooled distance r of |c_P(<= r) n_q - c_Q(<= r) n_p|."""
    n_p, n_q = len(P), len(Q)
    dist = distances_f32(P, Q)
    res = []
    for c in range(dist.shape[0]):
        dp, dq = dist[c, :n_p], dist[c, n_p:]
        r = dist[c][:, None]
        cp = (dp[None, :] <= r).sum(axis=1).astype(np.int64)
        cq = (dq[None, :] <= r).sum(axis=1).astype(np.int64)
        res.append(int(np.abs(cp * n_q - cq * n_p).max()))
    return res


@pytest.mark.parametrize("n_p,n_q,ties", [(40, 55, False), (200, 130, False), (90, 90, True)])
def test_rdks_d1_is_the_ks_statistic(oracle_mod, n_p, n_q, ties):
    g = np.random.default_rng(n_p + n_q)
    P = g.standard_normal((n_p, 1))
    Q = g.standard_normal((n_q, 1)) * 1.5 + 0.2
    if ties:
        P, Q = np.rint(P * 2), np.rint(Q * 2)
    P, Q = P.astype(np.float32), Q.astype(np.float32)
    r = oracle_mod.rdks(P, Q)
    assert abs(r.D - ks_2samp(P[:, 0], Q[:, 0]).statistic) < 1e-15
    assert r.num == oracle_mod.distance(P, Q).num
    assert list(r.per_corner) == [r.num, r.num]  # from 0 and from 1: the same ECDF gap


@pytest.mark.parametrize("d,n_p,n_q", [(2, 60, 70), (3, 150, 120), (5, 80, 200), (9, 50, 40)])
def test_rdks_matches_brute_force(oracle_mod, d, n_p, n_q):
    g = np.random.default_rng(d * 7 + n_p)
    P = g.standard_normal((n_p, d)).astype(np.float32)
    Q = (g.standard_normal((n_q, d)) + 0.3).astype(np.float32)
    Q[:5] = P[:5]  # shared points: equal distances across the samples
    r = oracle_mod.rdks(P, Q)
    brute = ks_numerators_brute(P, Q)
    assert list(r.per_corner) == brute
    assert r.num == max(brute) and r.argmax_corner == brute.index(max(brute))


def test_rdks_invariants(oracle_mod):
    g = np.random.default_rng(11)
    P = g.standard_normal((120, 4)).astype(np.float32)
    Q = (g.standard_normal((100, 4)) * 0.8).astype(np.float32)
    r = oracle_mod.rdks(P, Q)
    assert 0 <= r.num <= r.den
    assert oracle_mod.rdks(Q, P).num == r.num  # symmetric
    assert oracle_mod.rdks(P, P.copy()).num == 0  # identical samples
    # exact rescaling of every coordinate (a power of two) leaves the
    # normalised coordinates, hence every distance, unchanged
    r4 = oracle_mod.rdks(P * np.float32(4), Q * np.float32(4))
    assert r4.num == r.num and list(r4.per_corner) == list(r.per_corner)
    # a constant dimension adds the same amount to every distance of a corner
    Pc = np.concatenate([P, np.full((120, 1), 3, np.float32)], axis=1)
    Qc = np.concatenate([Q, np.full((100, 1), 3, np.float32)], axis=1)
    rc = oracle_mod.rdks(Pc, Qc)
    assert list(rc.per_corner[:5]) == list(r.per_corner)


@pytest.mark.parametrize("d,n_p,n_q,k", [(2, 70, 90, 3), (3, 120, 100, 4), (6, 60, 75, 2), (12, 40, 55, 3)])
def test_rdks_exact_on_a_dyadic_lattice(oracle_mod, d, n_p, n_q, k):
    """An independent pin of the d > 1 distances: coordinates on {0, .., 2^k}
    with both ends present in every dimension normalise to multiples of
    2^-k, so every squared distance from a corner is a multiple of 2^-2k below
    d + 1 and exact in fp32, whatever the order of the operations.  The
    distances are then computed in exact integer arithmetic (units of 2^-2k),
    and the per-corner statistic is scipy's two-sample KS statistic of the
    two distance lists."""
    g = np.random.default_rng(1000 + d)
    top = 2 ** k
    P = g.integers(0, top + 1, size=(n_p, d))
    Q = g.integers(0, top + 1, size=(n_q, d))
    P[0], Q[0] = 0, top  # both ends of every dimension present
    r = oracle_mod.rdks(P.astype(np.float32), Q.astype(np.float32))
    Z = np.concatenate([P, Q]).astype(np.int64)
    for c in range(d + 1):
        corner = np.zeros(d, np.int64)
        if c > 0:
            corner[c - 1] = top
        dist = ((Z - corner) ** 2).sum(axis=1)  # exact, in units of 2^-2k
        ks = ks_2samp(dist[:n_p], dist[n_p:]).statistic
        assert abs(r.per_corner[c] / (n_p * n_q) - ks) < 1e-12, c
