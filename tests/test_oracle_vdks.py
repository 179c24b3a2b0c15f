"""Pins for the oracle's vdKS (Sec. 2.2.2, Alg. 1, voxel approximation).
Readings: pooled per-dimension normalisation onto [0, 1], voxel coordinate
min(V-1, floor(u V)) in fp64, orthants split with >= per voxel coordinate
(Eq. g), absolute difference of the samples' proportions (Eq. d1).  CPU only."""
import itertools
from fractions import Fraction

import numpy as np
import pytest


def voxel_coords(P, Q, V):
    """Voxel coordinates of P and Q (fp64 arithmetic, same steps as the reading)."""
    Z = np.concatenate([P, Q]).astype(np.float64)
    lo, hi = Z.min(axis=0), Z.max(axis=0)
    span = hi - lo
    u = np.where(span > 0, (Z - lo) / np.where(span > 0, span, 1.0), 0.0)
    v = np.minimum(np.floor(u * V), V - 1).astype(np.int64)
    return v[:len(P)], v[len(P):]


def alg1_fraction(P, Q, V):
    """Alg. 1 written out: voxel occupation proportions of each sample over all
    V^d voxels, Diff = T - P, and for every filled voxel the maximum absolute
    sum of Diff over each of its orthants (exact fractions)."""
    vp, vq = voxel_coords(P, Q, V)
    d = P.shape[1]
    occ = {}
    for row in vp:
        occ.setdefault(tuple(row), [0, 0])[0] += 1
    for row in vq:
        occ.setdefault(tuple(row), [0, 0])[1] += 1
    n_p, n_q = len(P), len(Q)
    diff = {k: Fraction(c[1], n_q) - Fraction(c[0], n_p) for k, c in occ.items()}
    best = Fraction(0)
    for u in occ:  # filled voxels
        sums = [Fraction(0)] * (1 << d)
        for w in itertools.product(range(V), repeat=d):
            j = sum(1 << m for m in range(d) if w[m] >= u[m])
            sums[j] += diff.get(w, Fraction(0))
        best = max(best, max(abs(x) for x in sums))
    return best


@pytest.mark.parametrize("d,V,n_p,n_q", [(1, 5, 30, 40), (2, 3, 25, 20), (2, 4, 40, 31), (3, 3, 20, 26)])
def test_vdks_matches_alg1_written_out(oracle_mod, d, V, n_p, n_q):
    g = np.random.default_rng(d * 10 + V)
    P = g.standard_normal((n_p, d)).astype(np.float32)
    Q = (g.standard_normal((n_q, d)) * 1.3 + 0.2).astype(np.float32)
    r = oracle_mod.vdks(P, Q, V)
    assert Fraction(r.num, r.den) == alg1_fraction(P, Q, V)


@pytest.mark.parametrize("d,V", [(2, 4), (3, 8), (4, 6), (5, 3)])
def test_vdks_is_ddks_of_the_voxel_coordinates(oracle_mod, d, V):
    g = np.random.default_rng(100 + d)
    P = g.standard_normal((300, d)).astype(np.float32)
    Q = (g.standard_normal((250, d)) + 0.25).astype(np.float32)
    r = oracle_mod.vdks(P, Q, V)
    vp, vq = voxel_coords(P, Q, V)
    o = oracle_mod.distance(vp.astype(np.float32), vq.astype(np.float32))
    assert r.num == o.num and r.den == o.den
    # the reported maximiser attains the maximum, and it is a filled voxel
    u = np.array([(r.argmax_voxel // V ** m) % V for m in range(d)])
    code = lambda v: ((v >= u) * (1 << np.arange(d))).sum(axis=1)
    cp = np.bincount(code(vp), minlength=1 << d)
    cq = np.bincount(code(vq), minlength=1 << d)
    assert abs(int(cp[r.argmax_orthant]) * 250 - int(cq[r.argmax_orthant]) * 300) == r.num
    assert any((np.concatenate([vp, vq]) == u).all(axis=1))
    assert r.n_filled == len({tuple(x) for x in np.concatenate([vp, vq])})


@pytest.mark.parametrize("d,V", [(1, 7), (2, 5), (3, 4)])
def test_vdks_on_a_lattice_is_exact(oracle_mod, d, V):
    """Integer data on {0..V-1} with both ends present: each value gets its own
    voxel, in order, so vdKS equals the exact statistic."""
    g = np.random.default_rng(7 * d + V)
    P = g.integers(0, V, size=(60, d)).astype(np.float32)
    Q = g.integers(0, V, size=(45, d)).astype(np.float32)
    P[0], P[1] = 0, V - 1
    assert oracle_mod.vdks(P, Q, V).num == oracle_mod.distance(P, Q).num


def test_vdks_one_voxel_and_constant_dimension(oracle_mod):
    g = np.random.default_rng(3)
    P = g.standard_normal((40, 2)).astype(np.float32)
    Q = (g.standard_normal((50, 2)) + 1).astype(np.float32)
    assert oracle_mod.vdks(P, Q, 1).num == 0  # everything in one voxel
    r = oracle_mod.vdks(P, Q, 6)
    Pc = np.concatenate([P, np.full((40, 1), 2.5, np.float32)], axis=1)
    Qc = np.concatenate([Q, np.full((50, 1), 2.5, np.float32)], axis=1)
    rc = oracle_mod.vdks(Pc, Qc, 6)
    assert rc.num == r.num and rc.n_filled == r.n_filled
    # symmetry in the two samples
    assert oracle_mod.vdks(Q, P, 6).num == r.num
