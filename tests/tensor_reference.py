"""An independent, tiny-input formulation of ddKS used to pin the oracle.

It follows the paper's tensor method (Sec. 2.2.1) rather than the oracle's
binning loop: Eq. (g) builds the comparison tensors G = X >= S, and
Eq. (membership) evaluates each orthant separately as a product over
dimensions of square-wave selectors.  As printed, the selector's frequency
2^{-m-2} applied to G in {0,1} is constant; the reading used here (and
recorded in the design notes) applies the square wave to the orthant index j:
Sq(j, 2^{-m}) (1-based m) is 1 exactly when bit m-1 of j is clear, and the
point is in orthant j when every G[m] equals that bit.  Eq. (d1) then takes
the maximum absolute difference of the normalised memberships over the
concatenation of both origin sets.
"""
import numpy as np


def square_wave(x, f):
    """Sq(x, f) = ((-1)^floor(2 f x) + 1) / 2."""
    return ((-1.0) ** np.floor(2.0 * f * np.asarray(x, dtype=np.float64)) + 1.0) / 2.0


def membership(X, S):
    """M_{X,S}[k, j] = sum_i prod_m [G[i,m,k] == bit_{m}(j)] with G = X >= S^T."""
    X = np.asarray(X, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    d = X.shape[1]
    G = (X[:, :, None] >= S.T[None, :, :]).astype(np.float64)  # n_X x d x n_S
    M = np.zeros((S.shape[0], 1 << d), dtype=np.int64)
    for j in range(1 << d):
        ind = np.ones((X.shape[0], S.shape[0]))
        for m in range(1, d + 1):  # 1-based as in the paper
            sq = square_wave(j, 2.0 ** (-m))  # 1 when bit m-1 of j is clear
            ind = ind * np.abs(G[:, m - 1, :] - sq)
        M[:, j] = np.rint(ind.sum(axis=0)).astype(np.int64)
    return M


def ddks_tensor(P, Q):
    """(num, den) with D = num/den, evaluated at both origin sets."""
    P = np.asarray(P, dtype=np.float32)
    Q = np.asarray(Q, dtype=np.float32)
    n_p, n_q = P.shape[0], Q.shape[0]
    S = np.concatenate([P, Q])
    MP = membership(P, S)
    MQ = membership(Q, S)
    diff = np.abs(MP * n_q - MQ * n_p)
    return int(diff.max()), n_p * n_q, MP, MQ


def ks_1d_sortmerge(a, b):
    """Two-sample 1-D KS statistic sup_x |F_a(x) - F_b(x)| as an exact fraction
    (num, den=len(a)*len(b)), by walking the merged sorted values."""
    a = np.sort(np.asarray(a, dtype=np.float64).ravel())
    b = np.sort(np.asarray(b, dtype=np.float64).ravel())
    na, nb = a.size, b.size
    vals = np.unique(np.concatenate([a, b]))
    best = 0
    for v in vals:
        ca = np.searchsorted(a, v, side="right")
        cb = np.searchsorted(b, v, side="right")
        best = max(best, abs(ca * nb - cb * na))
    return best, na * nb
