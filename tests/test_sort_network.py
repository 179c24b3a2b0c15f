"""Host-side check of the tile-sort network schedule that k_rank_sort32 (32-bit
keys) and k_rank_pairs (64-bit (key, index) pairs) run on the GPU: a NumPy
model of the same stages on an (NT threads x KPT registers) tile, with each
cross-lane move written out as the lane operation the kernel uses (DPP quad
permutations, mirrors and bank-masked row shifts, the gfx950 permlane swaps,
LDS exchanges between waves).  The element type does not enter the schedule,
so the model runs on uint64 values.  CPU only."""
import numpy as np
import pytest

LANES = np.arange(64)


def wave_take(x, src):
    """x: (NT,) values; every lane l of every wave reads lane src[l] of its wave."""
    nt = x.shape[0]
    base = (np.arange(nt) // 64) * 64
    return x[base + np.tile(src, nt // 64)]


def bank(l):
    return (l % 16) // 4


def dpp_into(old, src, shift, banks):
    """update_dpp with a row shift (shift > 0: lane l reads l - shift of its
    row; < 0: l + |shift|) written only into the lanes of the given banks."""
    nt = old.shape[0]
    l = np.tile(LANES, nt // 64)
    sel = np.isin(bank(l), banks)
    moved = wave_take(src, np.clip(LANES - shift, 0, 63))
    return np.where(sel, moved, old)


def permlane_swap(x, y, a):
    """a = 16: odd 16-lane rows of x swapped with the even rows of y; a = 32:
    the upper half of x with the lower half of y."""
    l = np.tile(LANES, x.shape[0] // 64)
    hi = (l & a) != 0
    x2 = np.where(hi, wave_take(y, LANES ^ a), x)
    y2 = np.where(hi, y, wave_take(x, LANES ^ a))
    return x2, y2


def flip_lanes(x, lm, lane):
    mirror = {1: LANES ^ 1, 2: LANES ^ 3, 3: LANES ^ 7, 4: LANES ^ 15}
    if lm <= 4:
        return wave_take(x, mirror[lm])
    y = wave_take(x, LANES ^ 15)
    a, b = permlane_swap(y, y, 16)
    y = np.where(lane & 16, a, b)
    if lm == 6:
        a, b = permlane_swap(y, y, 32)
        y = np.where(lane & 32, a, b)
    return y


def cross_wave(v, tid, m, flip):
    p = v[tid ^ m]
    if flip:
        p = p[:, ::-1]
    lower = (tid & ((m + 1) // 2 if flip else m)) == 0
    return np.where(lower[:, None], np.minimum(v, p), np.maximum(v, p))


def sort_half(v, lj, kpt, tid, lane):
    j = 1 << lj
    if j < kpt:
        for r in range(kpt):
            if not r & j:
                lo, hi = np.minimum(v[:, r], v[:, r | j]), np.maximum(v[:, r], v[:, r | j])
                v[:, r], v[:, r | j] = lo, hi
    elif j <= 2 * kpt:
        a = j // kpt
        lower = (lane & a) == 0
        for r in range(kpt):
            p = wave_take(v[:, r], LANES ^ a)
            v[:, r] = np.where(lower, np.minimum(v[:, r], p), np.maximum(v[:, r], p))
    elif j <= 8 * kpt:
        a = j // kpt
        low, high = ([0, 2], [1, 3]) if a == 4 else ([0, 1], [2, 3])
        for b in range(kpt // 2):
            X, Y = v[:, 2 * b].copy(), v[:, 2 * b + 1].copy()
            X1 = dpp_into(X, Y, a, high)
            Y1 = dpp_into(Y, X, -a, low)
            mn, mx = np.minimum(X1, Y1), np.maximum(X1, Y1)
            v[:, 2 * b] = dpp_into(mn, mx, a, high)
            v[:, 2 * b + 1] = dpp_into(mx, mn, -a, low)
    elif j <= 32 * kpt:
        a = j // kpt
        for b in range(kpt // 2):
            x, y = permlane_swap(v[:, 2 * b].copy(), v[:, 2 * b + 1].copy(), a)
            mn, mx = permlane_swap(np.minimum(x, y), np.maximum(x, y), a)
            v[:, 2 * b], v[:, 2 * b + 1] = mn, mx
    else:
        v[:] = cross_wave(v, tid, j // kpt, False)
    if lj > 0:
        sort_half(v, lj - 1, kpt, tid, lane)


def sort_tile(v, kpt):
    nt = v.shape[0]
    tid = np.arange(nt)
    lane = tid & 63
    log_kpt = kpt.bit_length() - 1
    for lk in range(1, log_kpt + nt.bit_length()):
        k = 1 << lk
        if k <= kpt:
            for r in range(kpt):
                if not r & (k // 2):
                    a, b = v[:, r].copy(), v[:, r ^ (k - 1)].copy()
                    v[:, r], v[:, r ^ (k - 1)] = np.minimum(a, b), np.maximum(a, b)
        elif k <= 64 * kpt:
            lower = (lane & (k // (2 * kpt))) == 0
            p = np.stack([flip_lanes(v[:, kpt - 1 - r], lk - log_kpt, lane) for r in range(kpt)], axis=1)
            v[:] = np.where(lower[:, None], np.minimum(v, p), np.maximum(v, p))
        else:
            v[:] = cross_wave(v, tid, k // kpt - 1, True)
        if lk >= 2:
            sort_half(v, lk - 2, kpt, tid, lane)
    return v


@pytest.mark.parametrize("kpt,nt", [(8, 512), (4, 64), (4, 256), (4, 1024), (16, 256)])
def test_network_sorts_every_tile_shape(kpt, nt):
    g = np.random.default_rng(kpt * 1000 + nt)
    for trial in range(3):
        vals = g.integers(0, 2**63, size=nt * kpt, dtype=np.uint64)
        if trial == 1:
            vals = vals % np.uint64(7)  # many equal values
        if trial == 2:
            vals[nt * kpt // 3:] = np.uint64(2**64 - 1)  # the padding past N
        out = sort_tile(vals.reshape(nt, kpt).copy(), kpt)
        assert np.array_equal(out.reshape(-1), np.sort(vals))  # thread tid holds elements kpt tid ..


def test_model_lane_operations():
    """The lane moves of the model: a flip within the wave is lane ^ (2^LM - 1)
    for every LM, and the register-pair exchanges compare lane l with l ^ A."""
    x = np.arange(128, dtype=np.uint64)
    lane = np.arange(128) & 63
    for lm in range(1, 7):
        assert np.array_equal(flip_lanes(x, lm, lane), (np.arange(128) ^ ((1 << lm) - 1)).astype(np.uint64))
    for a in (16, 32):
        s0, s1 = permlane_swap(x, x, a)
        assert np.array_equal(np.where(lane & a, s0, s1), (np.arange(128) ^ a).astype(np.uint64))
