// Rank encoding for the 16-bit compare path.
//
// The sweep only ever asks whether x_m >= o_m for points and origins drawn
// from the same pooled set, so any map of each dimension's values onto
// integers that is strictly increasing on the values present gives exactly
// the same orthant codes.  With at most 65536 distinct values per dimension
// the ranks fit int16 (biased by -32768) and one saturating v_pk_sub_i16
// compares two dimensions.
//
// N <= 65536 (grid.y = dimension):
//   1. k_rank_sort32  sorts each tile of STILE order keys (an order-preserving
//                     uint32 image of the fp32 value) in registers, wave
//                     shuffles and LDS (bitonic network).
//   2. k_rank_count   stages every sorted tile in LDS in turn and adds up,
//                     for each of its points, the values of the tile strictly
//                     below its own (binary search): the rank, the number of
//                     pooled values below the point, fits 16 bits since
//                     N <= 65536.
// N > 65536:
//   1. k_rank_pairs   sorts tiles of (key, index) pairs (the same bitonic
//                     network on 64-bit values: registers, DPP, permlane
//                     swaps and LDS);
//   2. k_rank_place_count adds up, per pair, the pairs below it in every
//                     tile (binary searches in LDS-staged tiles), and
//      k_rank_scatter writes each pair at that sorted position;
//      k_rank_flags   counts first occurrences per segment,
//      k_rank_dense   dense rank = number of distinct values below, from the
//                     segment counts and a block scan; records the
//                     distinct-value count.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ddks_internal.h"

namespace ddks {

static constexpr int TILE = 4096;      // pairs per sorted tile (32 KB of LDS)
static constexpr int SEG = 4096;       // positions per flag segment
static constexpr int SEG_THREADS = 1024;

// Order-preserving image of a finite fp32 value (+0 and -0 are both mapped
// to +0 upstream): unsigned comparison of images == fp32 comparison.
__device__ __forceinline__ uint32_t order_key(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ------------------------------------------------------------ N <= 65536

// Value of point i in dimension m, P then Q (Q unread while i < n_p), with -0
// mapped to +0 so that the two compare equal.
__device__ __forceinline__ float point_value(const float *__restrict__ P, int64_t n_p,
                                             const float *__restrict__ Q, int64_t i, int d, int m)
{
    return (i < n_p ? P[i * d + m] : Q[(i - n_p) * d + m]) + 0.0f;
}

// Tiles of the N <= 65536 path: 2^LOG_STILE keys, sorted by one block of
// S32_THREADS threads holding SKPT keys each (4096 keys, 512 threads x 8:
// two waves per SIMD hide the exchange latencies that one wave of 16 keys
// per thread left exposed, 10.6 against 12.2 us at 40000 points x 4
// dimensions; 2048-key tiles sorted in 7.0 us but made the count slower).
#ifndef DDKS_STILE_LOG
#define DDKS_STILE_LOG 12
#endif
#ifndef DDKS_SORT_KPT
#define DDKS_SORT_KPT 8
#endif
static constexpr int LOG_STILE = DDKS_STILE_LOG;
static constexpr int STILE = 1 << LOG_STILE;
static constexpr int SKPT = DDKS_SORT_KPT;  // keys per thread
static constexpr int S32_THREADS = STILE / SKPT;
static_assert((SKPT == 4 || SKPT == 8 || SKPT == 16) && S32_THREADS >= 256 && S32_THREADS <= 1024, "tile size");

// ---- the tile sort: a bitonic network on KPT values per thread (element
// e = KPT tid + r of the tile in register r of thread tid), in the form where
// every compare-exchange puts the minimum at the lower element: phase lk
// (blocks of 2^lk elements) first pairs e with e ^ (2^lk - 1) (the "flip",
// which merges two sorted runs read in opposite directions), then e with
// e ^ j for j = 2^(lk-2) .. 1.  Distances below KPT are exchanges between a
// thread's registers; KPT .. 32 KPT are lane distances 1 .. 32 within a
// wave, exchanged through DPP and the gfx950 permlane swaps (no LDS traffic);
// the stages that cross waves go through LDS.  The values are 32-bit keys
// (k_rank_sort32) or 64-bit (key, index) pairs (k_rank_pairs), moved as two
// 32-bit halves along the same lanes.

// DPP controls (row = 16 lanes, bank = 4 lanes of a row).
constexpr int DPP_QUAD_X1 = 0xB1;  // quad_perm [1,0,3,2]: lane ^ 1
constexpr int DPP_QUAD_X2 = 0x4E;  // quad_perm [2,3,0,1]: lane ^ 2
constexpr int DPP_QUAD_X3 = 0x1B;  // quad_perm [3,2,1,0]: lane ^ 3
constexpr int DPP_ROW_SHL = 0x100;  // + n: lane l reads lane l + n of its row
constexpr int DPP_ROW_SHR = 0x110;  // + n: lane l reads lane l - n of its row
constexpr int DPP_ROW_MIRROR = 0x140;       // lane ^ 15
constexpr int DPP_ROW_HALF_MIRROR = 0x141;  // lane ^ 7

__device__ __forceinline__ uint32_t lo32(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }
__device__ __forceinline__ uint64_t join64(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp(uint64_t x)
{
    return join64(dpp<CTRL>(lo32(x)), dpp<CTRL>(hi32(x)));
}

// src moved by CTRL into the lanes of the banks in BANKS; old elsewhere.
template <int CTRL, int BANKS>
__device__ __forceinline__ uint32_t dpp_into(uint32_t old, uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, 0xf, BANKS, false);
}
template <int CTRL, int BANKS>
__device__ __forceinline__ uint64_t dpp_into(uint64_t old, uint64_t src)
{
    return join64(dpp_into<CTRL, BANKS>(lo32(old), lo32(src)), dpp_into<CTRL, BANKS>(hi32(old), hi32(src)));
}

// Permlane swap of x and y (A = 16: the odd 16-lane rows of x with the even
// rows of y; A = 32: the upper half of x with the lower half of y).
template <int A>
__device__ __forceinline__ void permlane_swap(uint32_t &x, uint32_t &y)
{
    if constexpr (A == 16) {
        const auto s = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        x = s[0];
        y = s[1];
    } else {
        const auto s = __builtin_amdgcn_permlane32_swap(x, y, false, false);
        x = s[0];
        y = s[1];
    }
}
template <int A>
__device__ __forceinline__ void permlane_swap(uint64_t &x, uint64_t &y)
{
    uint32_t xl = lo32(x), xh = hi32(x), yl = lo32(y), yh = hi32(y);
    permlane_swap<A>(xl, yl);
    permlane_swap<A>(xh, yh);
    x = join64(xl, xh);
    y = join64(yl, yh);
}

// The value of lane l ^ A (A = 16 or 32): a permlane swap of x with itself
// leaves the partner half in one of its two results.
template <int A, typename T>
__device__ __forceinline__ T lane_xor(T x, int lane)
{
    T a = x, b = x;
    permlane_swap<A>(a, b);
    return (lane & A) ? a : b;
}

// Partner value of a flip within the wave: lane l ^ (2^LM - 1), 1 <= LM <= 6.
template <int LM, typename T>
__device__ __forceinline__ T flip_lanes(T x, int lane)
{
    if constexpr (LM == 1) return dpp<DPP_QUAD_X1>(x);
    else if constexpr (LM == 2) return dpp<DPP_QUAD_X3>(x);
    else if constexpr (LM == 3) return dpp<DPP_ROW_HALF_MIRROR>(x);
    else if constexpr (LM == 4) return dpp<DPP_ROW_MIRROR>(x);
    else if constexpr (LM == 5) return lane_xor<16>(dpp<DPP_ROW_MIRROR>(x), lane);
    else return lane_xor<32>(lane_xor<16>(dpp<DPP_ROW_MIRROR>(x), lane), lane);
}

template <typename T>
__device__ __forceinline__ void cmpx(T &lo, T &hi)
{
    const T a = min(lo, hi), b = max(lo, hi);
    lo = a;
    hi = b;
}

// The network's shape: KPT values of type T per thread, NT threads, a tile
// of 2^LOG_TILE = KPT NT values; an LDS exchange buffer of NT x KPT values
// (16-byte words, WORDS per thread).
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
template <typename T, int KPT, int NT>
struct Net {
    static constexpr int LOG_KPT = ilog2(KPT);
    static constexpr int LOG_TILE = LOG_KPT + ilog2(NT);
    static constexpr int WORDS = KPT * (int)sizeof(T) / 16;
    static_assert((KPT == 4 || KPT == 8 || KPT == 16) && (NT == 64 || NT == 256 || NT == 512 || NT == 1024),
                  "shape");
    static_assert(WORDS >= 1, "exchange words");
};

template <typename T, int KPT>
__device__ __forceinline__ uint4 pack_word(const T (&v)[KPT], int q)
{
    if constexpr (sizeof(T) == 4)
        return make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    else
        return make_uint4(lo32(v[2 * q]), hi32(v[2 * q]), lo32(v[2 * q + 1]), hi32(v[2 * q + 1]));
}
template <typename T, int KPT>
__device__ __forceinline__ void unpack_word(T (&p)[KPT], int q, uint4 x)
{
    if constexpr (sizeof(T) == 4) {
        p[4 * q] = x.x;
        p[4 * q + 1] = x.y;
        p[4 * q + 2] = x.z;
        p[4 * q + 3] = x.w;
    } else {
        p[2 * q] = join64(x.x, x.y);
        p[2 * q + 1] = join64(x.z, x.w);
    }
}

// A stage whose partner thread is tid ^ M, in another wave (M >= 64), with
// the partner's registers reversed when FLIP.
template <typename T, int KPT, int NT, int M, bool FLIP>
__device__ __forceinline__ void sort_cross_wave(T (&v)[KPT], int tid, uint4 *buf)
{
    constexpr int W = Net<T, KPT, NT>::WORDS;
    const bool lower = (tid & (FLIP ? (M + 1) / 2 : M)) == 0;
#pragma unroll
    for (int q = 0; q < W; ++q) buf[q * NT + tid] = pack_word(v, q);
    __syncthreads();
    T p[KPT];
#pragma unroll
    for (int q = 0; q < W; ++q) unpack_word(p, q, buf[q * NT + (tid ^ M)]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const T x = p[FLIP ? KPT - 1 - r : r];
        v[r] = lower ? min(v[r], x) : max(v[r], x);
    }
}

// Half-cleaner stage j = 2^LJ.
template <typename T, int KPT, int NT, int LJ>
__device__ __forceinline__ void sort_half(T (&v)[KPT], int lane, int tid, uint4 *buf)
{
    constexpr int J = 1 << LJ;
    if constexpr (J < KPT) {
#pragma unroll
        for (int r = 0; r < KPT; ++r)
            if (!(r & J)) cmpx(v[r], v[r | J]);
    } else if constexpr (J <= 2 * KPT) {
        // lane ^ 1, lane ^ 2: partner value by quad_perm
        constexpr int A = J / KPT;
        const bool lower = (lane & A) == 0;
#pragma unroll
        for (int r = 0; r < KPT; ++r) {
            const T p = dpp<A == 1 ? DPP_QUAD_X1 : DPP_QUAD_X2>(v[r]);
            v[r] = lower ? min(v[r], p) : max(v[r], p);
        }
    } else if constexpr (J <= 8 * KPT) {
        // lane ^ 4, lane ^ 8 on register pairs (X, Y): row shifts masked by
        // bank put each pair's two elements in one lane (the lower one in
        // X1), compare-exchange, then the inverse shifts put them back
        constexpr int A = J / KPT;
        constexpr int LOW = A == 4 ? 0x5 : 0x3, HIGH = A == 4 ? 0xA : 0xC;
#pragma unroll
        for (int b = 0; b < KPT / 2; ++b) {
            const T X = v[2 * b], Y = v[2 * b + 1];
            const T X1 = dpp_into<DPP_ROW_SHR + A, HIGH>(X, Y);
            const T Y1 = dpp_into<DPP_ROW_SHL + A, LOW>(Y, X);
            const T mn = min(X1, Y1), mx = max(X1, Y1);
            v[2 * b] = dpp_into<DPP_ROW_SHR + A, HIGH>(mn, mx);
            v[2 * b + 1] = dpp_into<DPP_ROW_SHL + A, LOW>(mx, mn);
        }
    } else if constexpr (J <= 32 * KPT) {
        // lane ^ 16, lane ^ 32 on register pairs: a permlane swap of the
        // pair puts each pair's two elements in one lane, the same swap undoes it
        constexpr int A = J / KPT;
#pragma unroll
        for (int b = 0; b < KPT / 2; ++b) {
            T x = v[2 * b], y = v[2 * b + 1];
            permlane_swap<A>(x, y);
            T mn = min(x, y), mx = max(x, y);
            permlane_swap<A>(mn, mx);
            v[2 * b] = mn;
            v[2 * b + 1] = mx;
        }
    } else {
        sort_cross_wave<T, KPT, NT, J / KPT, false>(v, tid, buf);
    }
    if constexpr (LJ > 0) sort_half<T, KPT, NT, LJ - 1>(v, lane, tid, buf);
}

// Phase LK: the flip, then the half-cleaners.
template <typename T, int KPT, int NT, int LK>
__device__ __forceinline__ void sort_phase(T (&v)[KPT], int lane, int tid, uint4 *buf)
{
    constexpr int K = 1 << LK;
    if constexpr (K <= KPT) {
#pragma unroll
        for (int r = 0; r < KPT; ++r)
            if (!(r & (K / 2))) cmpx(v[r], v[r ^ (K - 1)]);
    } else if constexpr (K <= 64 * KPT) {
        const bool lower = (lane & (K / (2 * KPT))) == 0;
        T p[KPT];
#pragma unroll
        for (int r = 0; r < KPT; ++r) p[r] = flip_lanes<LK - Net<T, KPT, NT>::LOG_KPT>(v[KPT - 1 - r], lane);
#pragma unroll
        for (int r = 0; r < KPT; ++r) v[r] = lower ? min(v[r], p[r]) : max(v[r], p[r]);
    } else {
        sort_cross_wave<T, KPT, NT, K / KPT - 1, true>(v, tid, buf);
    }
    if constexpr (LK >= 2) sort_half<T, KPT, NT, LK - 2>(v, lane, tid, buf);
}

// Sorts the tile held in v (KPT values per thread, NT threads) ascending:
// afterwards thread tid holds elements KPT tid .. KPT tid + KPT - 1.
template <typename T, int KPT, int NT, int LK = 1>
__device__ __forceinline__ void sort_tile(T (&v)[KPT], int lane, int tid, uint4 *buf)
{
    sort_phase<T, KPT, NT, LK>(v, lane, tid, buf);
    if constexpr (LK < Net<T, KPT, NT>::LOG_TILE) sort_tile<T, KPT, NT, LK + 1>(v, lane, tid, buf);
}

// Sorts tile blockIdx.x of dimension blockIdx.y: K[m][t][0..STILE) = the order
// keys of points t*STILE .. t*STILE+STILE-1, ascending (0xffffffff past N).
// Thread tid reads points t*STILE + tid + S32_THREADS r (coalesced; a sort does not
// care where its inputs start).  Values are read from P (points 0 .. n_p - 1)
// then Q; flags (nullable): bit 0 is set if a value is NaN or infinite.
__global__ __launch_bounds__(S32_THREADS) void k_rank_sort32(const float *__restrict__ P, int64_t n_p,
                                                             const float *__restrict__ Q, int64_t N,
                                                             int d, int64_t tiles,
                                                             uint32_t *__restrict__ K,
                                                             uint32_t *__restrict__ flags)
{
    __shared__ uint4 buf[S32_THREADS * SKPT / 4];
    const int m = blockIdx.y;
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    uint32_t v[SKPT];
    bool bad = false;
#pragma unroll
    for (int r = 0; r < SKPT; ++r) {
        const int64_t i = t * STILE + tid + r * S32_THREADS;
        const float x = i < N ? point_value(P, n_p, Q, i, d, m) : 0.0f;
        bad |= !isfinite(x);
        v[r] = i < N ? order_key(x) : 0xffffffffu;
    }
    if (flags && __any(bad) && lane == 0) atomicOr(flags, 1u);
    sort_tile<uint32_t, SKPT, S32_THREADS>(v, lane, tid, buf);
    uint4 *out = reinterpret_cast<uint4 *>(K + ((size_t)m * tiles + t) * STILE) + tid * (SKPT / 4);
#pragma unroll
    for (int q = 0; q < SKPT / 4; ++q) out[q] = make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// The sorted tile in LDS is skewed by one word every 64 entries: the probes
// of one step of the binary search sit at multiples of STILE/2^k minus one,
// which without the skew all fall in the same LDS bank.
__device__ __forceinline__ int skew(int e) { return e + (e >> 6); }

// Number of entries of the sorted, skewed LDS tile below key (branchless
// binary search; 0..STILE).  With p the entries found below so far (a
// multiple of twice the current step), the search keeps a = the LDS byte
// address of entry skew(p) = p + p/64: the probe of step j, entry
// p + j - 1, then sits at a constant byte offset from a (4 (j - 1 + j/64 - 1)
// for j >= 64, 4 (j - 1) below), folded into the LDS instruction, and taking
// the step adds 4 (j + j/64) (or 4 j) to a.  At the end p = s - s/65 with
// s = skew(p).
__device__ __forceinline__ int count_below(const uint32_t *tile, uint32_t key)
{
    typedef const __attribute__((address_space(3))) uint32_t lds_cu32;
    const uint32_t a0 = (uint32_t)(uintptr_t)(lds_cu32 *)tile;
    uint32_t a = a0;
#pragma unroll
    for (int step = STILE / 2; step >= 1; step >>= 1) {
        const uint32_t off = 4u * (uint32_t)(step - 1 + (step >= 64 ? step / 64 - 1 : 0));
        const uint32_t inc = 4u * (uint32_t)(step + (step >= 64 ? step / 64 : 0));
        const uint32_t v = *(lds_cu32 *)(uintptr_t)(a + off);
        a += v < key ? inc : 0u;
    }
    const uint32_t sk = (a - a0) >> 2;
    const int p = (int)(sk - sk / 65u);
    return p + (*(lds_cu32 *)(uintptr_t)a < key ? 1 : 0);
}

// Writes the biased 16-bit rank of dimension m of point i.
__device__ __forceinline__ void put_rank(uint16_t *R16, int64_t i, int pw, int m, int64_t rank)
{
    R16[(i * pw) * 2 + m] = (uint16_t)(uint32_t)(rank - 32768);
}

// Block (part, m) of k_rank_count<KPT, TPS> takes RC_THREADS * KPT
// consecutive points of one tile (rc_parts(KPT) blocks per tile).
static constexpr int RC_THREADS = 256;
__host__ __device__ constexpr int rc_parts(int kpt) { return STILE / (RC_THREADS * kpt); }
constexpr int RC_TILE_WORDS = STILE + STILE / 64 + 1;  // one skewed tile in LDS

// The rank in dimension m of each of the block's points: the number of pooled
// values below it, summed over all sorted tiles.  The block stages TPS tiles
// at a time in LDS (skewed; the loads of the next TPS tiles are in flight
// while these are searched) and searches them side by side (branchless
// binary searches, TPS x KPT independent chains per thread).  Ranks fit 16
// bits since N <= 65536: the biased rank is written directly, and for m = 0
// the padding dimensions of each point are zeroed.
template <int KPT, int TPS>
__global__ __launch_bounds__(RC_THREADS) void k_rank_count(const float *__restrict__ P, int64_t n_p,
                                                           const float *__restrict__ Q, int64_t N, int d,
                                                           int pw, int64_t tiles,
                                                           const uint32_t *__restrict__ K,
                                                           uint16_t *__restrict__ R16)
{
    constexpr int LOADS = STILE / (4 * RC_THREADS);  // uint4 loads per thread and tile
    __shared__ uint32_t tile[TPS][RC_TILE_WORDS];
    const int m = blockIdx.y;
    const int tid = threadIdx.x;
    const int64_t first = (int64_t)blockIdx.x * (RC_THREADS * KPT);
    uint32_t key[KPT], rank[KPT];
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int64_t i = first + tid + r * RC_THREADS;
        key[r] = i < N ? order_key(point_value(P, n_p, Q, i, d, m)) : 0u;
        rank[r] = 0;
    }
    const uint4 *src = reinterpret_cast<const uint4 *>(K + (size_t)m * tiles * STILE);
    // A group's slots past the last tile hold a copy of the last tile, whose
    // counts are dropped: no branch separates the searches, so that their
    // chains interleave.
    uint4 nxt[TPS][LOADS];
    auto load = [&](int64_t u0) {
#pragma unroll
        for (int s = 0; s < TPS; ++s) {
            const int64_t u = u0 + s < tiles ? u0 + s : tiles - 1;
#pragma unroll
            for (int c = 0; c < LOADS; ++c) nxt[s][c] = src[u * (STILE / 4) + tid + c * RC_THREADS];
        }
    };
    load(0);
    for (int64_t u0 = 0; u0 < tiles; u0 += TPS) {
        __syncthreads();  // the previous group's searches are done
#pragma unroll
        for (int s = 0; s < TPS; ++s)
#pragma unroll
            for (int c = 0; c < LOADS; ++c) {
                const int e = skew(4 * (tid + c * RC_THREADS));  // 4 entries in one 64-entry row
                tile[s][e] = nxt[s][c].x;
                tile[s][e + 1] = nxt[s][c].y;
                tile[s][e + 2] = nxt[s][c].z;
                tile[s][e + 3] = nxt[s][c].w;
            }
        __syncthreads();
        if (u0 + TPS < tiles) load(u0 + TPS);
        int cnt[TPS][KPT];
#pragma unroll
        for (int s = 0; s < TPS; ++s)
#pragma unroll
            for (int r = 0; r < KPT; ++r) cnt[s][r] = count_below(tile[s], key[r]);
#pragma unroll
        for (int s = 0; s < TPS; ++s)
#pragma unroll
            for (int r = 0; r < KPT; ++r) rank[r] += u0 + s < tiles ? (uint32_t)cnt[s][r] : 0u;
    }
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int64_t i = first + tid + r * RC_THREADS;
        if (i >= N) continue;
        put_rank(R16, i, pw, m, rank[r]);
        if (m == 0)
            for (int mm = d; mm < 2 * pw; ++mm) R16[(i * pw) * 2 + mm] = 0;
    }
}

#ifndef DDKS_RC_KPT
#define DDKS_RC_KPT 1
#endif
#ifndef DDKS_RC_TPS
#define DDKS_RC_TPS 2
#endif
static constexpr int RC_KPT = DDKS_RC_KPT, RC_TPS = DDKS_RC_TPS;


// ------------------------------------------------------------ N > 65536

// Sorts (order key << 32 | index) pairs of column m = blockIdx.y, tile t =
// blockIdx.x, KPT x NT pairs per tile (~0 past N): 256 (4 x 64), 1024
// (4 x 256) or TILE = 4096 (8 x 512), by the network of k_rank_sort32 on
// 64-bit values (partners within a wave through DPP and permlane swaps, only
// the stages across waves through LDS).  Thread tid reads pairs t * tile +
// tid + NT r (the index travels in the pair, so the sort does not care).
// S != nullptr: one tile holds the whole column, whose N pairs are written
// sorted to S + m * N.  Otherwise the sorted tile goes to A + (m * tiles + t)
// * tile, and pos (the sorted positions that k_rank_place_count accumulates)
// is cleared at the same entries.
#ifndef DDKS_PAIR_KPT
#define DDKS_PAIR_KPT 8
#endif
static constexpr int PAIR_KPT = DDKS_PAIR_KPT;
static constexpr int PAIR_THREADS = TILE / PAIR_KPT;

template <int KPT, int NT>
__global__ __launch_bounds__(NT) void k_rank_pairs(const float *__restrict__ Z, int64_t N, int d,
                                                   int64_t tiles, uint64_t *__restrict__ A,
                                                   uint64_t *__restrict__ S, uint32_t *__restrict__ pos)
{
    constexpr int TP = KPT * NT;
    __shared__ uint4 buf[NT > 64 ? NT * Net<uint64_t, KPT, NT>::WORDS : 1];
    const int m = blockIdx.y;
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    uint64_t v[KPT];
#pragma unroll
    for (int r = 0; r < KPT; ++r) {
        const int64_t i = t * TP + tid + (int64_t)r * NT;
        v[r] = i < N ? ((uint64_t)order_key(Z[i * d + m]) << 32) | (uint64_t)i : ~0ull;
    }
    sort_tile<uint64_t, KPT, NT>(v, lane, tid, buf);
    const int e0 = KPT * tid;
    if (S) {
        uint64_t *out = S + (size_t)m * N;
#pragma unroll
        for (int r = 0; r < KPT; ++r)
            if (e0 + r < N) out[e0 + r] = v[r];
    } else {
        const size_t base = ((size_t)m * tiles + t) * TP + e0;
        uint4 *a = reinterpret_cast<uint4 *>(A + base);  // A and TP: 16-byte multiples
#pragma unroll
        for (int q = 0; q < KPT / 2; ++q) a[q] = make_uint4(lo32(v[2 * q]), hi32(v[2 * q]), lo32(v[2 * q + 1]), hi32(v[2 * q + 1]));
#pragma unroll
        for (int r = 0; r < KPT; ++r) pos[base + r] = 0u;
    }
}

// Sorted position of every (key, index) pair of several sorted tiles: work
// item w of column m is (tile t, span s) = (w mod tiles, w / tiles); its block
// stages the tiles of span s in LDS one after another and adds, for each pair
// of tile t, the number of entries below it (the pairs are all distinct, so
// the sum over all tiles, its own included, is its sorted position).  The
// tile is stored skewed by one entry every 32, so that the probes of one
// search step, 4096 / 2^k entries apart, spread over the banks.
static constexpr int PLACE_THREADS = TILE / 4;  // four pairs of tile t per thread
__device__ __forceinline__ int place_skew(int e) { return e + (e >> 5); }

__global__ __launch_bounds__(PLACE_THREADS) void k_rank_place_count(const uint64_t *__restrict__ A,
                                                                    int64_t tiles, int span,
                                                                    uint32_t *__restrict__ pos)
{
    __shared__ uint64_t tile[TILE + TILE / 32];
    const int m = blockIdx.y;
    const int tid = threadIdx.x;
    const uint64_t *Am = A + (size_t)m * tiles * TILE;
    const int64_t spans = (tiles + span - 1) / span;
    for (int64_t w = blockIdx.x; w < tiles * spans; w += gridDim.x) {
        const int64_t t = w % tiles, u0 = (w / tiles) * span;
        const int64_t u1 = std::min<int64_t>(tiles, u0 + span);
        uint64_t item[4];
        uint32_t cnt[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            item[r] = Am[t * TILE + r * PLACE_THREADS + tid];
            cnt[r] = 0;
        }
        for (int64_t u = u0; u < u1; ++u) {
            __syncthreads();  // the previous tile's searches are done
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int e = r * PLACE_THREADS + tid;
                tile[place_skew(e)] = Am[u * TILE + e];
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // entries below item[r]: uniform binary search over TILE = 2^12
                int lo = 0;
#pragma unroll
                for (int step = TILE / 2; step > 0; step >>= 1)
                    lo += tile[place_skew(lo + step - 1)] < item[r] ? step : 0;
                lo += tile[place_skew(lo)] < item[r] ? 1 : 0;
                cnt[r] += (uint32_t)lo;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (item[r] != ~0ull) atomicAdd(&pos[((size_t)m * tiles + t) * TILE + r * PLACE_THREADS + tid], cnt[r]);
        __syncthreads();  // before the next work item restages the tile
    }
}

__global__ void k_rank_scatter(const uint64_t *__restrict__ A, const uint32_t *__restrict__ pos, int64_t N,
                               int64_t tiles, uint64_t *__restrict__ S)
{
    const int m = blockIdx.y;
    const uint64_t *Am = A + (size_t)m * tiles * TILE;
    const uint32_t *Pm = pos + (size_t)m * tiles * TILE;
    uint64_t *Sm = S + (size_t)m * N;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tiles * TILE;
         q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t item = Am[q];
        if (item != ~0ull) Sm[Pm[q]] = item;
    }
}

// The two launches above for C columns of `tiles` sorted tiles in A.
static hipError_t launch_place(const uint64_t *A, int64_t N, int C, int64_t tiles, uint32_t *pos, uint64_t *S,
                               hipStream_t st)
{
    // spans of several tiles once tiles^2 * C work items would far exceed the
    // chip's block slots (fewer atomic adds); never more than 32 tiles
    const int span = (int)std::max<int64_t>(1, std::min<int64_t>(32, tiles * tiles * C / 2048));
    const int64_t items = tiles * ((tiles + span - 1) / span);
    hipLaunchKernelGGL(k_rank_place_count, dim3((unsigned)std::min<int64_t>(items, 65536), C),
                       dim3(PLACE_THREADS), 0, st, A, tiles, span, pos);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned blocks = (unsigned)std::min<int64_t>((tiles * TILE + 255) / 256, 4096);
    hipLaunchKernelGGL(k_rank_scatter, dim3(blocks, C), dim3(256), 0, st, A, pos, N, tiles, S);
    return hipGetLastError();
}

__device__ __forceinline__ bool first_of_run(const uint64_t *Sm, int64_t p)
{
    return p == 0 || (Sm[p] >> 32) != (Sm[p - 1] >> 32);
}

__global__ __launch_bounds__(SEG_THREADS) void k_rank_flags(const uint64_t *__restrict__ S,
                                                            int64_t N, int64_t segs,
                                                            uint32_t *__restrict__ C,
                                                            uint32_t *__restrict__ distinct_max)
{
    __shared__ uint32_t tot;
    const int m = blockIdx.y;
    const int64_t g = blockIdx.x;
    const uint64_t *Sm = S + (size_t)m * N;
    if (threadIdx.x == 0) tot = 0;
    if (threadIdx.x == 0 && g == 0 && m == 0) *distinct_max = 0u;  // consumed by k_rank_dense
    __syncthreads();
    uint32_t c = 0;
    for (int e = threadIdx.x; e < SEG; e += SEG_THREADS) {
        int64_t p = g * SEG + e;
        if (p < N && first_of_run(Sm, p)) ++c;
    }
    atomicAdd(&tot, c);
    __syncthreads();
    if (threadIdx.x == 0) C[(size_t)m * segs + g] = tot;
}

__global__ __launch_bounds__(SEG_THREADS) void k_rank_dense(const uint64_t *__restrict__ S,
                                                            int64_t N, int d, int pw, int64_t segs,
                                                            const uint32_t *__restrict__ C,
                                                            uint16_t *__restrict__ R16,
                                                            uint32_t *__restrict__ distinct_max,
                                                            uint32_t *__restrict__ R32,
                                                            uint32_t *__restrict__ RS)
{
    constexpr int PER = SEG / SEG_THREADS;  // consecutive positions per thread
    __shared__ uint32_t scan[SEG_THREADS];
    __shared__ uint32_t before;
    const int m = blockIdx.y;
    const int64_t g = blockIdx.x;
    const uint64_t *Sm = S + (size_t)m * N;
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (int64_t h = 0; h < g; ++h) b += C[(size_t)m * segs + h];
        before = b;
        if (g == segs - 1) {
            const uint32_t total = b + C[(size_t)m * segs + g];
            atomicMax(distinct_max, total);
            distinct_max[1 + m] = total;  // this dimension's count of distinct values
            RS[(size_t)m * (N + 1) + total] = (uint32_t)N;  // end of the last run
        }
    }
    uint32_t flags[PER];
    uint32_t c = 0;
    const int64_t p0 = g * SEG + (int64_t)threadIdx.x * PER;
    for (int e = 0; e < PER; ++e) {
        int64_t p = p0 + e;
        flags[e] = (p < N && first_of_run(Sm, p)) ? 1u : 0u;
        c += flags[e];
    }
    scan[threadIdx.x] = c;
    __syncthreads();
    // inclusive Hillis-Steele scan over the block's per-thread counts
    for (int off = 1; off < SEG_THREADS; off <<= 1) {
        uint32_t v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0u;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = before + scan[threadIdx.x] - c;  // distinct values before p0
    for (int e = 0; e < PER; ++e) {
        int64_t p = p0 + e;
        if (p >= N) break;
        run += flags[e];
        const int64_t i = (int64_t)(uint32_t)Sm[p];
        const int64_t rank = (int64_t)run - 1;
        if (rank < 65536) put_rank(R16, i, pw, m, rank);
        R32[i * d + m] = (uint32_t)rank;
        if (flags[e]) RS[(size_t)m * (N + 1) + rank] = (uint32_t)p;  // first sorted position of the rank
        if (m == 0)
            for (int mm = d; mm < 2 * pw; ++mm) R16[(i * pw) * 2 + mm] = 0;
    }
}

// A dimension m with more than 65536 distinct values (shift s = 4-bit field m
// of `shifts`, 0 for the other dimensions): each point's value is identified
// by F, the first sorted position of that value, which replaces its rank in
// R32, and its 16-bit code is F >> s (biased).  F is strictly increasing in
// the value, so compares on the codes are exact except between a point and an
// origin with the same code and a smaller F, which launch_rank_fixups corrects
// after the sweep: there are fewer than 2^s of them, ties or not, since they
// occupy sorted positions [(F_o >> s) << s, F_o).
__global__ void k_rank_shift(uint32_t *__restrict__ R32, const uint32_t *__restrict__ RS, int64_t N, int d,
                             int pw, uint32_t shifts, uint16_t *__restrict__ R16)
{
    const int64_t total = N * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / d;
        const int m = (int)(e - i * d);
        const uint32_t s = (shifts >> (4 * m)) & 15u;
        if (s == 0) continue;  // the dense rank already fits
        const uint32_t f = RS[(size_t)m * (N + 1) + R32[e]];
        R32[e] = f;
        put_rank(R16, i, pw, m, (int64_t)(f >> s));
    }
}

static int64_t tiles_of(int64_t N) { return (N + TILE - 1) / TILE; }
static int64_t stiles_of(int64_t N) { return (N + STILE - 1) / STILE; }

size_t rank16_scratch_bytes(int64_t N, int d)
{
    const int64_t tiles = tiles_of(N);
    if (N <= 65536) {
        const int64_t st = stiles_of(N);
        return (size_t)d * st * STILE * sizeof(uint32_t) + 256;
    }
    size_t a = (size_t)d * tiles * TILE * sizeof(uint64_t);
    size_t s = (size_t)d * N * sizeof(uint64_t);
    size_t c = (size_t)d * ((N + SEG - 1) / SEG) * sizeof(uint32_t);
    size_t r32 = (size_t)N * d * sizeof(uint32_t);          // full ranks
    size_t rs = (size_t)d * (N + 1) * sizeof(uint32_t);     // first sorted position per rank
    size_t pos = (size_t)d * tiles * TILE * sizeof(uint32_t);  // sorted position per tile entry
    return a + s + c + r32 + rs + pos + 256;
}

RankTables rank16_tables(void *scratch, int64_t N, int d)
{
    RankTables t;
    const int64_t tiles = tiles_of(N);
    uint64_t *A = (uint64_t *)scratch;
    t.S = A + (size_t)d * tiles * TILE;
    uint32_t *C = (uint32_t *)(t.S + (size_t)d * N);
    t.R32 = C + (size_t)d * ((N + SEG - 1) / SEG);
    t.RS = t.R32 + (size_t)N * d;
    return t;
}

hipError_t launch_rank16_shift(int64_t N, int d, uint32_t *R, void *scratch, uint32_t shifts, hipStream_t st)
{
    if (N <= 65536 || shifts == 0) return hipErrorInvalidValue;
    const RankTables t = rank16_tables(scratch, N, d);
    const unsigned blocks = (unsigned)std::min<int64_t>((N * d + 255) / 256, 4096);
    hipLaunchKernelGGL(k_rank_shift, dim3(blocks), dim3(256), 0, st, t.R32, t.RS, N, d,
                       point_words(PATH_R16, d), shifts, (uint16_t *)R);
    return hipGetLastError();
}

size_t sort_columns_scratch_bytes(int64_t N, int C)
{
    return (size_t)C * tiles_of(N) * TILE * (sizeof(uint64_t) + sizeof(uint32_t)) +
           (size_t)C * N * sizeof(uint64_t) + 256;
}

hipError_t launch_sort_columns(const float *X, int64_t N, int C, void *scratch, uint64_t **S_out,
                               hipStream_t st)
{
    if (N < 1 || C < 1 || C > 65535 || N > 0x7fffffffLL || ((uintptr_t)scratch & 15)) return hipErrorInvalidValue;
    const int64_t tiles = tiles_of(N);
    uint64_t *A = (uint64_t *)scratch;
    uint64_t *S = A + (size_t)C * tiles * TILE;
    uint32_t *pos = (uint32_t *)(S + (size_t)C * N);
    if (tiles == 1) {  // one tile: the sorted tile is the sorted column
        if (N <= 256)
            hipLaunchKernelGGL((k_rank_pairs<4, 64>), dim3(1, C), dim3(64), 0, st, X, N, C, tiles, A, S, pos);
        else if (N <= 1024)
            hipLaunchKernelGGL((k_rank_pairs<4, 256>), dim3(1, C), dim3(256), 0, st, X, N, C, tiles, A, S, pos);
        else
            hipLaunchKernelGGL((k_rank_pairs<PAIR_KPT, PAIR_THREADS>), dim3(1, C), dim3(PAIR_THREADS), 0, st, X, N, C, tiles, A, S,
                               pos);
        *S_out = S;
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_rank_pairs<PAIR_KPT, PAIR_THREADS>), dim3((unsigned)tiles, C), dim3(PAIR_THREADS), 0, st, X, N, C, tiles,
                       A, (uint64_t *)nullptr, pos);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_place(A, N, C, tiles, pos, S, st);
    *S_out = S;
    return e;
}

hipError_t launch_rank16_pq(const float *P, int64_t n_p, const float *Q, int64_t n_q, int d, uint32_t *R,
                            void *scratch, uint32_t *flags, hipStream_t st)
{
    const int64_t N = n_p + n_q;
    if (N < 1 || N > 65536) return hipErrorInvalidValue;
    const int pw = point_words(PATH_R16, d);
    const int64_t tiles = stiles_of(N);
    uint32_t *Kt = (uint32_t *)scratch;
    hipError_t e;
    hipLaunchKernelGGL(k_rank_sort32, dim3((unsigned)tiles, d), dim3(S32_THREADS), 0, st, P, n_p, Q, N, d,
                       tiles, Kt, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((k_rank_count<RC_KPT, RC_TPS>), dim3((unsigned)(tiles * rc_parts(RC_KPT)), d),
                       dim3(RC_THREADS), 0, st, P, n_p, Q, N, d, pw, tiles, Kt, (uint16_t *)R);
    return hipGetLastError();
}

hipError_t launch_rank16(const float *Z, int64_t N, int d, uint32_t *R, void *scratch, uint32_t *ctl,
                         hipStream_t st)
{
    const int pw = point_words(PATH_R16, d);
    const int64_t tiles = tiles_of(N);
    uint16_t *R16 = (uint16_t *)R;
    hipError_t e;
    if (N <= 65536) return launch_rank16_pq(Z, N, Z, 0, d, R, scratch, nullptr, st);
    if ((uintptr_t)scratch & 15) return hipErrorInvalidValue;  // the tile sort stores 16-byte words
    uint64_t *A = (uint64_t *)scratch;
    uint64_t *S = A + (size_t)d * tiles * TILE;
    uint32_t *C = (uint32_t *)(S + (size_t)d * N);
    const int64_t segs = (N + SEG - 1) / SEG;
    const RankTables tabs = rank16_tables(scratch, N, d);
    uint32_t *pos = tabs.RS + (size_t)d * (N + 1);
    hipLaunchKernelGGL((k_rank_pairs<PAIR_KPT, PAIR_THREADS>), dim3((unsigned)tiles, d), dim3(PAIR_THREADS), 0, st, Z, N, d,
                       tiles, A, (uint64_t *)nullptr, pos);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_place(A, N, d, tiles, pos, S, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_flags, dim3((unsigned)segs, d), dim3(SEG_THREADS), 0, st, S, N, segs, C,
                       ctl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_dense, dim3((unsigned)segs, d), dim3(SEG_THREADS), 0, st, S, N, d, pw,
                       segs, C, R16, ctl, tabs.R32, tabs.RS);
    return hipGetLastError();
}

}  // namespace ddks
