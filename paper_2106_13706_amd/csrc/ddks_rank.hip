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
//   2. k_rank_count   block (t, t') stages sorted tile t' in LDS and counts,
//                     for every point of tile t, the values of t' strictly
//                     below its own (binary search);
//   3. k_rank_sum     the rank of a point is the sum of its counts over all
//                     tiles: the number of pooled values below it, which fits
//                     16 bits since N <= 65536.
// N > 65536:
//   1. k_rank_tiles   sorts tiles of (key, index) pairs (bitonic, in
//                     registers, wave shuffles and LDS);
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

// Tiles of the N <= 65536 path.  2048-key tiles measured slower at 40000
// points x 4 dimensions: the sort took 8.9 instead of 14.4 us, but the
// counts (13.5 vs 9.1 us) and their sum (7.2 vs 4.6 us) grew more.
static constexpr int STILE = 4096;
static constexpr int S32_THREADS = STILE / 4;  // four keys per thread
static_assert(STILE == 4 * S32_THREADS, "k_rank_sort32 holds four keys per thread");
static constexpr int LOG_STILE = 12;
static_assert((1 << LOG_STILE) == STILE, "tile size");

// Sorts tile blockIdx.x of dimension blockIdx.y: K[m][t][0..STILE) = the order
// keys of points t*STILE .. t*STILE+STILE-1, ascending (0xffffffff past N).
// Bitonic network, fully unrolled: thread tid holds elements e = 4*tid + r;
// partners at distance j < 4 are in the same thread, j < 256 in the same wave
// (shuffles), j >= 256 in another wave (double-buffered LDS, one barrier per
// stage).  For j >= 4 the direction of a thread's four compare-exchanges is
// the same (it depends on bits of e above bit 1 only).
// Values are read from P (points 0 .. n_p - 1) then Q; flags (nullable): bit 0
// is set if a value is NaN or infinite.
__global__ __launch_bounds__(S32_THREADS) void k_rank_sort32(const float *__restrict__ P, int64_t n_p,
                                                             const float *__restrict__ Q, int64_t N,
                                                             int d, int64_t tiles,
                                                             uint32_t *__restrict__ K,
                                                             uint32_t *__restrict__ flags)
{
    __shared__ uint4 buf[2][S32_THREADS];
    const int m = blockIdx.y;
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x;
    const int e0 = 4 * tid;
    uint32_t v[4];
    bool bad = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = t * STILE + e0 + r;
        const float x = i < N ? point_value(P, n_p, Q, i, d, m) : 0.0f;
        bad |= !isfinite(x);
        v[r] = i < N ? order_key(x) : 0xffffffffu;
    }
    if (flags && __any(bad) && (tid & 63) == 0) atomicOr(flags, 1u);
    int cur = 0;
#pragma unroll
    for (int lk = 1; lk <= LOG_STILE; ++lk) {
        const int k = 1 << lk;
#pragma unroll
        for (int lj = lk - 1; lj >= 0; --lj) {
            const int j = 1 << lj;
            if (j >= 4) {
                const bool keep_min = ((e0 & j) == 0) == ((e0 & k) == 0);
                uint32_t pv[4];
                if (j >= 256) {
                    buf[cur][tid] = make_uint4(v[0], v[1], v[2], v[3]);
                    __syncthreads();
                    const uint4 p = buf[cur][tid ^ (j >> 2)];
                    pv[0] = p.x;
                    pv[1] = p.y;
                    pv[2] = p.z;
                    pv[3] = p.w;
                    cur ^= 1;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) pv[r] = __shfl_xor(v[r], j >> 2, 64);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = keep_min ? min(v[r], pv[r]) : max(v[r], pv[r]);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r & j) continue;
                    const bool up = (((e0 + r) & k) == 0);
                    const uint32_t lo = min(v[r], v[r | j]), hi = max(v[r], v[r | j]);
                    v[r] = up ? lo : hi;
                    v[r | j] = up ? hi : lo;
                }
            }
        }
    }
    uint4 *out = reinterpret_cast<uint4 *>(K + ((size_t)m * tiles + t) * STILE);
    out[tid] = make_uint4(v[0], v[1], v[2], v[3]);
}

// The sorted tile in LDS is skewed by one word every 64 entries: the probes
// of one step of the binary search sit at multiples of STILE/2^k minus one,
// which without the skew all fall in the same LDS bank.
__device__ __forceinline__ int skew(int e) { return e + (e >> 6); }

// Number of entries of the sorted, skewed LDS tile below key (branchless; 0..STILE).
__device__ __forceinline__ int count_below(const uint32_t *tile, uint32_t key)
{
    int p = 0;
#pragma unroll
    for (int step = STILE / 2; step >= 1; step >>= 1)
        if (tile[skew(p + step - 1)] < key) p += step;
    return p + (tile[skew(p)] < key ? 1 : 0);
}

// Writes the biased 16-bit rank of dimension m of point i.
__device__ __forceinline__ void put_rank(uint16_t *R16, int64_t i, int pw, int m, int64_t rank)
{
    R16[(i * pw) * 2 + m] = (uint16_t)(uint32_t)(rank - 32768);
}

// Block (t, u, m) with u = blockIdx.z: part[u][m][i] = number of values of
// sorted tile u below point i's value, for the points i of tile t.
__global__ __launch_bounds__(S32_THREADS) void k_rank_count(const float *__restrict__ P, int64_t n_p,
                                                            const float *__restrict__ Q, int64_t N,
                                                            int d, int64_t tiles,
                                                            const uint32_t *__restrict__ K,
                                                            uint16_t *__restrict__ part)
{
    __shared__ uint32_t tile[STILE + STILE / 64 + 1];
    const int m = blockIdx.y;
    const int64_t t = blockIdx.x, u = blockIdx.z;
    const int tid = threadIdx.x;
    const uint4 *src = reinterpret_cast<const uint4 *>(K + ((size_t)m * tiles + u) * STILE);
    {
        const uint4 v = src[tid];  // entries 4 tid .. 4 tid + 3, all in one 64-entry row
        const int e = skew(4 * tid);
        tile[e] = v.x;
        tile[e + 1] = v.y;
        tile[e + 2] = v.z;
        tile[e + 3] = v.w;
    }
    uint32_t key[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = t * STILE + tid + r * S32_THREADS;
        key[r] = i < N ? order_key(point_value(P, n_p, Q, i, d, m)) : 0u;
    }
    __syncthreads();
    uint16_t *pu = part + ((size_t)u * d + m) * tiles * STILE + t * STILE;
#pragma unroll
    for (int r = 0; r < 4; ++r) pu[tid + r * S32_THREADS] = (uint16_t)count_below(tile, key[r]);
}

// The rank of point i in dimension m (values below it over all tiles), from
// the partial counts; also zeroes the padding dimensions of each point.
__global__ void k_rank_sum(const uint16_t *__restrict__ part, int64_t N, int d, int pw,
                           int64_t tiles, uint16_t *__restrict__ R16)
{
    const int m = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t rank = 0;
        for (int64_t u = 0; u < tiles; ++u) rank += part[((size_t)u * d + m) * tiles * STILE + i];
        put_rank(R16, i, pw, m, rank);
        if (m == 0)
            for (int mm = d; mm < 2 * pw; ++mm) R16[(i * pw) * 2 + mm] = 0;
    }
}

// ------------------------------------------------------------ N > 65536

// Sorts (order key << 32 | index) pairs of column m = blockIdx.y, tile t =
// blockIdx.x, T = 256, 1024 or 4096 pairs per tile (~0 past N).  The same
// fully unrolled bitonic network as k_rank_sort32 on 64-bit pairs: a thread
// holds four pairs, partners within a wave go through shuffles and only the
// stages across waves (T > 256) through double-buffered LDS.  Single-tile
// sorts (T >= N) write the N sorted pairs straight to S + m * N; otherwise
// the tile goes to A + (m * tiles + t) * T.
struct Pair4 {
    uint64_t v[4];
};

// S != nullptr: one tile holds the whole column, written sorted to S.
// Otherwise the sorted tile goes to A, and pos (the sorted positions that
// k_rank_place_count accumulates) is cleared at the same entries.
template <int T>
__global__ __launch_bounds__(T / 4) void k_rank_tiles(const float *__restrict__ Z, int64_t N, int d,
                                                      int64_t tiles, uint64_t *__restrict__ A,
                                                      uint64_t *__restrict__ S, uint32_t *__restrict__ pos)
{
    constexpr int THREADS = T / 4;
    constexpr int LOG_T = T == 256 ? 8 : (T == 1024 ? 10 : 12);
    static_assert(T == 256 || T == 1024 || T == 4096, "tile sizes");
    __shared__ Pair4 buf[2][T > 256 ? THREADS : 1];
    const int m = blockIdx.y;
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x;
    const int e0 = 4 * tid;
    uint64_t v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = t * T + e0 + r;
        v[r] = i < N ? ((uint64_t)order_key(Z[i * d + m]) << 32) | (uint64_t)i : ~0ull;
    }
    int cur = 0;
#pragma unroll
    for (int lk = 1; lk <= LOG_T; ++lk) {
        const int k = 1 << lk;
#pragma unroll
        for (int lj = lk - 1; lj >= 0; --lj) {
            const int j = 1 << lj;
            if (j >= 4) {
                const bool keep_min = ((e0 & j) == 0) == ((e0 & k) == 0);
                uint64_t pv[4];
                if (j >= 256) {
                    if constexpr (T > 256) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) buf[cur][tid].v[r] = v[r];
                        __syncthreads();
#pragma unroll
                        for (int r = 0; r < 4; ++r) pv[r] = buf[cur][tid ^ (j >> 2)].v[r];
                        cur ^= 1;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) pv[r] = __shfl_xor(v[r], j >> 2, 64);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = keep_min ? min(v[r], pv[r]) : max(v[r], pv[r]);
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (r & j) continue;
                    const bool up = (((e0 + r) & k) == 0);
                    const uint64_t lo = min(v[r], v[r | j]), hi = max(v[r], v[r | j]);
                    v[r] = up ? lo : hi;
                    v[r | j] = up ? hi : lo;
                }
            }
        }
    }
    if (S) {
        uint64_t *out = S + (size_t)m * N;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (e0 + r < N) out[e0 + r] = v[r];
    } else {
        const size_t base = ((size_t)m * tiles + t) * T;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            A[base + e0 + r] = v[r];
            pos[base + e0 + r] = 0u;
        }
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
        size_t k = (size_t)d * st * STILE * sizeof(uint32_t);
        size_t part = (size_t)st * d * st * STILE * sizeof(uint16_t);
        return k + part + 256;
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
    if (N < 1 || C < 1 || C > 65535 || N > 0x7fffffffLL) return hipErrorInvalidValue;
    const int64_t tiles = tiles_of(N);
    uint64_t *A = (uint64_t *)scratch;
    uint64_t *S = A + (size_t)C * tiles * TILE;
    uint32_t *pos = (uint32_t *)(S + (size_t)C * N);
    if (tiles == 1) {  // one tile: the sorted tile is the sorted column
        if (N <= 256)
            hipLaunchKernelGGL(k_rank_tiles<256>, dim3(1, C), dim3(64), 0, st, X, N, C, tiles, A, S, pos);
        else if (N <= 1024)
            hipLaunchKernelGGL(k_rank_tiles<1024>, dim3(1, C), dim3(256), 0, st, X, N, C, tiles, A, S, pos);
        else
            hipLaunchKernelGGL(k_rank_tiles<TILE>, dim3(1, C), dim3(TILE / 4), 0, st, X, N, C, tiles, A, S,
                               pos);
        *S_out = S;
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_rank_tiles<TILE>, dim3((unsigned)tiles, C), dim3(TILE / 4), 0, st, X, N, C, tiles,
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
    uint16_t *part = (uint16_t *)(Kt + (size_t)d * tiles * STILE);
    hipError_t e;
    hipLaunchKernelGGL(k_rank_sort32, dim3((unsigned)tiles, d), dim3(S32_THREADS), 0, st, P, n_p, Q, N, d,
                       tiles, Kt, flags);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_count, dim3((unsigned)tiles, d, (unsigned)tiles), dim3(S32_THREADS), 0, st, P,
                       n_p, Q, N, d, tiles, Kt, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned sblocks = (unsigned)std::min<int64_t>((N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_rank_sum, dim3(sblocks, d), dim3(256), 0, st, part, N, d, pw, tiles, (uint16_t *)R);
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
    uint64_t *A = (uint64_t *)scratch;
    uint64_t *S = A + (size_t)d * tiles * TILE;
    uint32_t *C = (uint32_t *)(S + (size_t)d * N);
    const int64_t segs = (N + SEG - 1) / SEG;
    const RankTables tabs = rank16_tables(scratch, N, d);
    uint32_t *pos = tabs.RS + (size_t)d * (N + 1);
    hipLaunchKernelGGL(k_rank_tiles<TILE>, dim3((unsigned)tiles, d), dim3(TILE / 4), 0, st, Z, N, d,
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
