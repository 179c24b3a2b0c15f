// Rank encoding for the 16-bit compare path.
//
// The sweep only ever asks whether x_m >= o_m for points and origins drawn
// from the same pooled set, so any map of each dimension's values onto
// integers that is strictly increasing on the values present gives exactly
// the same orthant codes.  With at most 65536 distinct values per dimension
// the ranks fit int16 (biased by -32768) and one saturating v_pk_sub_i16
// compares two dimensions.
//
// Per dimension (grid.y = dimension):
//   1. k_rank_tiles  sorts tiles of TILE (key, index) pairs in LDS (bitonic);
//                    key = an order-preserving uint32 image of the fp32 value.
//   2a. N <= 65536:  k_rank_min     each value's rank = number of pooled values
//                                   strictly below it (binary search in every
//                                   sorted tile); fits 16 bits since N <= 65536.
//   2b. N > 65536:   k_rank_place   places each pair at its sorted position,
//                    k_rank_flags   counts first occurrences per segment,
//                    k_rank_dense   dense rank = number of distinct values
//                                   below, from the segment counts and a block
//                                   scan; records the distinct-value count.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ddks_internal.h"

namespace ddks {

static constexpr int TILE = 4096;      // pairs per sorted tile (32 KB of LDS)
static constexpr int TILE_THREADS = 1024;
static constexpr int SEG = 4096;       // positions per flag segment
static constexpr int SEG_THREADS = 1024;

// Order-preserving image of a finite fp32 value (+0 and -0 are both mapped
// to +0 upstream): unsigned comparison of images == fp32 comparison.
__device__ __forceinline__ uint32_t order_key(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(TILE_THREADS) void k_rank_tiles(const float *__restrict__ Z, int64_t N,
                                                             int d, int64_t tiles,
                                                             uint64_t *__restrict__ A)
{
    __shared__ uint64_t s[TILE];
    const int m = blockIdx.y;
    const int64_t t = blockIdx.x;
    for (int e = threadIdx.x; e < TILE; e += TILE_THREADS) {
        int64_t i = t * TILE + e;
        s[e] = i < N ? ((uint64_t)order_key(Z[i * d + m]) << 32) | (uint64_t)i : ~0ull;
    }
    __syncthreads();
    for (int k = 2; k <= TILE; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = threadIdx.x; p < TILE / 2; p += TILE_THREADS) {
                int i = 2 * j * (p / j) + (p % j);
                int l = i + j;
                bool up = (i & k) == 0;
                uint64_t a = s[i], b = s[l];
                if ((a > b) == up) {
                    s[i] = b;
                    s[l] = a;
                }
            }
            __syncthreads();
        }
    }
    uint64_t *out = A + (size_t)m * tiles * TILE + t * TILE;
    for (int e = threadIdx.x; e < TILE; e += TILE_THREADS) out[e] = s[e];
}

// Number of entries of the sorted tile below v.
__device__ __forceinline__ int lower_bound_tile(const uint64_t *__restrict__ tile, uint64_t v)
{
    int lo = 0, n = TILE;
    while (n > 0) {
        int half = n >> 1;
        if (tile[lo + half] < v) {
            lo += half + 1;
            n -= half + 1;
        } else {
            n = half;
        }
    }
    return lo;
}

// Writes the biased 16-bit rank of dimension m of point i.
__device__ __forceinline__ void put_rank(uint16_t *R16, int64_t i, int pw, int m, int64_t rank)
{
    R16[(i * pw) * 2 + m] = (uint16_t)(uint32_t)(rank - 32768);
}

__global__ void k_rank_min(const uint64_t *__restrict__ A, int64_t N, int d, int pw, int64_t tiles,
                           uint16_t *__restrict__ R16)
{
    const int m = blockIdx.y;
    const uint64_t *Am = A + (size_t)m * tiles * TILE;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tiles * TILE;
         q += (int64_t)gridDim.x * blockDim.x) {
        uint64_t item = Am[q];
        if (item == ~0ull) continue;
        const int64_t i = (int64_t)(uint32_t)item;
        const uint64_t probe = item & 0xffffffff00000000ull;  // (key, index 0)
        int64_t rank = 0;
        for (int64_t t = 0; t < tiles; ++t) rank += lower_bound_tile(Am + t * TILE, probe);
        put_rank(R16, i, pw, m, rank);
        if (m == 0)
            for (int mm = d; mm < 2 * pw; ++mm) R16[(i * pw) * 2 + mm] = 0;
    }
}

__global__ void k_rank_place(const uint64_t *__restrict__ A, int64_t N, int64_t tiles,
                             uint64_t *__restrict__ S)
{
    const int m = blockIdx.y;
    const uint64_t *Am = A + (size_t)m * tiles * TILE;
    uint64_t *Sm = S + (size_t)m * N;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tiles * TILE;
         q += (int64_t)gridDim.x * blockDim.x) {
        uint64_t item = Am[q];
        if (item == ~0ull) continue;
        int64_t pos = 0;
        for (int64_t t = 0; t < tiles; ++t) pos += lower_bound_tile(Am + t * TILE, item);
        Sm[pos] = item;
    }
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
                                                            uint32_t *__restrict__ distinct_max)
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
        if (g == segs - 1) atomicMax(distinct_max, b + C[(size_t)m * segs + g]);
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
        if (m == 0)
            for (int mm = d; mm < 2 * pw; ++mm) R16[(i * pw) * 2 + mm] = 0;
    }
}

static int64_t tiles_of(int64_t N) { return (N + TILE - 1) / TILE; }

size_t rank16_scratch_bytes(int64_t N, int d)
{
    const int64_t tiles = tiles_of(N);
    size_t a = (size_t)d * tiles * TILE * sizeof(uint64_t);
    size_t s = N > 65536 ? (size_t)d * N * sizeof(uint64_t) : 0;
    size_t c = N > 65536 ? (size_t)d * ((N + SEG - 1) / SEG) * sizeof(uint32_t) : 0;
    return a + s + c + 256;
}

hipError_t launch_rank16(const float *Z, int64_t N, int d, uint32_t *R, void *scratch,
                         uint32_t *distinct_max, hipStream_t st)
{
    const int pw = point_words(PATH_R16, d);
    const int64_t tiles = tiles_of(N);
    uint64_t *A = (uint64_t *)scratch;
    uint16_t *R16 = (uint16_t *)R;
    hipLaunchKernelGGL(k_rank_tiles, dim3((unsigned)tiles, d), dim3(TILE_THREADS), 0, st, Z, N, d,
                       tiles, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t items = tiles * TILE;
    unsigned blocks = (unsigned)std::min<int64_t>((items + 255) / 256, 4096);
    if (N <= 65536) {
        hipLaunchKernelGGL(k_rank_min, dim3(blocks, d), dim3(256), 0, st, A, N, d, pw, tiles, R16);
        return hipGetLastError();
    }
    uint64_t *S = A + (size_t)d * tiles * TILE;
    uint32_t *C = (uint32_t *)(S + (size_t)d * N);
    const int64_t segs = (N + SEG - 1) / SEG;
    hipLaunchKernelGGL(k_rank_place, dim3(blocks, d), dim3(256), 0, st, A, N, tiles, S);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_flags, dim3((unsigned)segs, d), dim3(SEG_THREADS), 0, st, S, N, segs, C,
                       distinct_max);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_dense, dim3((unsigned)segs, d), dim3(SEG_THREADS), 0, st, S, N, d, pw,
                       segs, C, R16, distinct_max);
    return hipGetLastError();
}

}  // namespace ddks
