// rdKS, the radial approximation of the statistic (arXiv:2106.13706,
// Sec. 2.2.3, Alg. 2), on gfx950.
//
// Readings: the pooled points are normalised per dimension onto [0, 1]
// (u = (x - lo)/(hi - lo), u = 0 where hi == lo); the corners are the origin
// and the unit points e_m of that space (d + 1 of them); the distance from a
// corner is the squared Euclidean distance in fp32, summed over the
// dimensions in ascending order with every operation rounded on its own (no
// fused multiply-add, so that it is reproducible bit for bit); per corner
// the statistic is the two-sample KS statistic of the two samples' distance
// lists, |c_P(r) n_Q - c_Q(r) n_P| at the largest, over the distinct
// distances r; D is the largest over the corners.
//
// Device work: extents (order-key minima and maxima per dimension), the
// N x (d + 1) distance matrix of the normalised coordinates (formed on the
// fly; one thread per point and corner below 32 dimensions), each
// column sorted as (key, index) pairs, then per corner a segmented scan of
// first-sample labels along the sorted order that scores the end of every
// run of equal distances.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ddks_internal.h"

namespace ddks {

// Scan segments of 1024 sorted positions, 256 threads of four: a column of
// 40000 positions gives 40 blocks per corner (4096-position segments of 1024
// threads took 10.7 us to score at d = 4 against 50 blocks in all).
static constexpr int RD_SEG = 1024;       // sorted positions per scan segment
static constexpr int RD_THREADS = 256;    // four positions per thread

// Order-preserving image of a finite fp32 value (-0 is mapped to +0
// upstream): unsigned comparison of images == fp32 comparison.
__device__ __forceinline__ uint32_t rd_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float rd_from_key(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void k_rd_extent_init(uint32_t *__restrict__ key, int d, unsigned long long *__restrict__ corner_num,
                                 int C)
{
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < d; m += gridDim.x * blockDim.x) {
        key[2 * m] = 0xffffffffu;  // running minimum
        key[2 * m + 1] = 0u;       // running maximum
    }
    // the per-corner maxima that k_rd_score raises
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x) corner_num[c] = 0ull;
}

// Per-dimension extents as order keys: block (chunk, m) reduces its share of
// dimension m's values and folds them in with one atomic pair (at most
// RD_EXTENT_CHUNKS updates per word).
static constexpr int RD_EXTENT_CHUNKS = 32;
__global__ __launch_bounds__(256) void k_rd_extent(const float *__restrict__ Z, int64_t N, int d,
                                                   uint32_t *__restrict__ key)
{
    __shared__ uint32_t slo[4], shi[4];
    const int m = blockIdx.y;
    uint32_t lo = 0xffffffffu, hi = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = rd_key(Z[i * d + m]);
        lo = min(lo, k);
        hi = max(hi, k);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        slo[w] = lo;
        shi[w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 4; ++v) {
            lo = min(lo, slo[v]);
            hi = max(hi, shi[v]);
        }
        atomicMin(&key[2 * m], lo);
        atomicMax(&key[2 * m + 1], hi);
    }
}

// Normalised coordinate u of value x in dimension m: (x - lo) / (hi - lo),
// each operation rounded on its own; 0 in a constant dimension.
__device__ __forceinline__ float rd_u(float x, const uint32_t *__restrict__ lohi, int m)
{
    const float lo = rd_from_key(lohi[2 * m]), hi = rd_from_key(lohi[2 * m + 1]);
    return hi > lo ? __fdiv_rn(__fsub_rn(x, lo), __fsub_rn(hi, lo)) : 0.0f;
}

// Dist[i * C + c] = sum over m ascending of (u_m - [c == m + 1])^2, C = d + 1,
// u_m formed from Z on the fly (a thread per (point, corner); d < 32).
__global__ void k_rd_dist(const float *__restrict__ Z, const uint32_t *__restrict__ lohi, int64_t N, int d,
                          float *__restrict__ Dist)
{
    const int C = d + 1;
    const int64_t total = N * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / C;
        const int c = (int)(e % C);
        const float *z = Z + i * d;
        float acc = 0.0f;
        for (int m = 0; m < d; ++m) {
            const float t = __fsub_rn(rd_u(z[m], lohi, m), c == m + 1 ? 1.0f : 0.0f);
            acc = __fadd_rn(acc, __fmul_rn(t, t));
        }
        Dist[e] = acc;
    }
}

// The same distances for many dimensions: block per point (grid-stride), one
// thread per corner.  Since u - 0 == u exactly, corner c's sum is the
// ascending sum of the rounded squares u_m^2 with the term m = c - 1 replaced
// by the rounded (u_m - 1)^2, so both squares are formed once per point and
// staged in LDS (2 d <= 8192 floats); the operations and their order are
// those of k_rd_dist.
__global__ __launch_bounds__(1024) void k_rd_dist_rows(const float *__restrict__ Z,
                                                       const uint32_t *__restrict__ lohi, int64_t N, int d,
                                                       float *__restrict__ Dist)
{
    extern __shared__ float4 sq4[];  // as floats: sq[m] = u_m^2, sq[d + m] = (u_m - 1)^2
    float *sq = reinterpret_cast<float *>(sq4);
    const int C = d + 1;
    for (int64_t i = blockIdx.x; i < N; i += gridDim.x) {
        __syncthreads();  // the previous point's squares have been used
        for (int m = threadIdx.x; m < d; m += blockDim.x) {
            const float u = rd_u(Z[i * d + m], lohi, m);
            const float t = __fsub_rn(u, 1.0f);
            sq[m] = __fmul_rn(u, u);
            sq[d + m] = __fmul_rn(t, t);
        }
        __syncthreads();
        for (int c = threadIdx.x; c < C; c += blockDim.x) {
            // the same additions in the same order, the squares read four at
            // a time where they are 16-byte aligned
            float acc = 0.0f;
            const int j = c - 1;  // the replaced term (none for the origin corner)
            int m = 0;
#pragma unroll 2
            for (; m + 4 <= j; m += 4) {
                const float4 q = sq4[m >> 2];
                acc = __fadd_rn(__fadd_rn(__fadd_rn(__fadd_rn(acc, q.x), q.y), q.z), q.w);
            }
            for (; m < j; ++m) acc = __fadd_rn(acc, sq[m]);
            if (j >= 0) acc = __fadd_rn(acc, sq[d + j]);
            for (m = j + 1; m < d && (m & 3); ++m) acc = __fadd_rn(acc, sq[m]);
#pragma unroll 2
            for (; m + 4 <= d; m += 4) {
                const float4 q = sq4[m >> 2];
                acc = __fadd_rn(__fadd_rn(__fadd_rn(__fadd_rn(acc, q.x), q.y), q.z), q.w);
            }
            for (; m < d; ++m) acc = __fadd_rn(acc, sq[m]);
            Dist[i * C + c] = acc;
        }
    }
}

// cnt[m * segs + g] = first-sample points among sorted positions of segment g.
__global__ __launch_bounds__(RD_THREADS) void k_rd_seg(const uint64_t *__restrict__ S, int64_t N,
                                                       int64_t segs, int64_t n_p,
                                                       uint32_t *__restrict__ cnt)
{
    __shared__ uint32_t tot;
    const int m = blockIdx.y;
    const int64_t g = blockIdx.x;
    const uint64_t *Sm = S + (size_t)m * N;
    if (threadIdx.x == 0) tot = 0;
    __syncthreads();
    uint32_t c = 0;
    for (int e = threadIdx.x; e < RD_SEG; e += RD_THREADS) {
        const int64_t p = g * RD_SEG + e;
        if (p < N && (int64_t)(uint32_t)Sm[p] < n_p) ++c;
    }
    atomicAdd(&tot, c);
    __syncthreads();
    if (threadIdx.x == 0) cnt[(size_t)m * segs + g] = tot;
}

// Scores every run end of segment g of corner m and folds the maximum into
// corner_num[m].  NT threads of RD_PER positions each: NT = RD_THREADS covers
// a segment; a column of one segment (N <= RD_SEG, cnt unread) may take a
// smaller block that still covers its N positions.
static constexpr int RD_PER = RD_SEG / RD_THREADS;
template <int NT>
__global__ __launch_bounds__(NT) void k_rd_score(const uint64_t *__restrict__ S, int64_t N,
                                                 int64_t segs, int64_t n_p, int64_t n_q,
                                                 const uint32_t *__restrict__ cnt,
                                                 unsigned long long *__restrict__ corner_num)
{
    constexpr int PER = RD_PER;
    constexpr int NW = NT / 64;
    __shared__ uint32_t wsum[NW];
    __shared__ unsigned long long before;
    __shared__ unsigned long long bmax;
    const int m = blockIdx.y;
    const int64_t g = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t *Sm = S + (size_t)m * N;
    if (tid == 0) {
        before = 0ull;
        bmax = 0ull;
    }
    // the thread's PER pairs and the next one (its last run may end there),
    // all loaded up front
    const int64_t p0 = g * RD_SEG + (int64_t)tid * PER;
    uint64_t v[PER + 1];
#pragma unroll
    for (int e = 0; e <= PER; ++e) v[e] = p0 + e < N ? Sm[p0 + e] : ~0ull;
    int64_t b = 0;  // first-sample points of the earlier segments
    for (int64_t h = tid; h < g; h += NT) b += cnt[(size_t)m * segs + h];
    __syncthreads();
    if (b) atomicAdd(&before, (unsigned long long)b);
    uint32_t lab[PER];
    uint32_t c = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        lab[e] = (p0 + e < N && (int64_t)(uint32_t)v[e] < n_p) ? 1u : 0u;
        c += lab[e];
    }
    uint32_t x = c;  // inclusive scan within the wave, then over the waves
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t wb = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) wb += q < w ? wsum[q] : 0u;
    int64_t cp = (int64_t)before + wb + x - c;  // first-sample points before p0
    unsigned long long best = 0ull;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int64_t p = p0 + e;
        if (p >= N) break;
        cp += lab[e];
        const bool run_end = p + 1 == N || (v[e + 1] >> 32) != (v[e] >> 32);
        if (!run_end) continue;
        const int64_t cq = (p + 1) - cp;
        const int64_t sd = cp * n_q - cq * n_p;
        const unsigned long long sc = (unsigned long long)(sd < 0 ? -sd : sd);
        best = sc > best ? sc : best;
    }
    atomicMax(&bmax, best);
    __syncthreads();
    if (tid == 0 && bmax > 0ull) atomicMax(&corner_num[m], bmax);
}

// D = the largest corner numerator; ties go to the lowest corner (one block).
__global__ __launch_bounds__(1024) void k_rd_final(const unsigned long long *__restrict__ corner_num, int C,
                                                   uint32_t *__restrict__ flags, ResultDev *__restrict__ out)
{
    __shared__ unsigned long long sn[16];
    __shared__ int sc[16];
    unsigned long long best = 0ull;
    int bc = 0x7fffffff;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        const unsigned long long v = corner_num[c];
        if (v > best || (v == best && c < bc)) {
            best = v;
            bc = c;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long v = __shfl_xor(best, off, 64);
        const int c = __shfl_xor(bc, off, 64);
        if (v > best || (v == best && c < bc)) {
            best = v;
            bc = c;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sn[w] = best;
        sc[w] = bc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < (int)(blockDim.x >> 6); ++v)
            if (sn[v] > best || (sn[v] == best && sc[v] < bc)) {
                best = sn[v];
                bc = sc[v];
            }
        out->num = best;
        out->origin = bc;
        out->code = 0;
        out->flags = *flags;
        out->ge = 0;
        *flags = 0u;
    }
}

// ---------------------------------------------------------------- host side

static constexpr int RD_ROWS_MIN_D = 32;  // from here on, distances with the row in LDS

static int64_t rd_segs(int64_t N) { return (N + RD_SEG - 1) / RD_SEG; }

size_t rdks_scratch_bytes(int64_t N, int d)
{
    const int C = d + 1;
    size_t b = 0;
    b += (size_t)2 * d * sizeof(uint32_t);      // extents (order keys)
    b += (size_t)N * C * sizeof(float);         // Dist
    b += (size_t)C * rd_segs(N) * sizeof(uint32_t) + 256;
    b += sort_columns_scratch_bytes(N, C);
    return b + 8 * 256;  // each region rounded up to 256 bytes
}

hipError_t launch_rdks(const float *Z, int64_t N, int64_t n_p, int d, void *scratch,
                       unsigned long long *corner_num, uint32_t *flags, ResultDev *out, hipStream_t s)
{
    const int C = d + 1;
    if (N < 1 || d < 1 || C > 65535) return hipErrorInvalidValue;
    char *base = (char *)scratch;
    uint32_t *lohi = (uint32_t *)base;
    base += ((size_t)2 * d * sizeof(uint32_t) + 255) & ~(size_t)255;
    float *Dist = (float *)base;
    base += ((size_t)N * C * sizeof(float) + 255) & ~(size_t)255;
    uint32_t *cnt = (uint32_t *)base;
    const int64_t segs = rd_segs(N);
    base += ((size_t)C * segs * sizeof(uint32_t) + 255) & ~(size_t)255;
    auto grid = [](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); };
    hipLaunchKernelGGL(k_rd_extent_init, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, s, lohi, d, corner_num, C);
    const unsigned chunks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + 1023) / 1024, RD_EXTENT_CHUNKS));
    hipLaunchKernelGGL(k_rd_extent, dim3(chunks, (unsigned)d), dim3(256), 0, s, Z, N, d, lohi);
    if (d >= RD_ROWS_MIN_D)
        hipLaunchKernelGGL(k_rd_dist_rows, dim3((unsigned)std::min<int64_t>(N, 4096)), dim3(1024),
                           (size_t)2 * d * sizeof(float), s, Z, lohi, N, d, Dist);
    else
        hipLaunchKernelGGL(k_rd_dist, dim3(grid(N * C)), dim3(256), 0, s, Z, lohi, N, d, Dist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t *S = nullptr;
    if ((e = launch_sort_columns(Dist, N, C, base, &S, s)) != hipSuccess) return e;
    if (segs > 1) {
        hipLaunchKernelGGL(k_rd_seg, dim3((unsigned)segs, C), dim3(RD_THREADS), 0, s, S, N, segs, n_p, cnt);
        hipLaunchKernelGGL(k_rd_score<RD_THREADS>, dim3((unsigned)segs, C), dim3(RD_THREADS), 0, s, S, N, segs,
                           n_p, N - n_p, cnt, corner_num);
    } else if (N <= 64 * RD_PER) {  // one segment: no counts of earlier segments to read
        hipLaunchKernelGGL(k_rd_score<64>, dim3(1, C), dim3(64), 0, s, S, N, segs, n_p, N - n_p, cnt, corner_num);
    } else {
        hipLaunchKernelGGL(k_rd_score<RD_THREADS>, dim3(1, C), dim3(RD_THREADS), 0, s, S, N, segs, n_p, N - n_p,
                           cnt, corner_num);
    }
    hipLaunchKernelGGL(k_rd_final, dim3(1), dim3(1024), 0, s, corner_num, C, flags, out);
    return hipGetLastError();
}

}  // namespace ddks
