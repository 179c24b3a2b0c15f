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
// Device work: extents (one block per dimension), normalised coordinates,
// the N x (d + 1) distance matrix (one thread per point and corner), each
// column sorted as (key, index) pairs, then per corner a segmented scan of
// first-sample labels along the sorted order that scores the end of every
// run of equal distances.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ddks_internal.h"

namespace ddks {

static constexpr int RD_SEG = 4096;       // sorted positions per scan segment
static constexpr int RD_THREADS = 1024;   // four positions per thread

// Per-dimension minimum and maximum (block m, reduction over the points).
__global__ __launch_bounds__(256) void k_rd_extent(const float *__restrict__ Z, int64_t N, int d,
                                                   float *__restrict__ lohi)
{
    __shared__ float slo[4], shi[4];
    const int m = blockIdx.x;
    float lo = INFINITY, hi = -INFINITY;
    for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
        const float v = Z[i * d + m];
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, off, 64));
        hi = fmaxf(hi, __shfl_xor(hi, off, 64));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        slo[w] = lo;
        shi[w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 4; ++v) {
            lo = fminf(lo, slo[v]);
            hi = fmaxf(hi, shi[v]);
        }
        lohi[2 * m] = lo;
        lohi[2 * m + 1] = hi;
    }
}

// Normalised coordinates u (N x d), each value (x - lo) / (hi - lo) rounded once
// per operation.
__global__ void k_rd_norm(const float *__restrict__ Z, int64_t N, int d, const float *__restrict__ lohi,
                          float *__restrict__ U)
{
    const int64_t total = N * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(e % d);
        const float lo = lohi[2 * m], hi = lohi[2 * m + 1];
        U[e] = hi > lo ? __fdiv_rn(__fsub_rn(Z[e], lo), __fsub_rn(hi, lo)) : 0.0f;
    }
}

// Dist[i * C + c] = sum over m ascending of (u_m - [c == m + 1])^2, C = d + 1.
__global__ void k_rd_dist(const float *__restrict__ U, int64_t N, int d, float *__restrict__ Dist)
{
    const int C = d + 1;
    const int64_t total = N * C;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / C;
        const int c = (int)(e % C);
        const float *u = U + i * d;
        float acc = 0.0f;
        for (int m = 0; m < d; ++m) {
            const float t = __fsub_rn(u[m], c == m + 1 ? 1.0f : 0.0f);
            acc = __fadd_rn(acc, __fmul_rn(t, t));
        }
        Dist[e] = acc;
    }
}

__global__ void k_rd_zero(unsigned long long *__restrict__ v, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = 0ull;
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
// corner_num[m].
__global__ __launch_bounds__(RD_THREADS) void k_rd_score(const uint64_t *__restrict__ S, int64_t N,
                                                         int64_t segs, int64_t n_p, int64_t n_q,
                                                         const uint32_t *__restrict__ cnt,
                                                         unsigned long long *__restrict__ corner_num)
{
    constexpr int PER = RD_SEG / RD_THREADS;
    __shared__ uint32_t scan[RD_THREADS];
    __shared__ int64_t before;
    __shared__ unsigned long long bmax;
    const int m = blockIdx.y;
    const int64_t g = blockIdx.x;
    const uint64_t *Sm = S + (size_t)m * N;
    if (threadIdx.x == 0) {
        int64_t b = 0;
        for (int64_t h = 0; h < g; ++h) b += cnt[(size_t)m * segs + h];
        before = b;
        bmax = 0ull;
    }
    const int64_t p0 = g * RD_SEG + (int64_t)threadIdx.x * PER;
    uint32_t lab[PER];
    uint32_t c = 0;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int64_t p = p0 + e;
        lab[e] = (p < N && (int64_t)(uint32_t)Sm[p] < n_p) ? 1u : 0u;
        c += lab[e];
    }
    scan[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < RD_THREADS; off <<= 1) {  // inclusive block scan
        const uint32_t v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0u;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t cp = before + scan[threadIdx.x] - c;  // first-sample points before p0
    unsigned long long best = 0ull;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int64_t p = p0 + e;
        if (p >= N) break;
        cp += lab[e];
        const bool run_end = p + 1 == N || (Sm[p + 1] >> 32) != (Sm[p] >> 32);
        if (!run_end) continue;
        const int64_t cq = (p + 1) - cp;
        const int64_t sd = cp * n_q - cq * n_p;
        const unsigned long long sc = (unsigned long long)(sd < 0 ? -sd : sd);
        best = sc > best ? sc : best;
    }
    atomicMax(&bmax, best);
    __syncthreads();
    if (threadIdx.x == 0 && bmax > 0ull) atomicMax(&corner_num[m], bmax);
}

__global__ void k_rd_final(const unsigned long long *__restrict__ corner_num, int C,
                           uint32_t *__restrict__ flags, ResultDev *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long best = corner_num[0];
    int bc = 0;
    for (int c = 1; c < C; ++c)
        if (corner_num[c] > best) {
            best = corner_num[c];
            bc = c;
        }
    out->num = best;
    out->origin = bc;
    out->code = 0;
    out->flags = *flags;
    out->ge = 0;
    *flags = 0u;
}

// ---------------------------------------------------------------- host side

static int64_t rd_segs(int64_t N) { return (N + RD_SEG - 1) / RD_SEG; }

size_t rdks_scratch_bytes(int64_t N, int d)
{
    const int C = d + 1;
    size_t b = 0;
    b += (size_t)2 * d * sizeof(float);         // extents
    b += (size_t)N * d * sizeof(float);         // U
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
    float *lohi = (float *)base;
    base += ((size_t)2 * d * sizeof(float) + 255) & ~(size_t)255;
    float *U = (float *)base;
    base += ((size_t)N * d * sizeof(float) + 255) & ~(size_t)255;
    float *Dist = (float *)base;
    base += ((size_t)N * C * sizeof(float) + 255) & ~(size_t)255;
    uint32_t *cnt = (uint32_t *)base;
    const int64_t segs = rd_segs(N);
    base += ((size_t)C * segs * sizeof(uint32_t) + 255) & ~(size_t)255;
    auto grid = [](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); };
    hipLaunchKernelGGL(k_rd_extent, dim3((unsigned)d), dim3(256), 0, s, Z, N, d, lohi);
    hipLaunchKernelGGL(k_rd_norm, dim3(grid(N * d)), dim3(256), 0, s, Z, N, d, lohi, U);
    hipLaunchKernelGGL(k_rd_dist, dim3(grid(N * C)), dim3(256), 0, s, U, N, d, Dist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t *S = nullptr;
    if ((e = launch_sort_columns(Dist, N, C, base, &S, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rd_zero, dim3(grid(C)), dim3(256), 0, s, corner_num, C);
    hipLaunchKernelGGL(k_rd_seg, dim3((unsigned)segs, C), dim3(RD_THREADS), 0, s, S, N, segs, n_p, cnt);
    hipLaunchKernelGGL(k_rd_score, dim3((unsigned)segs, C), dim3(RD_THREADS), 0, s, S, N, segs, n_p,
                       N - n_p, cnt, corner_num);
    hipLaunchKernelGGL(k_rd_final, dim3(1), dim3(64), 0, s, corner_num, C, flags, out);
    return hipGetLastError();
}

}  // namespace ddks
