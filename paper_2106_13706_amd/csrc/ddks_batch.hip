// gfx950 kernels for the permutation test (Sec. 3 and Sec. 4.2 of
// arXiv:2106.13706): the ddKS statistic of B relabellings of one pooled
// sample.
//
// A point's orthant relative to an origin does not depend on the labels, so
// each (origin, point) code is computed once and applied to PB relabellings
// at a time: a wave holds 64 origins and, for every bin, one 16-bit counter
// of first-sample points per relabelling, four relabellings per 64-bit LDS
// word (ds_add_u64 of a per-point increment whose four 16-bit fields are
// the point's label bits).  The second sample's count follows from the
// label-free total: c_Q = c_all - c_P, with c_all taken from the counts of
// the observed split.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>

#include <algorithm>

#include "ddks_device.h"

namespace ddks {

typedef __attribute__((address_space(3))) uint64_t lds_u64;

__device__ __forceinline__ void lds_add64(uint32_t byte_addr, uint64_t v)
{
    __hip_atomic_fetch_add((lds_u64 *)(uintptr_t)byte_addr, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Per-point increments: inc[(q * n + x) * NS + s] packs the label bits of
// point x for relabellings q*PB + 4s + t, t = 0..3, in 16-bit field t.
__global__ void k_perm_increments(const uint32_t *__restrict__ labels, int64_t n, int64_t words,
                                  int B, int PB, int64_t groups_q, uint64_t *__restrict__ inc)
{
    const int NS = PB / 4;
    const int64_t total = groups_q * n * NS;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e % NS;
        const int64_t x = (e / NS) % n;
        const int64_t q = e / (NS * n);
        uint64_t v = 0;
        for (int t = 0; t < 4; ++t) {
            int64_t b = q * PB + 4 * s + t;
            if (b < B) {
                uint64_t bit = (labels[b * words + x / 32] >> (x % 32)) & 1u;
                v |= bit << (16 * t);
            }
        }
        inc[e] = v;
    }
}

// Flags bit 1 of *flags when a label row does not hold exactly n_p set bits
// among its first n bits, or sets a bit at or beyond n.
__global__ __launch_bounds__(256) void k_perm_check_labels(const uint32_t *__restrict__ labels,
                                                          int64_t n, int64_t words, int64_t n_p,
                                                          uint32_t *__restrict__ flags)
{
    __shared__ uint32_t tot;
    __shared__ uint32_t stray;
    const int64_t b = blockIdx.x;
    if (threadIdx.x == 0) {
        tot = 0;
        stray = 0;
    }
    __syncthreads();
    uint32_t c = 0, bad = 0;
    for (int64_t w = threadIdx.x; w < words; w += blockDim.x) {
        uint32_t v = labels[b * words + w];
        if (w == words - 1 && (n % 32) != 0) {
            uint32_t keep = (1u << (n % 32)) - 1u;
            bad |= v & ~keep;
            v &= keep;
        }
        c += __builtin_popcount(v);
    }
    atomicAdd(&tot, c);
    if (bad) atomicOr(&stray, 1u);
    __syncthreads();
    if (threadIdx.x == 0 && (tot != (uint32_t)n_p || stray)) atomicOr(flags, 2u);
}

__global__ void k_zero_u64(uint64_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int D, int PATH, int PB, int W>
__global__ __launch_bounds__(W * 64) void k_perm(const void *__restrict__ Zv, int64_t N, int64_t n_p,
                                                 int64_t n_q, const uint64_t *__restrict__ inc, int B,
                                                 const uint32_t *__restrict__ obs_counts,
                                                 unsigned long long *__restrict__ nums)
{
    typedef typename Layout<PATH, D>::T T;
    constexpr int BINS = Geo<D>::BINS;
    constexpr int NS = PB / 4;                    // 64-bit words (4 relabellings) per bin
    constexpr int PW = Layout<PATH, D>::PW;
    constexpr int U = 4;                          // points per unrolled block
    constexpr int NP = Geo<D>::NPERM;
    constexpr uint32_t SLOT = BINS * 64 * 8;      // bytes of one word-slot over all bins
    extern __shared__ uint64_t smem64[];
    const T *__restrict__ Z = static_cast<const T *>(Zv);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t group = blockIdx.x;
    const int64_t q = blockIdx.y;

    // The W waves share the 64 origins and the counters (each counts points of
    // a first sample, at most n_p <= 65535) and split the points.
    for (int i = threadIdx.x; i < NS * BINS * 64; i += W * 64) smem64[i] = 0;
    const int64_t k = group * 64 + lane;
    Origin<PATH, D> org;
    org.load(Z, k < N ? k : N - 1);
    __syncthreads();
    const int64_t per = (N + W - 1) / W;
    int64_t i0 = (int64_t)w * per, i1 = i0 + per;
    i0 = i0 < N ? i0 : N;
    i1 = i1 < N ? i1 : N;
    i0 = __builtin_amdgcn_readfirstlane((int)i0);
    i1 = __builtin_amdgcn_readfirstlane((int)i1);

    const uint32_t base = (uint32_t)(uintptr_t)(lds_u64 *)(smem64 + Geo<D>::KOFF * 64 + lane);
    const uint32_t w0 = dot_wts(D, 0), w1 = dot_wts(D, 1);
    const uint64_t *__restrict__ incq = inc + q * N * NS;
    int64_t i = i0;
    for (; i + U <= i1; i += U) {
        T buf[U * PW];
        uint64_t iv[U * NS];
#pragma unroll
        for (int e = 0; e < U * PW; ++e) buf[e] = Z[i * PW + e];
#pragma unroll
        for (int e = 0; e < U * NS; ++e) iv[e] = incq[i * NS + e];
        uint32_t R[2][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint32_t r[Geo<D>::NREG];
            signs<PATH, D>(buf + u * PW, org, r);
            R[0][u] = group_bytes<D>(r, 0);
            R[1][u] = NP > 1 ? group_bytes<D>(r, 1) : 0u;
        }
        uint32_t a[4];
        addr4<NP, 9>(R, base, a, w0, w1);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int s = 0; s < NS; ++s) lds_add64(a[u] + s * SLOT, iv[u * NS + s]);
    }
    for (; i < i1; ++i) {
        T buf[PW];
#pragma unroll
        for (int e = 0; e < PW; ++e) buf[e] = Z[i * PW + e];
        uint32_t r[Geo<D>::NREG];
        signs<PATH, D>(buf, org, r);
        uint32_t R0 = group_bytes<D>(r, 0);
        uint32_t R1 = NP > 1 ? group_bytes<D>(r, 1) : 0u;
        uint32_t a = addr1<NP, 9>(R0, R1, base, w0, w1);
#pragma unroll
        for (int s = 0; s < NS; ++s) lds_add64(a + s * SLOT, incq[i * NS + s]);
    }
    __syncthreads();

    // Score every relabelling of this group for the lane's origin.
    const bool valid = k < N;
    uint64_t best[PB];
#pragma unroll
    for (int t = 0; t < PB; ++t) best[t] = 0;
    for (int j = w; j < BINS; j += W) {  // this wave's share of the bins
        const int code = j ^ Geo<D>::FLIP;
        uint32_t call = 0;
        if (valid) {
            const uint2 oc = *reinterpret_cast<const uint2 *>(obs_counts + ((size_t)k * BINS + code) * 2);
            call = oc.x + oc.y;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint64_t wv = smem64[(s * BINS + j) * 64 + lane];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t cp = (uint32_t)(wv >> (16 * t)) & 0xffffu;
                const uint64_t sc = score(cp, call - cp, n_p, n_q);
                if (sc > best[s * 4 + t]) best[s * 4 + t] = sc;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < PB; ++t) {
        uint64_t v = valid ? best[t] : 0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            uint64_t o = __shfl_xor(v, off, 64);
            v = o > v ? o : v;
        }
        const int64_t b = q * PB + t;
        if (lane == 0 && b < B) atomicMax(nums + b, (unsigned long long)v);
    }
}

// res->ge = number of relabellings whose numerator is >= the observed one
// (all share one denominator, so the comparison is exact on numerators).
__global__ __launch_bounds__(256) void k_count_ge(const unsigned long long *__restrict__ nums, int B,
                                                  ResultDev *__restrict__ res)
{
    __shared__ unsigned long long tot;
    if (threadIdx.x == 0) tot = 0;
    __syncthreads();
    const unsigned long long obs = res->num;
    unsigned long long c = 0;
    for (int b = threadIdx.x; b < B; b += blockDim.x) c += nums[b] >= obs ? 1ull : 0ull;
    atomicAdd(&tot, c);
    __syncthreads();
    if (threadIdx.x == 0) res->ge = tot;
}

// ---------------------------------------------------------------- host side

hipError_t launch_count_ge(const unsigned long long *nums, int B, ResultDev *res, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_ge, dim3(1), dim3(256), 0, s, nums, B, res);
    return hipGetLastError();
}

size_t perm_lds_bytes(int d, int pb) { return (size_t)(pb / 4) * ((size_t)1 << d) * 64 * 8; }

int perm_max_group(int d)
{
    // 64-bit slots at most 64 KB apart (the ds_add immediate offset), and the
    // histograms of one wave within the 160 KB of LDS.
    return d <= 6 ? 8 : 4;
}

hipError_t launch_perm_prepare(const uint32_t *labels, int64_t n, int B, int64_t n_p, int pb,
                               uint64_t *inc, uint32_t *flags, unsigned long long *nums,
                               hipStream_t s)
{
    const int64_t words = (n + 31) / 32;
    const int64_t gq = (B + pb - 1) / pb;
    if (B > 0) {
        hipLaunchKernelGGL(k_perm_check_labels, dim3((unsigned)B), dim3(256), 0, s, labels, n, words,
                           n_p, flags);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t total = gq * n * (pb / 4);
        unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
        hipLaunchKernelGGL(k_perm_increments, dim3(blocks), dim3(256), 0, s, labels, n, words, B, pb,
                           gq, inc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        unsigned zb = (unsigned)std::min<int64_t>((B + 255) / 256, 1024);
        hipLaunchKernelGGL(k_zero_u64, dim3(zb), dim3(256), 0, s, (uint64_t *)nums, (int64_t)B);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <int D, int PATH, int PB, int W>
static hipError_t launch_perm_t(const void *Z, int64_t N, int64_t n_p, const uint64_t *inc, int B,
                                const uint32_t *obs, unsigned long long *nums, hipStream_t s)
{
    const size_t lds = perm_lds_bytes(D, PB);
    static std::once_flag attr;
    if (lds > 64 * 1024)
        std::call_once(attr, [lds] {
            if (hipFuncSetAttribute((const void *)k_perm<D, PATH, PB, W>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
                (void)hipGetLastError();
        });
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((B + PB - 1) / PB));
    hipLaunchKernelGGL((k_perm<D, PATH, PB, W>), grid, dim3(W * 64), lds, s, Z, N, n_p, N - n_p, inc, B,
                       obs, nums);
    return hipGetLastError();
}

template <int D, int PATH, int PB>
static hipError_t launch_perm_w(int waves, const void *Z, int64_t N, int64_t n_p, const uint64_t *inc,
                                int B, const uint32_t *obs, unsigned long long *nums, hipStream_t s)
{
    switch (waves) {
    case 4: return launch_perm_t<D, PATH, PB, 4>(Z, N, n_p, inc, B, obs, nums, s);
    case 8: return launch_perm_t<D, PATH, PB, 8>(Z, N, n_p, inc, B, obs, nums, s);
    case 16: return launch_perm_t<D, PATH, PB, 16>(Z, N, n_p, inc, B, obs, nums, s);
    default: return hipErrorInvalidValue;
    }
}

template <int D, int PATH>
static hipError_t launch_perm_d(int pb, int waves, const void *Z, int64_t N, int64_t n_p, const uint64_t *inc,
                                int B, const uint32_t *obs, unsigned long long *nums, hipStream_t s)
{
    if (pb == 4) return launch_perm_w<D, PATH, 4>(waves, Z, N, n_p, inc, B, obs, nums, s);
    if constexpr (D <= 6)
        if (pb == 8) return launch_perm_w<D, PATH, 8>(waves, Z, N, n_p, inc, B, obs, nums, s);
    return hipErrorInvalidValue;
}

template <int PATH>
static hipError_t launch_perm_p(int d, int pb, int waves, const void *Z, int64_t N, int64_t n_p,
                                const uint64_t *inc, int B, const uint32_t *obs,
                                unsigned long long *nums, hipStream_t s)
{
    switch (d) {
    case 1: return launch_perm_d<1, PATH>(pb, waves, Z, N, n_p, inc, B, obs, nums, s);
    case 2: return launch_perm_d<2, PATH>(pb, waves, Z, N, n_p, inc, B, obs, nums, s);
    case 3: return launch_perm_d<3, PATH>(pb, waves, Z, N, n_p, inc, B, obs, nums, s);
    case 4: return launch_perm_d<4, PATH>(pb, waves, Z, N, n_p, inc, B, obs, nums, s);
    case 5: return launch_perm_d<5, PATH>(pb, waves, Z, N, n_p, inc, B, obs, nums, s);
    case 6: return launch_perm_d<6, PATH>(pb, waves, Z, N, n_p, inc, B, obs, nums, s);
    case 7: return launch_perm_d<7, PATH>(pb, waves, Z, N, n_p, inc, B, obs, nums, s);
    case 8: return launch_perm_d<8, PATH>(pb, waves, Z, N, n_p, inc, B, obs, nums, s);
    default: return hipErrorInvalidValue;
    }
}

bool perm_shape_ok(int d, int pb, int waves)
{
    return (pb == 4 || (pb == 8 && d <= 6)) && (waves == 4 || waves == 8 || waves == 16);
}

hipError_t launch_perm(int path, int d, int pb, int waves, const void *Z, int64_t N, int64_t n_p,
                       const uint64_t *inc, int B, const uint32_t *obs_counts,
                       unsigned long long *nums, hipStream_t s)
{
    if (B < 1 || N < 2 || n_p < 1 || n_p >= N || n_p > 65535) return hipErrorInvalidValue;
    if (path == PATH_F32) return launch_perm_p<PATH_F32>(d, pb, waves, Z, N, n_p, inc, B, obs_counts, nums, s);
    if (path == PATH_R16) return launch_perm_p<PATH_R16>(d, pb, waves, Z, N, n_p, inc, B, obs_counts, nums, s);
    return hipErrorInvalidValue;
}

}  // namespace ddks
