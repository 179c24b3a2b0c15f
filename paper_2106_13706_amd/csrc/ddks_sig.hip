// Analytic significance of a ddKS statistic (arXiv:2106.13706, Sec. 3,
// Eq. ddks_significance) on the device, in fp64.
//
//   S = 1 - prod_{origins k, orthants j} P(delta <= D | n_P, n_T, lambda_kj)
//
// with lambda_kj = (c_T[k][j] + 1) / (n_T + 2) (Bayes estimator with a uniform
// prior) and delta = |a/n_P - b/n_T|, a ~ Bi(n_P, lambda), b ~ Bi(n_T, lambda)
// (Eq. abs_difference, Eq. binomial_probability).  In integers,
// delta <= D  <=>  |a*n_T - b*n_P| <= num, so for each a the admissible b form
// the window [lo_a, hi_a].  Each factor is evaluated through its complement
//   tail = sum_a Bi(a) * (F_T(lo_a - 1) + 1 - F_T(hi_a)),
// with the lower and upper binomial tails summed separately so that neither
// needs a difference of probabilities, and S = -expm1(sum log1p(-tail)).
//
// lambda depends only on c_T, so the product is grouped by the value of c_T:
// a histogram of c_T over all (k, j), one tail per distinct value, then one
// fixed-order reduction (deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ddks_internal.h"

namespace ddks {

static constexpr int SIG_THREADS = 256;

__global__ void k_sig_lgamma(double *L, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= n;
         k += (int64_t)gridDim.x * blockDim.x)
        L[k] = lgamma((double)k + 1.0);  // log k!
}

__global__ void k_sig_zero(unsigned long long *h, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        h[i] = 0;
}

__global__ void k_sig_hist(const uint32_t *__restrict__ counts, int64_t entries, int64_t n_q,
                           unsigned long long *__restrict__ hist, uint32_t *__restrict__ flags)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < entries;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t t = counts[e * 2 + 1];
        if ((int64_t)t > n_q) {
            atomicOr(flags, 4u);
            continue;
        }
        atomicAdd(&hist[t], 1ull);
    }
}

__device__ __forceinline__ double log_binom_pmf(const double *L, int64_t n, int64_t k, double ll,
                                                double l1m)
{
    return L[n] - L[k] - L[n - k] + (double)k * ll + (double)(n - k) * l1m;
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

// Inclusive block scan of one value per thread (Hillis-Steele in LDS).
__device__ double block_scan(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < SIG_THREADS; off <<= 1) {
        double u = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0.0;
        __syncthreads();
        sh[threadIdx.x] += u;
        __syncthreads();
    }
    double r = sh[threadIdx.x];
    __syncthreads();
    return r;
}

__device__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = SIG_THREADS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// One block per value t of c_T (grid-stride): terms[t] = hist[t] * log1p(-tail_t).
// rows: per block 2*(n_q+2) doubles: lower[b] = P(B < b), upper[b] = P(B > b).
__global__ __launch_bounds__(SIG_THREADS) void k_sig_tail(const double *__restrict__ L,
                                                          const unsigned long long *__restrict__ hist,
                                                          int64_t n_p, int64_t n_q, uint64_t num,
                                                          double *__restrict__ rows,
                                                          double *__restrict__ terms)
{
    __shared__ double sh[SIG_THREADS];
    __shared__ double carry;
    double *lower = rows + (size_t)blockIdx.x * 2 * (n_q + 2);
    double *upper = lower + (n_q + 2);
    for (int64_t t = blockIdx.x; t <= n_q; t += gridDim.x) {
        const unsigned long long h = hist[t];
        if (h == 0) {
            if (threadIdx.x == 0) terms[t] = 0.0;
            continue;
        }
        const double lam = ((double)t + 1.0) / ((double)n_q + 2.0);
        const double ll = log(lam), l1m = log1p(-lam);
        // lower[b] = sum_{b' < b} pmf(b'), b = 0..n_q+1 (prefix sums, chunk by chunk)
        if (threadIdx.x == 0) carry = 0.0;
        __syncthreads();
        for (int64_t c0 = 0; c0 <= n_q; c0 += SIG_THREADS) {
            const int64_t b = c0 + threadIdx.x;
            const double p = b <= n_q ? exp(log_binom_pmf(L, n_q, b, ll, l1m)) : 0.0;
            const double incl = block_scan(p, sh);
            if (b <= n_q) lower[b + 1] = carry + incl;
            __syncthreads();
            if (threadIdx.x == SIG_THREADS - 1) carry += incl;
            __syncthreads();
        }
        if (threadIdx.x == 0) lower[0] = 0.0;
        // upper[b] = sum_{b' > b} pmf(b'), summed from the top
        if (threadIdx.x == 0) carry = 0.0;
        __syncthreads();
        for (int64_t c0 = 0; c0 <= n_q; c0 += SIG_THREADS) {
            const int64_t b = n_q - (c0 + threadIdx.x);  // descending
            const double p = b >= 0 ? exp(log_binom_pmf(L, n_q, b, ll, l1m)) : 0.0;
            const double incl = block_scan(p, sh);      // sum over b' >= b within the chunk
            if (b >= 0) upper[b] = carry + incl - p;    // strictly above b
            __syncthreads();
            if (threadIdx.x == SIG_THREADS - 1) carry += incl;
            __syncthreads();
        }
        // tail = sum_a Bi(a; n_p) * (P(B < lo_a) + P(B > hi_a))
        double part = 0.0;
        for (int64_t a = threadIdx.x; a <= n_p; a += SIG_THREADS) {
            const int64_t lo = -floor_div((int64_t)num - a * n_q, n_p);  // ceil((a n_q - num)/n_p)
            const int64_t hi = floor_div(a * n_q + (int64_t)num, n_p);
            double excl;
            const int64_t lo_c = lo < 0 ? 0 : lo;
            const int64_t hi_c = hi > n_q ? n_q : hi;
            if (lo_c > hi_c)
                excl = 1.0;
            else
                excl = lower[lo_c] + upper[hi_c];
            part += exp(log_binom_pmf(L, n_p, a, ll, l1m)) * excl;
        }
        double tail = block_sum(part, sh);
        if (threadIdx.x == 0) {
            tail = tail < 0.0 ? 0.0 : (tail > 1.0 ? 1.0 : tail);
            terms[t] = (double)h * log1p(-tail);
        }
        __syncthreads();
    }
}

// S = -expm1(sum_t terms[t]), summed in a fixed order.
__global__ __launch_bounds__(SIG_THREADS) void k_sig_final(const double *__restrict__ terms,
                                                           int64_t n, double *__restrict__ S)
{
    __shared__ double sh[SIG_THREADS];
    double part = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += SIG_THREADS) part += terms[i];
    double tot = block_sum(part, sh);
    if (threadIdx.x == 0) *S = -expm1(tot) + 0.0;  // +0 rather than -0 when every tail is 0
}

size_t significance_scratch_bytes(int64_t n_p, int64_t n_q, int rows)
{
    const int64_t nmax = std::max(n_p, n_q);
    return (size_t)(nmax + 1) * 8 + (size_t)(n_q + 1) * 8 * 2 + (size_t)rows * 2 * (n_q + 2) * 8 + 64;
}

hipError_t launch_significance(const uint32_t *counts, int64_t N, int d, int64_t n_p, int64_t n_q,
                               uint64_t num, void *scratch, int rows, uint32_t *flags, double *S,
                               hipStream_t s)
{
    const int64_t nmax = std::max(n_p, n_q);
    double *L = (double *)scratch;
    unsigned long long *hist = (unsigned long long *)(L + nmax + 1);
    double *terms = (double *)(hist + n_q + 1);
    double *rowbuf = terms + n_q + 1;
    const int64_t entries = N << d;
    auto blocks = [](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); };
    hipLaunchKernelGGL(k_sig_lgamma, dim3(blocks(nmax + 1)), dim3(256), 0, s, L, nmax);
    hipLaunchKernelGGL(k_sig_zero, dim3(blocks(n_q + 1)), dim3(256), 0, s, hist, n_q + 1);
    hipLaunchKernelGGL(k_sig_hist, dim3(blocks(entries)), dim3(256), 0, s, counts, entries, n_q, hist,
                       flags);
    hipLaunchKernelGGL(k_sig_tail, dim3((unsigned)rows), dim3(SIG_THREADS), 0, s, L, hist, n_p, n_q,
                       num, rowbuf, terms);
    hipLaunchKernelGGL(k_sig_final, dim3(1), dim3(SIG_THREADS), 0, s, terms, n_q + 1, S);
    return hipGetLastError();
}

}  // namespace ddks
