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
// a histogram of c_T over all (k, j), one tail per distinct value (one wave
// each, sums over windows around the means outside which the left-out mass
// is below ~1e-304, by Bernstein's inequality), then one fixed-order reduction
// (deterministic).  The Poisson model (Sec. 3's large-sample replacement of
// each binomial pmf by the Poisson pmf of the same mean, over the same
// supports 0..m) adds the Poisson mass beyond each sample size to the tail:
// P(delta <= D) = Z_a Z_b - excluded, so 1 - P = (1 - Z_a Z_b) + excluded.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ddks_internal.h"

namespace ddks {

static constexpr int SIG_THREADS = 256;
constexpr int SIG_BINOMIAL = SIG_MODEL_BINOMIAL, SIG_POISSON = SIG_MODEL_POISSON;

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

// Histogram of the second-sample counts c_T over all (origin, orthant)
// entries.  With n_q + 1 <= HIST_LDS values a block first counts its share in
// LDS (values repeat a lot, and same-address global atomics serialise), then
// adds its non-zero bins to the global histogram; otherwise it adds directly.
static constexpr int HIST_LDS = 32768;  // 128 KB of 32-bit LDS counters

template <bool LDS>
__global__ __launch_bounds__(1024) void k_sig_hist(const uint32_t *__restrict__ counts, int64_t entries,
                                                   int64_t n_q, unsigned long long *__restrict__ hist,
                                                   uint32_t *__restrict__ flags)
{
    extern __shared__ uint32_t lh[];
    if constexpr (LDS) {
        for (int64_t v = threadIdx.x; v <= n_q; v += blockDim.x) lh[v] = 0;
        __syncthreads();
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < entries;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t t = counts[e * 2 + 1];
        if ((int64_t)t > n_q) {
            atomicOr(flags, 4u);
            continue;
        }
        if constexpr (LDS)
            atomicAdd(&lh[t], 1u);
        else
            atomicAdd(&hist[t], 1ull);
    }
    if constexpr (LDS) {
        __syncthreads();
        for (int64_t v = threadIdx.x; v <= n_q; v += blockDim.x)
            if (lh[v]) atomicAdd(&hist[v], (unsigned long long)lh[v]);
    }
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

// log pmf of k successes in m trials at rate lam: binomial (Eq.
// binomial_probability), or Poisson of mean mu = m lam (Sec. 3's large-sample
// replacement).  L[k] = log k! for k up to one window past max(n_p, n_q).
template <int MODEL>
__device__ __forceinline__ double log_pmf(const double *L, int64_t m, int64_t k, double ll,
                                          double l1m, double lmu, double mu)
{
    if constexpr (MODEL == SIG_POISSON) return (double)k * lmu - mu - L[k];
    return L[m] - L[k] - L[m - k] + (double)k * ll + (double)(m - k) * l1m;
}

__device__ __forceinline__ double wave_scan(double v)  // inclusive, over the 64 lanes
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        double u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Half-width x of the summation window around the mean.  By Bernstein's
// inequality a count x or more away from its mean has probability at most
// exp(-x^2 / (2 (sigma^2 + x/3))); with x = 700/3 + sqrt((700/3)^2 +
// 1400 sigma^2) that is exp(-700) ~ 1e-304, so every term left out is far
// below the precision S is computed to.
__host__ __device__ __forceinline__ int64_t window_halfwidth(double sigma)
{
    return (int64_t)ceil(700.0 / 3.0 + sqrt(700.0 * 700.0 / 9.0 + 1400.0 * sigma * sigma)) + 1;
}

// P(X > m), X ~ Poisson(mu), summed directly 64 terms at a time over
// (m, mu + w] (beyond mu + w the mass is below ~1e-304; L[k] = log k! is
// tabulated that far), stopping early once the terms stop mattering.
__device__ double pois_upper_wave(const double *L, int64_t m, double mu, int64_t w)
{
    const int lane = threadIdx.x & 63;
    const double lmu = log(mu);
    const int64_t kmax = (int64_t)ceil(mu) + w;
    double total = 0.0;
    for (int64_t k0 = m + 1; k0 <= kmax; k0 += 64) {
        const int64_t k = k0 + lane;
        const double c = wave_sum(k <= kmax ? exp((double)k * lmu - mu - L[k]) : 0.0);
        total += c;
        if ((double)k0 > mu && (c == 0.0 || c < total * 1e-18)) break;
    }
    return total;
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

// One wave per value t of c_T (grid-stride over waves):
//   terms[t] = hist[t] * log1p(-tail_t).
// rows: per wave 2 * wmax doubles: lower[i] = sum of the pmf of b over
// [b_lo, b_lo + i), upper[i] = sum over (b_lo + i, b_hi], on the window
// [b_lo, b_hi] around b's mean.
template <int MODEL>
__global__ __launch_bounds__(SIG_THREADS) void k_sig_tail(const double *__restrict__ L,
                                                          const unsigned long long *__restrict__ hist,
                                                          int64_t n_p, int64_t n_q, uint64_t num_imm,
                                                          const uint64_t *__restrict__ num_dev,
                                                          int64_t wmax, double *__restrict__ rows,
                                                          double *__restrict__ terms)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    double *lower = rows + (size_t)wave * 2 * wmax;
    double *upper = lower + wmax;
    const int64_t num = (int64_t)(num_dev ? *num_dev : num_imm);
    for (int64_t t = wave; t <= n_q; t += nwaves) {
        const unsigned long long h = hist[t];
        if (h == 0) {
            if (lane == 0) terms[t] = 0.0;
            continue;
        }
        const double lam = ((double)t + 1.0) / ((double)n_q + 2.0);
        const double ll = log(lam), l1m = log1p(-lam);
        const double muq = (double)n_q * lam, mup = (double)n_p * lam;
        const double lmuq = log(muq), lmup = log(mup);
        const double sq = MODEL == SIG_POISSON ? sqrt(muq) : sqrt(muq * (1.0 - lam));
        const double sp = MODEL == SIG_POISSON ? sqrt(mup) : sqrt(mup * (1.0 - lam));
        const int64_t wq = window_halfwidth(sq), wp = window_halfwidth(sp);
        const int64_t b_lo = max((int64_t)0, (int64_t)floor(muq) - wq);
        const int64_t b_hi = min(n_q, (int64_t)ceil(muq) + wq);
        const int64_t a_lo = max((int64_t)0, (int64_t)floor(mup) - wp);
        const int64_t a_hi = min(n_p, (int64_t)ceil(mup) + wp);
        const int64_t nb = b_hi - b_lo + 1;  // <= wmax - 1

        double carry = 0.0;
        for (int64_t c0 = 0; c0 < nb; c0 += 64) {
            const int64_t i = c0 + lane;
            const double p = i < nb ? exp(log_pmf<MODEL>(L, n_q, b_lo + i, ll, l1m, lmuq, muq)) : 0.0;
            const double incl = wave_scan(p);
            if (i < nb) lower[i + 1] = carry + incl;
            carry += __shfl(incl, 63, 64);
        }
        if (lane == 0) lower[0] = 0.0;
        const double tot_b = carry;
        carry = 0.0;
        for (int64_t c0 = 0; c0 < nb; c0 += 64) {
            const int64_t i = nb - 1 - (c0 + lane);  // descending
            const double p = i >= 0 ? exp(log_pmf<MODEL>(L, n_q, b_lo + i, ll, l1m, lmuq, muq)) : 0.0;
            const double incl = wave_scan(p);         // over b >= b_lo + i within the chunk
            if (i >= 0) upper[i] = carry + incl - p;  // strictly above b_lo + i
            carry += __shfl(incl, 63, 64);
        }
        __threadfence_block();  // the rows are read back by other lanes of the wave

        double part = 0.0;
        for (int64_t a = a_lo + lane; a <= a_hi; a += 64) {
            const int64_t lo = -floor_div(num - a * n_q, n_p);  // ceil((a n_q - num)/n_p)
            const int64_t hi = floor_div(a * n_q + num, n_p);
            const int64_t lo_c = lo < 0 ? 0 : lo;
            const int64_t hi_c = hi > n_q ? n_q : hi;
            double excl;
            if (lo_c > hi_c) {
                excl = MODEL == SIG_POISSON ? tot_b : 1.0;  // every b is excluded
            } else {
                const double below = lo_c <= b_lo ? 0.0 : (lo_c > b_hi ? tot_b : lower[lo_c - b_lo]);
                const double above = hi_c >= b_hi ? 0.0 : (hi_c < b_lo ? tot_b : upper[hi_c - b_lo]);
                excl = below + above;
            }
            part += exp(log_pmf<MODEL>(L, n_p, a, ll, l1m, lmup, mup)) * excl;
        }
        double tail = wave_sum(part);
        if constexpr (MODEL == SIG_POISSON) {
            // mass of either Poisson count beyond its sample size
            const double ua = pois_upper_wave(L, n_p, mup, wp), ub = pois_upper_wave(L, n_q, muq, wq);
            tail += ua + ub - ua * ub;
        }
        if (lane == 0) {
            tail = tail < 0.0 ? 0.0 : (tail > 1.0 ? 1.0 : tail);
            terms[t] = (double)h * log1p(-tail);
        }
        __threadfence_block();  // this wave's rows are rewritten for its next value
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

// Largest summation window (entries of b) for n_q trials over every rate,
// plus the two ends: sigma^2 = n_q lambda (1 - lambda) <= n_q / 4 for the
// binomial, n_q lambda < n_q for the Poisson model.
static int64_t sig_wmax(int64_t n_q, int model)
{
    const double sig = model == SIG_POISSON ? sqrt((double)n_q) : 0.5 * sqrt((double)n_q);
    const int64_t w = window_halfwidth(sig);
    return std::min<int64_t>(n_q + 1, 2 * w + 3) + 2;
}

int significance_rows(int64_t n_q, int model)
{
    // one pair of window rows per wave in flight (at most 8192 waves and
    // 384 MB of rows), a multiple of the four waves of a block
    const int64_t per = 16 * sig_wmax(n_q, model);
    const int64_t r = std::min<int64_t>({(int64_t)(384ull << 20) / per, n_q + 4, 8192});
    return (int)std::max<int64_t>(4, r / 4 * 4);
}

// Entries of the log-factorial table: up to max(n_p, n_q), and one window
// further for the Poisson mass beyond the sample sizes.
static int64_t sig_lmax(int64_t n_p, int64_t n_q)
{
    const int64_t nmax = std::max(n_p, n_q);
    return nmax + window_halfwidth(sqrt((double)nmax)) + 2;
}

size_t significance_scratch_bytes(int64_t n_p, int64_t n_q, int rows, int model)
{
    return (size_t)(sig_lmax(n_p, n_q) + 1) * 8 + (size_t)(n_q + 1) * 8 * 2 +
           (size_t)rows * 2 * sig_wmax(n_q, model) * 8 + 64;
}

hipError_t launch_significance(const uint32_t *counts, int64_t N, int d, int64_t n_p, int64_t n_q,
                               uint64_t num, const uint64_t *num_dev, int model, void *scratch,
                               int rows, uint32_t *flags, double *S, hipStream_t s)
{
    const int64_t lmax = sig_lmax(n_p, n_q);
    double *L = (double *)scratch;
    unsigned long long *hist = (unsigned long long *)(L + lmax + 1);
    double *terms = (double *)(hist + n_q + 1);
    double *rowbuf = terms + n_q + 1;
    const int64_t entries = N << d;
    const int64_t wmax = sig_wmax(n_q, model);
    auto blocks = [](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); };
    if (rows < 4 || rows % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sig_lgamma, dim3(blocks(lmax + 1)), dim3(256), 0, s, L, lmax);
    hipLaunchKernelGGL(k_sig_zero, dim3(blocks(n_q + 1)), dim3(256), 0, s, hist, n_q + 1);
    if (n_q + 1 <= HIST_LDS) {
        // about one block per CU, each with its own LDS histogram
        const unsigned hb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((entries + 1023) / 1024, 256));
        const size_t lds = (size_t)(n_q + 1) * sizeof(uint32_t);
        static bool attr = false;
        if (!attr) {
            if (hipFuncSetAttribute((const void *)k_sig_hist<true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    HIST_LDS * (int)sizeof(uint32_t)) != hipSuccess)
                (void)hipGetLastError();
            attr = true;
        }
        hipLaunchKernelGGL(k_sig_hist<true>, dim3(hb), dim3(1024), lds, s, counts, entries, n_q, hist,
                           flags);
    } else {
        hipLaunchKernelGGL(k_sig_hist<false>, dim3(blocks(entries)), dim3(1024), 0, s, counts, entries,
                           n_q, hist, flags);
    }
    const unsigned tb = (unsigned)(rows / 4);  // four waves per block
    if (model == SIG_POISSON)
        hipLaunchKernelGGL(k_sig_tail<SIG_POISSON>, dim3(tb), dim3(SIG_THREADS), 0, s, L, hist, n_p,
                           n_q, num, num_dev, wmax, rowbuf, terms);
    else
        hipLaunchKernelGGL(k_sig_tail<SIG_BINOMIAL>, dim3(tb), dim3(SIG_THREADS), 0, s, L, hist, n_p,
                           n_q, num, num_dev, wmax, rowbuf, terms);
    hipLaunchKernelGGL(k_sig_final, dim3(1), dim3(SIG_THREADS), 0, s, terms, n_q + 1, S);
    return hipGetLastError();
}

}  // namespace ddks
