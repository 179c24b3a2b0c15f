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
#include <mutex>

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
// dk and dm are k and m as doubles (exact: both are far below 2^53), kept
// by the callers' loops so that no 64-bit conversion runs per term.
template <int MODEL>
__device__ __forceinline__ double log_pmf(const double *L, int64_t m, int64_t k, double dm, double dk,
                                          double ll, double l1m, double lmu, double mu)
{
    if constexpr (MODEL == SIG_POISSON) return dk * lmu - mu - L[k];
    return L[m] - L[k] - L[m - k] + dk * ll + (dm - dk) * l1m;
}

// e^x for the log-probabilities x the sums exponentiate, by the table-driven
// reduction of P. T. P. Tang (ACM TOMS 15(2), 1989): x = (32 m + j) ln2/32 + r
// with |r| <= ln2/64, e^x = 2^m 2^(j/32) e^r, and e^r - 1 from its Taylor
// polynomial of degree 6 (remainder below 4e-18 relative at |r| = ln2/64).
// E[j] = 2^(j/32), j = 0..31, correctly rounded.  ln2/32 is split as
// EXP_LN2_32_HI (the leading 29 bits of its significand, so n HI is exact for
// |n| < 2^24) + EXP_LN2_32_LO; both and 32/ln2 come from a 60-digit ln2.
// Below -746 the result is below half the smallest subnormal: 0.
static constexpr double EXP_INV_LN2_32 = 0x1.71547652b82fep+5;
static constexpr double EXP_LN2_32_HI = 0x1.62e42ff000000p-6;
static constexpr double EXP_LN2_32_LO = -0x1.718432a1b0e26p-40;
static constexpr double EXP_MIN_ARG = -746.0;

__device__ __forceinline__ double exp_tab(double x, const double *E)
{
    const double xc = x > EXP_MIN_ARG ? x : EXP_MIN_ARG;  // keeps n within int range
    const double n = rint(xc * EXP_INV_LN2_32);
    const double r = fma(n, -EXP_LN2_32_LO, fma(n, -EXP_LN2_32_HI, xc));
    const int ni = (int)n;
    double q = fma(r, 1.0 / 720.0, 1.0 / 120.0);
    q = fma(r, q, 1.0 / 24.0);
    q = fma(r, q, 1.0 / 6.0);
    q = fma(r, q, 0.5);
    q = fma(r, q, 1.0);
    const double t = E[ni & 31];
    const double v = ldexp(fma(t, r * q, t), ni >> 5);  // arithmetic shift: floor(n / 32)
    return x > EXP_MIN_ARG ? v : 0.0;
}

// The table E of exp_tab in kernel arguments (filled on the host), copied to
// each block's LDS.
struct Exp2Table {
    double t[32];
};

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
// exp(-x^2 / (2 (sigma^2 + x/3))); with x = K/3 + sqrt(K^2/9 + 2 K sigma^2)
// that is exp(-K).  K = 700 (~1e-304) leaves out nothing S could show; the
// tail kernel first sums with K = SIG_K_NARROW and keeps that result when the
// tail is large enough for the left-out mass to be negligible beside it.
static constexpr double SIG_K_FULL = 700.0, SIG_K_NARROW = 100.0;
static constexpr double SIG_NARROW_MIN_TAIL = 1e-30;  // e^-100 ~ 4e-44 left out, < 1e-13 relative
static constexpr double SIG_WIDE_FIRST_Z = 12.0;       // normal tail ~4e-33
__host__ __device__ __forceinline__ int64_t window_halfwidth(double sigma, double K = SIG_K_FULL)
{
    return (int64_t)ceil(K / 3.0 + sqrt(K * K / 9.0 + 2.0 * K * sigma * sigma)) + 1;
}

// P(X > m), X ~ Poisson(mu), summed directly 64 terms at a time over
// (m, mu + w] (beyond mu + w the mass is below ~1e-304; L[k] = log k! is
// tabulated that far), stopping early once the terms stop mattering.
__device__ double pois_upper_wave(const double *L, const double *E, int64_t m, double mu, int64_t w)
{
    const int lane = threadIdx.x & 63;
    const double lmu = log(mu);
    const int64_t kmax = (int64_t)ceil(mu) + w;
    double total = 0.0;
    double dk = (double)(m + 1 + lane);
    for (int64_t k0 = m + 1; k0 <= kmax; k0 += 64, dk += 64.0) {
        const int64_t k = k0 + lane;
        const double c = wave_sum(k <= kmax ? exp_tab(dk * lmu - mu - L[k], E) : 0.0);
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

// One sample's side of a tail: n trials, pmf parameters, summation window [lo, hi].
struct SigSide {
    int64_t n, lo, hi;
    double lmu, mu, dn;  // dn = n as a double
};

// pmf of k (dk = k as a double) on side s.
template <int MODEL>
__device__ __forceinline__ double pmf(const double *L, const double *E, const SigSide &s, int64_t k, double dk,
                                      double ll, double l1m)
{
    return exp_tab(log_pmf<MODEL>(L, s.n, k, s.dn, dk, ll, l1m, s.lmu, s.mu), E);
}

// The same from the table entries already loaded: lk = log k!, lmk = log (n-k)!
// (binomial only), ln = log n!.
template <int MODEL>
__device__ __forceinline__ double pmf_of(double ln, double lk, double lmk, const double *E, const SigSide &s,
                                         double dk, double ll, double l1m)
{
    if constexpr (MODEL == SIG_POISSON) return exp_tab(dk * s.lmu - s.mu - lk, E);
    return exp_tab(ln - lk - lmk + dk * ll + (s.dn - dk) * l1m, E);
}

// Table entries of term k of side s (the second one for the binomial only).
template <int MODEL>
__device__ __forceinline__ void pmf_load(const double *L, const SigSide &s, int64_t k, double &lk, double &lmk)
{
    lk = L[k];
    if constexpr (MODEL != SIG_POISSON) lmk = L[s.n - k];
}

// sum of the pmf of side s over [k0, k1), one wave.
template <int MODEL>
__device__ double range_sum(const double *L, const double *E, const SigSide &s, int64_t k0, int64_t k1, double ll,
                            double l1m)
{
    const int lane = threadIdx.x & 63;
    double v = 0.0, dk = (double)(k0 + lane);
    for (int64_t k = k0 + lane; k < k1; k += 64, dk += 64.0) v += pmf<MODEL>(L, E, s, k, dk, ll, l1m);
    return wave_sum(v);
}

__device__ __forceinline__ double wave_excl_prefix(double v)  // sum over lanes below
{
    const double incl = wave_scan(v);
    const double e = __shfl_up(incl, 1, 64);
    return (threadIdx.x & 63) ? e : 0.0;
}

__device__ __forceinline__ double wave_excl_suffix(double v)  // sum over lanes above
{
    const int lane = threadIdx.x & 63;
    const double r = wave_scan(__shfl(v, 63 - lane, 64));  // prefix over reversed lanes
    const double e = __shfl(r, (62 - lane) & 63, 64);
    return lane < 63 ? e : 0.0;
}

// (q, r) with x = q n + r, 0 <= r < n (n > 0).
struct QR {
    int64_t q, r;
};
__device__ __forceinline__ QR divmod_floor(int64_t x, int64_t n)
{
    int64_t q = floor_div(x, n);
    return QR{q, x - q * n};
}
__device__ __forceinline__ void qr_add(QR &v, const QR &d, int64_t n)
{
    v.q += d.q;
    v.r += d.r;
    if (v.r >= n) {
        v.r -= n;
        v.q += 1;
    }
}
__device__ __forceinline__ void qr_sub(QR &v, const QR &d, int64_t n)
{
    v.q -= d.q;
    v.r -= d.r;
    if (v.r < 0) {
        v.r += n;
        v.q -= 1;
    }
}

// tail = sum over the outer count o in [O.lo, O.hi] of pmf_O(o) times the
// inner mass outside the admissible window of o, |o I.n - i O.n| <= num,
// i.e. i in [lo(o), hi(o)] with lo(o) = ceil((o I.n - num)/O.n) and
// hi(o) = floor((o I.n + num)/O.n), both nondecreasing in o.  The inner mass
// below lo(o) and the mass above hi(o) are summed in two passes (ascending and
// descending o), so that neither is a difference of probabilities.  Lane l of
// a chunk owns the R consecutive outer counts o = O0 + l R + r; it sums the
// inner pmf over its own span of targets, and one wave scan per chunk adds the
// spans of the lanes below it (above it, in the descending pass).  An o with
// no admissible i counts its whole inner mass (inner_tot) once.
template <int MODEL, int R>
__device__ double tail_two_pass(const double *L, const double *E, const SigSide &O, const SigSide &I, int64_t num,
                                double ll, double l1m)
{
    const int lane = threadIdx.x & 63;
    constexpr int64_t SPAN = 64 * R;
    const QR step = divmod_floor(I.n, O.n);           // x and y grow by I.n per outer count
    const QR cstep = divmod_floor(SPAN * I.n, O.n);   // ... and by SPAN I.n per chunk
    auto lo_of = [&](const QR &x) { return x.q + (x.r > 0 ? 1 : 0); };
    auto tgt_lo = [&](int64_t lo) { return lo < I.lo ? I.lo : (lo > I.hi + 1 ? I.hi + 1 : lo); };
    auto tgt_hi = [&](int64_t hi) { return hi + 1 < I.lo ? I.lo : (hi + 1 > I.hi + 1 ? I.hi + 1 : hi + 1); };
    const QR xtop = divmod_floor(O.hi * I.n - num, O.n), ytop = divmod_floor(O.hi * I.n + num, O.n);
    const int64_t T_top = tgt_lo(lo_of(xtop)), U_top = tgt_hi(ytop.q);
    const int64_t nch = (O.hi - O.lo + SPAN) / SPAN;
    const double Ln_I = MODEL == SIG_POISSON ? 0.0 : L[I.n];

    double acc_tail = 0.0, p_empty = 0.0;
    // ---- ascending pass: mass below lo(o)
    {
        const int64_t o0 = O.lo + lane * R;
        QR x = divmod_floor(o0 * I.n - num, O.n), y = divmod_floor(o0 * I.n + num, O.n);
        double carry = range_sum<MODEL>(L, E, I, I.lo, tgt_lo(lo_of(divmod_floor(O.lo * I.n - num, O.n))), ll, l1m);
        for (int64_t c = 0; c < nch; ++c) {
            const int64_t of = O.lo + c * SPAN + lane * R;
            int64_t T[R + 1];
            bool empty[R];
            QR xs = x, ys = y;
#pragma unroll
            for (int r = 0; r <= R; ++r) {
                const int64_t o = of + r;
                const int64_t lo = lo_of(xs), hi = ys.q;
                T[r] = o <= O.hi ? tgt_lo(lo) : T_top;
                if (r < R) empty[r] = (lo < 0 ? 0 : lo) > (hi > I.n ? I.n : hi);
                qr_add(xs, step, O.n);
                qr_add(ys, step, O.n);
            }
            // the lane's targets [T[0], T[R]) in ascending order, each term's
            // table entries loaded one term ahead (the last load repeats an
            // entry in range)
            double part[R], acc = 0.0, lk = 0.0, lmk = 0.0;
            int64_t i = T[0];
            double di = (double)i;
            if (i < T[R]) pmf_load<MODEL>(L, I, i, lk, lmk);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                part[r] = acc;
                for (; i < T[r + 1]; ++i, di += 1.0) {
                    double lk1 = 0.0, lmk1 = 0.0;
                    pmf_load<MODEL>(L, I, i + 1 < T[R] ? i + 1 : i, lk1, lmk1);
                    acc += pmf_of<MODEL>(Ln_I, lk, lmk, E, I, di, ll, l1m);
                    lk = lk1;
                    lmk = lmk1;
                }
            }
            const double pre = wave_excl_prefix(acc);
            const double tot = wave_sum(acc);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t o = of + r;
                if (o <= O.hi) {
                    const double po = pmf<MODEL>(L, E, O, o, (double)of + (double)r, ll, l1m);
                    if (empty[r])
                        p_empty += po;
                    else
                        acc_tail += po * (carry + pre + part[r]);
                }
            }
            carry += tot;
            qr_add(x, cstep, O.n);
            qr_add(y, cstep, O.n);
        }
        double inner_tot = 1.0;  // the whole binomial mass
        if constexpr (MODEL == SIG_POISSON) inner_tot = carry + range_sum<MODEL>(L, E, I, T_top, I.hi + 1, ll, l1m);
        acc_tail += p_empty * inner_tot;
    }
    // ---- descending pass: mass above hi(o)
    {
        const int64_t o0 = O.lo + (nch - 1) * SPAN + lane * R;
        QR x = divmod_floor(o0 * I.n - num, O.n), y = divmod_floor(o0 * I.n + num, O.n);
        double carry = range_sum<MODEL>(L, E, I, U_top, I.hi + 1, ll, l1m);
        for (int64_t c = nch - 1; c >= 0; --c) {
            const int64_t of = O.lo + c * SPAN + lane * R;
            int64_t U[R + 1];
            bool empty[R];
            QR xs = x, ys = y;
#pragma unroll
            for (int r = 0; r <= R; ++r) {
                const int64_t o = of + r;
                const int64_t lo = lo_of(xs), hi = ys.q;
                U[r] = o <= O.hi ? tgt_hi(hi) : U_top;
                if (r < R) empty[r] = (lo < 0 ? 0 : lo) > (hi > I.n ? I.n : hi);
                qr_add(xs, step, O.n);
                qr_add(ys, step, O.n);
            }
            // the lane's targets [U[0], U[R]) in descending order, loaded one
            // term ahead as in the ascending pass
            double sfx[R], acc = 0.0, lk = 0.0, lmk = 0.0;
            int64_t i = U[R] - 1;
            double di = (double)i;
            if (i >= U[0]) pmf_load<MODEL>(L, I, i, lk, lmk);
#pragma unroll
            for (int r = R - 1; r >= 0; --r) {
                for (; i >= U[r]; --i, di -= 1.0) {
                    double lk1 = 0.0, lmk1 = 0.0;
                    pmf_load<MODEL>(L, I, i - 1 >= U[0] ? i - 1 : i, lk1, lmk1);
                    acc += pmf_of<MODEL>(Ln_I, lk, lmk, E, I, di, ll, l1m);
                    lk = lk1;
                    lmk = lmk1;
                }
                sfx[r] = acc;
            }
            const double suf = wave_excl_suffix(acc);
            const double tot = wave_sum(acc);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t o = of + r;
                if (o <= O.hi && !empty[r])
                    acc_tail += pmf<MODEL>(L, E, O, o, (double)of + (double)r, ll, l1m) * (carry + suf + sfx[r]);
            }
            carry += tot;
            qr_sub(x, cstep, O.n);
            qr_sub(y, cstep, O.n);
        }
    }
    return wave_sum(acc_tail);
}

// One wave per value t of c_T (grid-stride over waves):
//   terms[t] = hist[t] * log1p(-tail_t).
// The sums are latency-bound (each term's table loads, dependent scans):
// built for 3 waves per SIMD (168 VGPRs, a few spilled outside the term
// loops) rather than the 2 that its ~210 VGPRs allow, with 4 outer counts per
// lane in the wide windows (against 8: binomial call 0.767 -> 0.718 ms, Poisson
// 0.749 -> 0.701 ms at 2 x 20000 points, with the one-term-ahead loads).
template <int MODEL>
__global__ __launch_bounds__(SIG_THREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_sig_tail(const double *__restrict__ L,
                                                          const unsigned long long *__restrict__ hist,
                                                          int64_t n_p, int64_t n_q, uint64_t num_imm,
                                                          const uint64_t *__restrict__ num_dev,
                                                          double *__restrict__ terms, Exp2Table e2)
{
    __shared__ double E[32];
    if (threadIdx.x < 32) E[threadIdx.x] = e2.t[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
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
        const double sq = MODEL == SIG_POISSON ? sqrt(muq) : sqrt(muq * (1.0 - lam));
        const double sp = MODEL == SIG_POISSON ? sqrt(mup) : sqrt(mup * (1.0 - lam));
        // the tail over windows of width K around both means
        auto tail_k = [&](double K) {
            const int64_t wq = window_halfwidth(sq, K), wp = window_halfwidth(sp, K);
            SigSide A, B;
            A.n = n_p;
            A.mu = mup;
            A.lmu = log(mup);
            A.dn = (double)n_p;
            A.lo = max((int64_t)0, (int64_t)floor(mup) - wp);
            A.hi = min(n_p, (int64_t)ceil(mup) + wp);
            B.n = n_q;
            B.mu = muq;
            B.lmu = log(muq);
            B.dn = (double)n_q;
            B.lo = max((int64_t)0, (int64_t)floor(muq) - wq);
            B.hi = min(n_q, (int64_t)ceil(muq) + wq);
            // the larger window is the outer one, so that the lanes stay busy
            // (the condition |a n_q - b n_p| > num is symmetric in the two sides)
            const bool a_outer = (A.hi - A.lo) >= (B.hi - B.lo);
            const SigSide &O = a_outer ? A : B;
            const SigSide &I = a_outer ? B : A;
            return (O.hi - O.lo + 1 >= 4 * 64) ? tail_two_pass<MODEL, 4>(L, E, O, I, num, ll, l1m)
                                               : tail_two_pass<MODEL, 1>(L, E, O, I, num, ll, l1m);
        };
        // A normal approximation of delta (variance lam (1 - lam) (1/n_p + 1/n_q),
        // lam (1/n_p + 1/n_q) for the Poisson model) picks the first window:
        // where D lies more than SIG_WIDE_FIRST_Z of its deviations out, the
        // tail is far below SIG_NARROW_MIN_TAIL and the narrow windows would be
        // summed in vain.  The estimate only decides the work: the wide windows
        // are valid for every tail.
        const double var_d = (MODEL == SIG_POISSON ? lam : lam * (1.0 - lam)) *
                             (1.0 / (double)n_p + 1.0 / (double)n_q);
        const double z = ((double)num / ((double)n_p * (double)n_q)) / sqrt(var_d);
        const bool wide_first = z > SIG_WIDE_FIRST_Z;  // wave-uniform
        double tail = tail_k(wide_first ? SIG_K_FULL : SIG_K_NARROW);
        if (!wide_first && !(tail >= SIG_NARROW_MIN_TAIL)) tail = tail_k(SIG_K_FULL);  // wave-uniform
        const int64_t wq = window_halfwidth(sq), wp = window_halfwidth(sp);
        if constexpr (MODEL == SIG_POISSON) {
            // mass of either Poisson count beyond its sample size
            const double ua = pois_upper_wave(L, E, n_p, mup, wp), ub = pois_upper_wave(L, E, n_q, muq, wq);
            tail += ua + ub - ua * ub;
        }
        if (lane == 0) {
            tail = tail < 0.0 ? 0.0 : (tail > 1.0 ? 1.0 : tail);
            terms[t] = (double)h * log1p(-tail);
        }
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
int significance_rows(int64_t n_q, int model)
{
    // waves in flight: one per value of c_T up to 8192, a multiple of the four
    // waves of a block
    (void)model;
    const int64_t r = std::min<int64_t>(n_q + 4, 8192);
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
    (void)rows;
    (void)model;
    return (size_t)(sig_lmax(n_p, n_q) + 1) * 8 + (size_t)(n_q + 1) * 8 * 2 + 64;
}

hipError_t launch_significance(const uint32_t *counts, int64_t N, int d, int64_t n_p, int64_t n_q,
                               uint64_t num, const uint64_t *num_dev, int model, void *scratch,
                               int rows, uint32_t *flags, double *S, hipStream_t s)
{
    const int64_t lmax = sig_lmax(n_p, n_q);
    double *L = (double *)scratch;
    unsigned long long *hist = (unsigned long long *)(L + lmax + 1);
    double *terms = (double *)(hist + n_q + 1);
    const int64_t entries = N << d;
    auto blocks = [](int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); };
    if (rows < 4 || rows % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sig_lgamma, dim3(blocks(lmax + 1)), dim3(256), 0, s, L, lmax);
    hipLaunchKernelGGL(k_sig_zero, dim3(blocks(n_q + 1)), dim3(256), 0, s, hist, n_q + 1);
    if (n_q + 1 <= HIST_LDS) {
        // about one block per CU, each with its own LDS histogram
        const unsigned hb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((entries + 1023) / 1024, 256));
        const size_t lds = (size_t)(n_q + 1) * sizeof(uint32_t);
        // once per process (serving threads and plain calls may get here together)
        static std::once_flag attr;
        std::call_once(attr, [] {
            if (hipFuncSetAttribute((const void *)k_sig_hist<true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    HIST_LDS * (int)sizeof(uint32_t)) != hipSuccess)
                (void)hipGetLastError();
        });
        hipLaunchKernelGGL(k_sig_hist<true>, dim3(hb), dim3(1024), lds, s, counts, entries, n_q, hist,
                           flags);
    } else {
        hipLaunchKernelGGL(k_sig_hist<false>, dim3(blocks(entries)), dim3(1024), 0, s, counts, entries,
                           n_q, hist, flags);
    }
    // 2^(j/32), correctly rounded: from the 64-bit-significand long double
    static const Exp2Table e2 = [] {
        Exp2Table t;
        for (int j = 0; j < 32; ++j) t.t[j] = (double)exp2l((long double)j / 32.0L);
        return t;
    }();
    const unsigned tb = (unsigned)(rows / 4);  // four waves per block
    if (model == SIG_POISSON)
        hipLaunchKernelGGL(k_sig_tail<SIG_POISSON>, dim3(tb), dim3(SIG_THREADS), 0, s, L, hist, n_p,
                           n_q, num, num_dev, terms, e2);
    else
        hipLaunchKernelGGL(k_sig_tail<SIG_BINOMIAL>, dim3(tb), dim3(SIG_THREADS), 0, s, L, hist, n_p,
                           n_q, num, num_dev, terms, e2);
    hipLaunchKernelGGL(k_sig_final, dim3(1), dim3(SIG_THREADS), 0, s, terms, n_q + 1, S);
    return hipGetLastError();
}

}  // namespace ddks
