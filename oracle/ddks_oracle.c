/*
 * ddks_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of the exact ddKS
 * statistic (Hagen et al., "Accelerated Computation of a High Dimensional
 * Kolmogorov-Smirnov Distance", arXiv:2106.13706).  It exists to check the
 * GPU library, never to serve it: only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * What it computes (all citations are to the paper):
 *
 *   Sec. 2.1, Eq. (ddks_tensor_definition): the cumulative-density tensors
 *   C_{X,x} are evaluated at every point of both samples, origins taken in
 *   the order P then T (the paper's T is called Q here).
 *
 *   Sec. 2.1 (loop method) / Sec. 2.2.1, Eq. (g): for each origin o and each
 *   point x, the point lies on the upper side of dimension m when
 *   x_m >= o_m (IEEE comparison: -0 == +0, ties go to the upper side, so the
 *   origin counts itself in the all-upper orthant).  The orthant of x is
 *   code = sum_m [x_m >= o_m] * 2^m; each of the 2^d orthants is one
 *   choice of side (below or at-or-above) in every dimension.
 *
 *   Eq. (membership) counts the points of each sample per orthant; Eq. (d1)
 *   takes the maximum absolute difference.  Reading of the normalisation:
 *   the difference is between proportions, |c_P/n_P - c_Q/n_Q| (the Fig. 2a
 *   caption calls the value normalised; Sec. 3, Eq. abs_difference).
 *   It is evaluated exactly in integers as |c_P*n_Q - c_Q*n_P| = num, with
 *   den = n_P*n_Q and D = num/den.
 *
 *   Ties in the maximum are reported at the lowest origin index (P then Q
 *   order), then the lowest orthant code (strict '>' while scanning in
 *   ascending order).  D itself is unique.
 *
 *   Sec. 3: analytic significance S = 1 - prod_{orthant,origin}
 *   P(delta <= D | n_P, n_T, lambda), lambda = (M_T + 1)/(N_T + 2) (Bayes
 *   estimator with a uniform prior), delta the absolute difference of two
 *   binomial proportions (Eq. abs_difference, Eq. binomial_probability,
 *   Eq. ddks_significance).  Sec. 3 also proposes, for large samples and
 *   small rates, replacing each binomial pmf by the Poisson pmf of the same
 *   mean and carrying the derivation through; reading: the sums keep their
 *   support 0..m (the set Delta), so P(delta <= D) is the windowed sum of
 *   products of Poisson pmfs over that support.
 *
 *   Sec. 2.2.2, Alg. 1 (vdKS): the voxel approximation -- the pooled points
 *   binned on a V^d grid of the normalised data, orthant sums of the two
 *   samples' voxel counts around every filled voxel (readings at
 *   ddks_oracle_vdks).
 *
 *   Sec. 2.2.3, Alg. 2 (rdKS): the radial approximation -- for each of d + 1
 *   corners of the normalised space, the two-sample KS statistic of the
 *   samples' distances from that corner (readings at ddks_oracle_rdks).
 *
 *   Sec. 3 / Sec. 4.2: permutation test -- the statistic recomputed for
 *   relabelled pooled samples; here each relabelling is rebuilt as two
 *   samples in index order and the definition is re-run from scratch.
 *
 * Precision: the inputs are fp32; comparisons are done on their exact
 * double-precision values (identical to fp32 comparison), counts are
 * uint32, scores int64, D one double division, S in fp64.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -4

/* Rate models of the significance (Sec. 3). */
#define DDKS_ORACLE_BINOMIAL 0
#define DDKS_ORACLE_POISSON 1

/* ------------------------------------------------------------------------- */
/* Exact statistic by the definition                                         */
/* ------------------------------------------------------------------------- */

typedef struct {
    /* inputs */
    const float *P, *Q;
    int64_t n_p, n_q;
    int d;
    int64_t k_begin, k_end; /* origin range [k_begin, k_end) in P-then-Q order */
    uint32_t *counts;       /* nullable, [N][2^d][2] */
    uint64_t *origin_num;   /* nullable, [N] best score per origin */
    int32_t *origin_code;   /* nullable, [N] its (lowest) orthant */
    /* outputs of this chunk */
    uint64_t best_num;
    int64_t best_k;
    int32_t best_j;
    int status;
} chunk_job;

/* The k-th origin of the concatenation P then Q (Eq. ddks_tensor_definition). */
static const float *origin_at(const chunk_job *job, int64_t k)
{
    if (k < job->n_p) return job->P + k * job->d;
    return job->Q + (k - job->n_p) * job->d;
}

/* Orthant code of x relative to o: bit m set when x_m >= o_m (Eq. g). */
static uint32_t orthant_code(const float *x, const float *o, int d)
{
    uint32_t code = 0;
    for (int m = 0; m < d; ++m) {
        double xm = (double)x[m];
        double om = (double)o[m];
        if (xm >= om) code |= (uint32_t)1 << m;
    }
    return code;
}

static void *run_chunk(void *arg)
{
    chunk_job *job = (chunk_job *)arg;
    const int d = job->d;
    const uint32_t bins = (uint32_t)1 << d;
    uint32_t *cP = (uint32_t *)calloc(bins, sizeof(uint32_t));
    uint32_t *cQ = (uint32_t *)calloc(bins, sizeof(uint32_t));
    job->best_num = 0;
    job->best_k = -1;
    job->best_j = -1;
    job->status = ORACLE_OK;
    if (!cP || !cQ) {
        free(cP);
        free(cQ);
        job->status = ORACLE_ENOMEM;
        return NULL;
    }
    for (int64_t k = job->k_begin; k < job->k_end; ++k) {
        const float *o = origin_at(job, k);
        memset(cP, 0, bins * sizeof(uint32_t));
        memset(cQ, 0, bins * sizeof(uint32_t));
        /* Eq. (membership): count the points of each sample per orthant. */
        for (int64_t i = 0; i < job->n_p; ++i) cP[orthant_code(job->P + i * d, o, d)] += 1;
        for (int64_t i = 0; i < job->n_q; ++i) cQ[orthant_code(job->Q + i * d, o, d)] += 1;
        /* Eq. (d1), normalised: |cP/nP - cQ/nQ| scaled by nP*nQ. */
        uint64_t k_best = 0;
        int32_t k_best_j = 0;
        for (uint32_t j = 0; j < bins; ++j) {
            int64_t a = (int64_t)cP[j] * job->n_q;
            int64_t b = (int64_t)cQ[j] * job->n_p;
            uint64_t s = (uint64_t)(a > b ? a - b : b - a);
            if (s > k_best) {
                k_best = s;
                k_best_j = (int32_t)j;
            }
            if (job->counts) {
                job->counts[((size_t)k * bins + j) * 2 + 0] = cP[j];
                job->counts[((size_t)k * bins + j) * 2 + 1] = cQ[j];
            }
        }
        if (job->origin_num) job->origin_num[k] = k_best;
        if (job->origin_code) job->origin_code[k] = k_best_j;
        /* first origin attaining a strictly larger score wins */
        if (job->best_k < 0 || k_best > job->best_num) {
            job->best_num = k_best;
            job->best_k = k;
            job->best_j = k_best_j;
        }
    }
    free(cP);
    free(cQ);
    return NULL;
}

/*
 * ddks_oracle_distance: exact ddKS of P (n_p x d, row-major fp32) and
 * Q (n_q x d).  n_threads >= 1 splits the origins into contiguous chunks.
 * counts (nullable): [n_p+n_q][2^d][2] uint32, sample 0 = P.
 * origin_num / origin_code (nullable): per-origin maximum score and orthant.
 * Outputs num (den = n_p*n_q) and the argmax (origin in P-then-Q order,
 * orthant code).
 */
int ddks_oracle_distance(const float *P, int64_t n_p, const float *Q, int64_t n_q, int32_t d,
                         int32_t n_threads, uint32_t *counts, uint64_t *origin_num,
                         int32_t *origin_code, uint64_t *num, int64_t *arg_origin,
                         int32_t *arg_orthant)
{
    if (!P || !Q || !num || n_p < 1 || n_q < 1 || d < 1 || d > 16) return ORACLE_EINVAL;
    if (n_p > 0x7fffffffLL || n_q > 0x7fffffffLL) return ORACLE_EINVAL;
    const int64_t N = n_p + n_q;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > N) n_threads = (int32_t)N;

    chunk_job *jobs = (chunk_job *)calloc((size_t)n_threads, sizeof(chunk_job));
    pthread_t *tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return ORACLE_ENOMEM;
    }
    for (int t = 0; t < n_threads; ++t) {
        jobs[t].P = P;
        jobs[t].Q = Q;
        jobs[t].n_p = n_p;
        jobs[t].n_q = n_q;
        jobs[t].d = d;
        jobs[t].k_begin = N * t / n_threads;
        jobs[t].k_end = N * (t + 1) / n_threads;
        jobs[t].counts = counts;
        jobs[t].origin_num = origin_num;
        jobs[t].origin_code = origin_code;
    }
    int spawned = 0;
    for (int t = 1; t < n_threads; ++t) {
        if (pthread_create(&tids[t], NULL, run_chunk, &jobs[t]) != 0) break;
        spawned = t;
    }
    run_chunk(&jobs[0]);
    for (int t = 1; t <= spawned; ++t) pthread_join(tids[t], NULL);
    for (int t = spawned + 1; t < n_threads; ++t) run_chunk(&jobs[t]); /* threads we could not start */

    /* Merge chunk results in ascending origin order with strict '>',
       identical to the serial scan. */
    int status = ORACLE_OK;
    uint64_t best = 0;
    int64_t bk = -1;
    int32_t bj = -1;
    for (int t = 0; t < n_threads; ++t) {
        if (jobs[t].status != ORACLE_OK) status = jobs[t].status;
        if (jobs[t].best_k < 0) continue;
        if (bk < 0 || jobs[t].best_num > best) {
            best = jobs[t].best_num;
            bk = jobs[t].best_k;
            bj = jobs[t].best_j;
        }
    }
    free(jobs);
    free(tids);
    if (status != ORACLE_OK) return status;
    *num = best;
    if (arg_origin) *arg_origin = bk;
    if (arg_orthant) *arg_orthant = bj;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* Permutation test: every relabelling re-run through the definition          */
/* ------------------------------------------------------------------------- */

/*
 * Z: pooled points (n x d).  labels: B rows of ceil(n/32) uint32 words; bit i
 * of a row (word i/32, bit i%32) set means point i belongs to the first
 * sample.  Every row must have exactly n_p set bits.  nums[b] receives the
 * numerator of the statistic for row b (shared den = n_p*(n-n_p)).
 */
int ddks_oracle_permutation(const float *Z, int64_t n, int32_t d, int64_t n_p,
                            const uint32_t *labels, int32_t B, int32_t n_threads,
                            uint64_t *nums)
{
    if (!Z || !labels || !nums || n < 2 || n_p < 1 || n_p >= n || d < 1 || d > 16 || B < 0)
        return ORACLE_EINVAL;
    const int64_t words = (n + 31) / 32;
    float *A = (float *)malloc((size_t)n_p * d * sizeof(float));
    float *Bs = (float *)malloc((size_t)(n - n_p) * d * sizeof(float));
    if (!A || !Bs) {
        free(A);
        free(Bs);
        return ORACLE_ENOMEM;
    }
    int status = ORACLE_OK;
    for (int32_t b = 0; b < B && status == ORACLE_OK; ++b) {
        const uint32_t *row = labels + (size_t)b * words;
        int64_t ia = 0, ib = 0;
        for (int64_t i = 0; i < n; ++i) {
            int in_first = (row[i / 32] >> (i % 32)) & 1u;
            if (in_first) {
                if (ia >= n_p) { status = ORACLE_EINVAL; break; }
                memcpy(A + ia * d, Z + i * d, (size_t)d * sizeof(float));
                ++ia;
            } else {
                if (ib >= n - n_p) { status = ORACLE_EINVAL; break; }
                memcpy(Bs + ib * d, Z + i * d, (size_t)d * sizeof(float));
                ++ib;
            }
        }
        if (status != ORACLE_OK) break;
        if (ia != n_p) { status = ORACLE_EINVAL; break; }
        status = ddks_oracle_distance(A, n_p, Bs, n - n_p, d, n_threads, NULL, NULL, NULL,
                                      &nums[b], NULL, NULL);
    }
    free(A);
    free(Bs);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Analytic significance (Sec. 3)                                             */
/* ------------------------------------------------------------------------- */

/* Binomial pmf p(n : m, lambda) = C(m,n) lambda^n (1-lambda)^(m-n)
   (Eq. binomial_probability), evaluated in log space. */
static double binom_pmf(int64_t k, int64_t m, double lam)
{
    if (k < 0 || k > m) return 0.0;
    if (lam <= 0.0) return k == 0 ? 1.0 : 0.0;
    if (lam >= 1.0) return k == m ? 1.0 : 0.0;
    double lc = lgamma((double)m + 1.0) - lgamma((double)k + 1.0) - lgamma((double)(m - k) + 1.0);
    return exp(lc + (double)k * log(lam) + (double)(m - k) * log1p(-lam));
}

/* Poisson pmf e^-mu mu^k / k!, the replacement of Eq. binomial_probability
   that Sec. 3 proposes for large samples and small rates (mu = m * lambda). */
static double pois_pmf(int64_t k, double mu)
{
    if (k < 0) return 0.0;
    if (mu <= 0.0) return k == 0 ? 1.0 : 0.0;
    return exp((double)k * log(mu) - mu - lgamma((double)k + 1.0));
}

/* P(X > m) for X ~ Poisson(mu): the terms k > m summed directly (no
   difference of probabilities), until they stop mattering. */
static double pois_upper(int64_t m, double mu)
{
    double sum = 0.0;
    for (int64_t k = m + 1;; ++k) {
        double t = pois_pmf(k, mu);
        sum += t;
        if ((double)k > mu && (t == 0.0 || t < sum * 1e-18)) break;
    }
    return sum;
}

static double model_pmf(int64_t k, int64_t m, double lam, int model)
{
    if (model == DDKS_ORACLE_POISSON) return k > m ? 0.0 : pois_pmf(k, (double)m * lam);
    return binom_pmf(k, m, lam);
}

static int64_t floor_div(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

static int64_t ceil_div(int64_t a, int64_t b) /* b > 0 */
{
    return -floor_div(-a, b);
}

/*
 * Probability, under H0 with common rate lambda, that
 * |a/n_p - b/n_q| > num/(n_p*n_q), a ~ Bi(n_p, lambda), b ~ Bi(n_q, lambda):
 * the complement of Sec. 3's p(d <= delta), summed directly over the
 * excluded (a, b) so that no cancellation occurs.
 * |a/n_p - b/n_q| <= num/(n_p n_q)  <=>  |a*n_q - b*n_p| <= num.
 *
 * model DDKS_ORACLE_POISSON: each binomial pmf replaced by the Poisson pmf of
 * mean m*lambda over the same support 0..m (Sec. 3's large-sample
 * approximation, carried through the same sums).  Then
 * p(d <= delta) = Z_a Z_b - excluded with Z the pmf mass on the support, and
 * its complement is (1 - Z_a Z_b) + excluded, where
 * 1 - Z_a Z_b = U_a + U_b - U_a U_b and U = P(Poisson > m) is summed directly.
 */
double ddks_oracle_tail_model(int64_t n_p, int64_t n_q, double lam, uint64_t num, int model)
{
    double *pb = (double *)malloc((size_t)(n_q + 1) * sizeof(double));
    double *below = (double *)malloc((size_t)(n_q + 2) * sizeof(double)); /* below[t] = sum_{b<t} */
    double *above = (double *)malloc((size_t)(n_q + 2) * sizeof(double)); /* above[t] = sum_{b>=t} */
    if (!pb || !below || !above) {
        free(pb);
        free(below);
        free(above);
        return NAN;
    }
    for (int64_t b = 0; b <= n_q; ++b) pb[b] = model_pmf(b, n_q, lam, model);
    below[0] = 0.0;
    for (int64_t t = 1; t <= n_q + 1; ++t) below[t] = below[t - 1] + pb[t - 1];
    above[n_q + 1] = 0.0;
    for (int64_t t = n_q; t >= 0; --t) above[t] = above[t + 1] + pb[t];

    double tail = 0.0;
    for (int64_t a = 0; a <= n_p; ++a) {
        int64_t lo = ceil_div(a * n_q - (int64_t)num, n_p);
        int64_t hi = floor_div(a * n_q + (int64_t)num, n_p);
        if (lo < 0) lo = 0;
        if (hi > n_q) hi = n_q;
        double excluded;
        if (lo > hi) {
            /* no b is close enough: all of b's mass (1 for the binomial) */
            excluded = model == DDKS_ORACLE_POISSON ? below[n_q + 1] : 1.0;
        } else {
            excluded = below[lo] + above[hi + 1];
        }
        tail += model_pmf(a, n_p, lam, model) * excluded;
    }
    if (model == DDKS_ORACLE_POISSON) {
        const double ua = pois_upper(n_p, (double)n_p * lam);
        const double ub = pois_upper(n_q, (double)n_q * lam);
        tail += ua + ub - ua * ub;
    }
    free(pb);
    free(below);
    free(above);
    if (tail < 0.0) tail = 0.0;
    if (tail > 1.0) tail = 1.0;
    return tail;
}

double ddks_oracle_tail(int64_t n_p, int64_t n_q, double lam, uint64_t num)
{
    return ddks_oracle_tail_model(n_p, n_q, lam, num, DDKS_ORACLE_BINOMIAL);
}

/*
 * Analytic significance S of a statistic num/(n_p*n_q) from the membership
 * counts [N][2^d][2] (sample 0 = P, sample 1 = T/Q) over all N = n_p + n_q
 * origins (Eq. ddks_significance):
 *   S = 1 - prod_{j,k} P(delta <= D | lambda_jk),
 *   lambda_jk = (c_Q[k][j] + 1) / (n_q + 2).
 * Computed as S = -expm1(sum log1p(-tail_jk)); tails are cached by the
 * value of c_Q (the only thing lambda depends on).
 */
int ddks_oracle_significance_model(const uint32_t *counts, int64_t n_p, int64_t n_q, int32_t d,
                                   uint64_t num, int model, double *S_out)
{
    if (model != DDKS_ORACLE_BINOMIAL && model != DDKS_ORACLE_POISSON) return ORACLE_EINVAL;
    if (!counts || !S_out || n_p < 1 || n_q < 1 || d < 1 || d > 16) return ORACLE_EINVAL;
    const int64_t N = n_p + n_q;
    const uint32_t bins = (uint32_t)1 << d;
    double *cache = (double *)malloc((size_t)(n_q + 1) * sizeof(double));
    char *have = (char *)calloc((size_t)(n_q + 1), 1);
    if (!cache || !have) {
        free(cache);
        free(have);
        return ORACLE_ENOMEM;
    }
    double log_keep = 0.0;
    int status = ORACLE_OK;
    for (int64_t k = 0; k < N && status == ORACLE_OK; ++k) {
        for (uint32_t j = 0; j < bins; ++j) {
            uint32_t t = counts[((size_t)k * bins + j) * 2 + 1];
            if ((int64_t)t > n_q) { status = ORACLE_EINVAL; break; }
            if (!have[t]) {
                double lam = ((double)t + 1.0) / ((double)n_q + 2.0);
                cache[t] = ddks_oracle_tail_model(n_p, n_q, lam, num, model);
                have[t] = 1;
            }
            log_keep += log1p(-cache[t]);
        }
    }
    free(cache);
    free(have);
    if (status != ORACLE_OK) return status;
    *S_out = -expm1(log_keep);
    return ORACLE_OK;
}

int ddks_oracle_significance(const uint32_t *counts, int64_t n_p, int64_t n_q, int32_t d,
                             uint64_t num, double *S_out)
{
    return ddks_oracle_significance_model(counts, n_p, n_q, d, num, DDKS_ORACLE_BINOMIAL, S_out);
}

/* ------------------------------------------------------------------------- */
/* Counts for a chosen subset of origins (same definition, one origin at a    */
/* time), for checking large inputs at sampled origins.                        */
/* ------------------------------------------------------------------------- */

/*
 * idx[n_idx]: origin indices in P-then-Q order.  counts_out: [n_idx][2^d][2]
 * uint32 (sample 0 = P).
 */
int ddks_oracle_origin_counts(const float *P, int64_t n_p, const float *Q, int64_t n_q, int32_t d,
                              const int64_t *idx, int64_t n_idx, uint32_t *counts_out)
{
    if (!P || !Q || !idx || !counts_out || n_p < 1 || n_q < 1 || d < 1 || d > 16)
        return ORACLE_EINVAL;
    const uint32_t bins = (uint32_t)1 << d;
    chunk_job job;
    memset(&job, 0, sizeof(job));
    job.P = P;
    job.Q = Q;
    job.n_p = n_p;
    job.n_q = n_q;
    job.d = d;
    for (int64_t t = 0; t < n_idx; ++t) {
        int64_t k = idx[t];
        if (k < 0 || k >= n_p + n_q) return ORACLE_EINVAL;
        const float *o = origin_at(&job, k);
        uint32_t *c = counts_out + (size_t)t * bins * 2;
        memset(c, 0, (size_t)bins * 2 * sizeof(uint32_t));
        for (int64_t i = 0; i < n_p; ++i) c[orthant_code(P + i * d, o, d) * 2 + 0] += 1;
        for (int64_t i = 0; i < n_q; ++i) c[orthant_code(Q + i * d, o, d) * 2 + 1] += 1;
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* vdKS: voxel approximation of the statistic (Sec. 2.2.2, Alg. 1)            */
/* ------------------------------------------------------------------------- */

/*
 * Readings of Alg. 1:
 *  - NormalizeData maps each dimension of the pooled points linearly onto
 *    [0, 1]: u = (x - lo) / (hi - lo) with lo, hi the pooled minimum and
 *    maximum (u = 0 where hi == lo);
 *  - IndexFromPoint gives the voxel coordinate v_m = min(V - 1, floor(u_m V))
 *    with V voxels per dimension -- all of it in fp64 (the float inputs
 *    convert exactly, then one subtraction, one division, one product);
 *  - SumOrthants splits the voxels around a filled voxel as Eq. g splits the
 *    points around an origin: bit m of the orthant is [w_m >= u_m], so the
 *    origin voxel lies in its own all-upper orthant;
 *  - the value of an orthant is the absolute difference of the two samples'
 *    proportions in it (Eq. d1), taken exactly in integers as
 *    |c_P n_q - c_Q n_p|, over every filled voxel (either sample).
 * The reported maximiser is the lowest voxel key sum_m v_m V^m, then the
 * lowest orthant code.
 */
typedef struct {
    uint64_t key;
    int sample; /* 0 = P, 1 = Q */
} vox_point;

static int cmp_vox_point(const void *a, const void *b)
{
    const vox_point *x = (const vox_point *)a, *y = (const vox_point *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->sample - y->sample;
}

int ddks_oracle_vdks(const float *P, int64_t n_p, const float *Q, int64_t n_q, int32_t d, int32_t V,
                     uint64_t *num, int64_t *arg_voxel, int32_t *arg_orthant, int64_t *n_filled)
{
    if (!P || !Q || !num || n_p < 1 || n_q < 1 || d < 1 || d > 16 || V < 1) return ORACLE_EINVAL;
    {
        double cells = 1.0;
        for (int m = 0; m < d; ++m) cells *= (double)V;
        if (cells > 4.0e18) return ORACLE_EINVAL; /* keys must fit 63 bits */
    }
    const int64_t N = n_p + n_q;
    double lo[16], hi[16];
    for (int m = 0; m < d; ++m) {
        lo[m] = INFINITY;
        hi[m] = -INFINITY;
    }
    for (int64_t i = 0; i < N; ++i) {
        const float *x = i < n_p ? P + i * d : Q + (i - n_p) * d;
        for (int m = 0; m < d; ++m) {
            double v = (double)x[m];
            if (!isfinite(v)) return ORACLE_EINVAL;
            if (v < lo[m]) lo[m] = v;
            if (v > hi[m]) hi[m] = v;
        }
    }
    vox_point *pts = (vox_point *)malloc((size_t)N * sizeof(vox_point));
    if (!pts) return ORACLE_ENOMEM;
    for (int64_t i = 0; i < N; ++i) {
        const float *x = i < n_p ? P + i * d : Q + (i - n_p) * d;
        uint64_t key = 0, scale = 1;
        for (int m = 0; m < d; ++m) {
            int64_t v = 0;
            if (hi[m] > lo[m]) {
                double u = ((double)x[m] - lo[m]) / (hi[m] - lo[m]);
                v = (int64_t)floor(u * (double)V);
                if (v > V - 1) v = V - 1;
                if (v < 0) v = 0;
            }
            key += (uint64_t)v * scale;
            scale *= (uint64_t)V;
        }
        pts[i].key = key;
        pts[i].sample = i < n_p ? 0 : 1;
    }
    qsort(pts, (size_t)N, sizeof(vox_point), cmp_vox_point);
    /* the filled voxels, in key order, with their counts per sample */
    int64_t M = 0;
    for (int64_t i = 0; i < N; ++i)
        if (i == 0 || pts[i].key != pts[i - 1].key) ++M;
    uint64_t *vk = (uint64_t *)malloc((size_t)M * sizeof(uint64_t));
    int64_t *vc = (int64_t *)calloc((size_t)M * 2, sizeof(int64_t));
    int32_t *coord = (int32_t *)malloc((size_t)M * d * sizeof(int32_t));
    const uint32_t bins = (uint32_t)1 << d;
    int64_t *cp = (int64_t *)malloc(bins * sizeof(int64_t));
    int64_t *cq = (int64_t *)malloc(bins * sizeof(int64_t));
    if (!vk || !vc || !coord || !cp || !cq) {
        free(pts);
        free(vk);
        free(vc);
        free(coord);
        free(cp);
        free(cq);
        return ORACLE_ENOMEM;
    }
    M = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (i == 0 || pts[i].key != pts[i - 1].key) {
            vk[M] = pts[i].key;
            uint64_t k = pts[i].key;
            for (int m = 0; m < d; ++m) {
                coord[M * d + m] = (int32_t)(k % (uint64_t)V);
                k /= (uint64_t)V;
            }
            ++M;
        }
        vc[(M - 1) * 2 + pts[i].sample] += 1;
    }
    uint64_t best = 0;
    int64_t bk = 0;
    int32_t bj = 0;
    int have = 0;
    for (int64_t a = 0; a < M; ++a) {
        memset(cp, 0, bins * sizeof(int64_t));
        memset(cq, 0, bins * sizeof(int64_t));
        for (int64_t b = 0; b < M; ++b) {
            uint32_t code = 0;
            for (int m = 0; m < d; ++m)
                if (coord[b * d + m] >= coord[a * d + m]) code |= 1u << m;
            cp[code] += vc[b * 2];
            cq[code] += vc[b * 2 + 1];
        }
        for (uint32_t j = 0; j < bins; ++j) {
            int64_t diff = cp[j] * n_q - cq[j] * n_p;
            uint64_t sc = (uint64_t)(diff < 0 ? -diff : diff);
            if (!have || sc > best) {
                best = sc;
                bk = (int64_t)vk[a];
                bj = (int32_t)j;
                have = 1;
            }
        }
    }
    *num = best;
    if (arg_voxel) *arg_voxel = bk;
    if (arg_orthant) *arg_orthant = bj;
    if (n_filled) *n_filled = M;
    free(pts);
    free(vk);
    free(vc);
    free(coord);
    free(cp);
    free(cq);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------- */
/* rdKS: radial approximation of the statistic (Sec. 2.2.3, Alg. 2)           */
/* ------------------------------------------------------------------------- */

/*
 * Readings of Alg. 2:
 *  - IdentifyCorners gives the d + 1 corners of the normalised sample space,
 *    the origin and the unit points e_m (the paper's 3-D example), after each
 *    dimension of the pooled points is mapped onto [0, 1] as for vdKS:
 *    u = (x - lo) / (hi - lo), u = 0 where hi == lo;
 *  - the distance from a corner is the squared Euclidean distance (the same
 *    order as the distance), in single precision like the inputs:
 *    s = sum over m ascending of (u_m - c_m)^2, every subtraction, division,
 *    product and sum rounded on its own (no fused multiply-add);
 *  - GetDFromCornerLists is the two-sample KS statistic of the two distance
 *    lists: the largest |F_P(r) - F_T(r)| over the distinct distances r, with
 *    F(r) the fraction of a sample at distance <= r (the printed merge walk
 *    lacks the absolute value and would score in the middle of tied runs);
 *    in integers |c_P(r) n_q - c_Q(r) n_p|;
 *  - D is the largest over the corners; the reported corner is the lowest
 *    maximising one (0 = the origin, m + 1 = e_m).
 */
typedef struct {
    float dist;
    int sample;
} rd_point;

static int cmp_rd_point(const void *a, const void *b)
{
    const rd_point *x = (const rd_point *)a, *y = (const rd_point *)b;
    if (x->dist != y->dist) return x->dist < y->dist ? -1 : 1;
    return x->sample - y->sample;
}

int ddks_oracle_rdks(const float *P, int64_t n_p, const float *Q, int64_t n_q, int32_t d,
                     uint64_t *num, int32_t *arg_corner, uint64_t *per_corner)
{
    if (!P || !Q || !num || n_p < 1 || n_q < 1 || d < 1) return ORACLE_EINVAL;
    const int64_t N = n_p + n_q;
    float *lo = (float *)malloc((size_t)d * sizeof(float));
    float *hi = (float *)malloc((size_t)d * sizeof(float));
    float *u = (float *)malloc((size_t)N * d * sizeof(float));
    rd_point *pts = (rd_point *)malloc((size_t)N * sizeof(rd_point));
    if (!lo || !hi || !u || !pts) {
        free(lo);
        free(hi);
        free(u);
        free(pts);
        return ORACLE_ENOMEM;
    }
    for (int m = 0; m < d; ++m) {
        lo[m] = INFINITY;
        hi[m] = -INFINITY;
    }
    int bad = 0;
    for (int64_t i = 0; i < N; ++i) {
        const float *x = i < n_p ? P + i * d : Q + (i - n_p) * d;
        for (int m = 0; m < d; ++m) {
            if (!isfinite(x[m])) bad = 1;
            if (x[m] < lo[m]) lo[m] = x[m];
            if (x[m] > hi[m]) hi[m] = x[m];
        }
    }
    if (bad) {
        free(lo);
        free(hi);
        free(u);
        free(pts);
        return ORACLE_EINVAL;
    }
    for (int64_t i = 0; i < N; ++i) {
        const float *x = i < n_p ? P + i * d : Q + (i - n_p) * d;
        for (int m = 0; m < d; ++m) {
            volatile float span = hi[m] - lo[m];
            volatile float diff = x[m] - lo[m];
            u[i * d + m] = hi[m] > lo[m] ? diff / span : 0.0f;
        }
    }
    uint64_t best = 0;
    int32_t bc = 0;
    for (int c = 0; c <= d; ++c) {
        for (int64_t i = 0; i < N; ++i) {
            volatile float acc = 0.0f;
            for (int m = 0; m < d; ++m) {
                volatile float t = u[i * d + m] - (c == m + 1 ? 1.0f : 0.0f);
                volatile float sq = t * t;
                acc = acc + sq;
            }
            pts[i].dist = acc;
            pts[i].sample = i < n_p ? 0 : 1;
        }
        qsort(pts, (size_t)N, sizeof(rd_point), cmp_rd_point);
        int64_t cp = 0, cq = 0;
        uint64_t bestc = 0;
        for (int64_t i = 0; i < N; ++i) {
            if (pts[i].sample == 0) ++cp;
            else ++cq;
            if (i + 1 < N && pts[i + 1].dist == pts[i].dist) continue; /* end of a tied run only */
            int64_t diff = cp * n_q - cq * n_p;
            uint64_t sc = (uint64_t)(diff < 0 ? -diff : diff);
            if (sc > bestc) bestc = sc;
        }
        if (per_corner) per_corner[c] = bestc;
        if (c == 0 || bestc > best) {
            best = bestc;
            bc = c;
        }
    }
    *num = best;
    if (arg_corner) *arg_corner = bc;
    free(lo);
    free(hi);
    free(u);
    free(pts);
    return ORACLE_OK;
}
