/*
 * ddks.h -- C ABI of libddks, an MI355X (gfx950) implementation of the exact
 * d-dimensional two-sample Kolmogorov-Smirnov statistic (ddKS) of Hagen et
 * al., "Accelerated Computation of a High Dimensional Kolmogorov-Smirnov
 * Distance" (arXiv:2106.13706).
 *
 * The statistic (Sec. 2.1, Eq. ddks_tensor_definition): every point of both
 * samples P and Q (the paper's T) is an origin, taken in the order P then Q.
 * Relative to an origin o, a point x lies in the orthant with code
 *     code = sum_{m<d} [x_m >= o_m] * 2^m
 * (Eq. g: IEEE '>=', so -0 == +0 and a tied coordinate goes to the upper
 * side; the origin counts itself).  c_P[o][code] and c_Q[o][code] count the
 * points of each sample per orthant (Eq. membership).  D is the maximum over
 * origins and orthants of |c_P/n_P - c_Q/n_Q| (Eq. d1, normalised by the
 * sample sizes).  The library evaluates it exactly in integers:
 *     num = max |c_P*n_Q - c_Q*n_P|,  den = n_P*n_Q,  D = num/den
 * and reports the first maximiser (lowest origin index, then lowest code).
 *
 * Conventions for every call:
 *   - Return value: DDKS_OK (0) or a negative ddks_status.  On error the
 *     outputs are left unspecified and ddks_last_error() describes it.
 *   - Points are fp32, row-major, n rows of d contiguous values, 1 <= d <= 8.
 *     Values must be finite (the samples live in R^d); -0 is accepted and
 *     compares equal to +0; subnormals are compared exactly.
 *   - Without DDKS_DEVICE_PTRS, point/label/count pointers are host memory;
 *     with it they are device memory on the context's device (for example
 *     a torch tensor's data_ptr()).  Inputs are only borrowed for the call.
 *   - Calls on one context are serialised internally; a context may be used
 *     from several threads.  Different contexts are independent.
 *   - A HIP error poisons the context: every later call returns
 *     DDKS_E_DEVICE.  Destroy it and create another.
 */
#ifndef DDKS_H
#define DDKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ddks_status {
    DDKS_OK = 0,
    DDKS_E_INVALID_ARG = -1,   /* null pointer, d outside [1,8], n < 1, bad label row, ... */
    DDKS_E_NO_DEVICE = -2,     /* no usable gfx950 device with that ordinal */
    DDKS_E_DEVICE = -3,        /* a HIP call failed; the context is poisoned */
    DDKS_E_NOMEM = -4,         /* the request cannot fit the context's device-memory budget */
    DDKS_E_NONFINITE = -5,     /* an input value is NaN or +-inf */
    DDKS_E_AGAIN = -6,         /* serving queue full; retry later */
    DDKS_E_PENDING = -7,       /* serving result not ready within the timeout */
    DDKS_E_UNKNOWN_TICKET = -8,/* ticket never issued, or already collected */
    DDKS_E_NOT_SUPPORTED = -9  /* request outside what this build supports */
} ddks_status;

/* ddks_options.flags and per-call flags */
#define DDKS_DEVICE_PTRS 0x1u   /* pointer arguments are device memory */
#define DDKS_FORCE_F32 0x2u     /* per call: skip the 16-bit rank encoding, compare raw fp32 */
#define DDKS_FORCE_RANK16 0x10u /* per call: use the rank encoding even for small inputs */
#define DDKS_NO_AUTOTUNE 0x4u   /* ctx option: use the built-in launch heuristics only */
#define DDKS_PROFILE_KERNELS 0x8u /* ctx option: time the sweep kernels with HIP events */
#define DDKS_WITH_SIGNIFICANCE 0x20u /* ddks_distance: also compute the analytic significance S */
#define DDKS_SIG_POISSON 0x40u    /* significance: Poisson instead of binomial counts (Sec. 3) */

typedef struct ddks_ctx ddks_ctx;

typedef struct ddks_options {
    int32_t device;            /* HIP device ordinal */
    void *stream;              /* hipStream_t to run on; NULL = a library-owned stream */
    uint64_t mem_budget;       /* device bytes this context may hold; 0 = 90% of free memory */
    uint32_t flags;            /* DDKS_NO_AUTOTUNE */
    int32_t serve_streams;     /* serving: concurrent launch streams (0 = 4) */
    int32_t serve_queue_depth; /* serving: max requests held (admitted or waiting); 0 = 65536 */
    const char *tune_cache;    /* autotuner cache file; NULL = none (in-memory only) */
} ddks_options;

typedef struct ddks_result {
    uint64_t num;             /* max |c_P*n_Q - c_Q*n_P| */
    uint64_t den;             /* n_P*n_Q */
    double D;                 /* (double)num / (double)den, correctly rounded */
    int64_t argmax_origin;    /* index into P then Q of the first maximising origin */
    int32_t argmax_orthant;   /* its lowest maximising orthant code */
    int32_t d;
    int64_t n_p, n_q;
    double S;                 /* analytic significance (DDKS_WITH_SIGNIFICANCE), else -1 */
} ddks_result;

/* Fills *opt with defaults (device 0, library stream, budget 0, no flags). */
void ddks_default_options(ddks_options *opt);

/* Creates a context on opt->device (opt may be NULL for defaults).
 * Caller owns *out and releases it with ddks_destroy.
 * Errors: DDKS_E_INVALID_ARG, DDKS_E_NO_DEVICE, DDKS_E_DEVICE, DDKS_E_NOMEM. */
int ddks_create(const ddks_options *opt, ddks_ctx **out);

/* Drains serving work, frees every device buffer and the context. NULL is a no-op. */
int ddks_destroy(ddks_ctx *ctx);

/*
 * Exact ddKS of P (n_p x d) and Q (n_q x d); Sec. 2.1 Eq. ddks_tensor_definition.
 * counts (nullable): caller-allocated uint32 [n_p+n_q][2^d][2], origin-major
 * in P-then-Q order, sample 0 = P -- the membership matrices M of
 * Eq. membership for both origin sets.  Host memory unless DDKS_DEVICE_PTRS.
 * Synchronous: returns after the result (and counts) are available.  When
 * the result is the call's only host output, the call returns once the
 * final kernel has written it, which may be just before that kernel ends
 * on the context's stream; work queued on that stream still runs after it.
 * flags DDKS_WITH_SIGNIFICANCE: out->S also receives the analytic
 * significance of the result (as ddks_significance, DDKS_SIG_POISSON for the
 * Poisson model), computed on the device from counts that stay there;
 * otherwise out->S = -1.
 * Compares: from N = n_p + n_q = 8192 up to N = 2^22 on 16-bit codes of each
 * dimension's value order (past 65536 distinct values, or past 65536 points
 * in a call replayed as a graph, a dimension is coded coarsely and corrected
 * exactly after the sweep), else on fp32; the result is the same either way.
 * Limits: 1 <= n_p, n_q; n_p + n_q <= 2^31 - 1; 1 <= d <= 8.
 * Errors: DDKS_E_INVALID_ARG, DDKS_E_NONFINITE, DDKS_E_NOMEM, DDKS_E_DEVICE.
 */
int ddks_distance(ddks_ctx *ctx, const float *P, int64_t n_p, const float *Q, int64_t n_q,
                  int32_t d, uint32_t flags, ddks_result *out, uint32_t *counts);

/*
 * ddks_distance for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid hipMalloc, processes whose device
 * memory map must not change once set up): the same result, and the same counts, as ddks_distance, computed
 * in a static 64 MiB device scratch array instead of buffers the call would
 * allocate.  It calls no hipMalloc, hipFree or allocating library routine.
 * P, Q (n_p x d, n_q x d fp32) and counts (nullable, uint32
 * [n_p+n_q][2^d][2]) are device memory on the context's device
 * (DDKS_DEVICE_PTRS is implied).  flags: DDKS_FORCE_F32 / DDKS_FORCE_RANK16
 * as for ddks_distance (rank codes only up to 65536 points, fp32 compares
 * beyond); DDKS_WITH_SIGNIFICANCE is not supported.  Uses the context's launch
 * shape with as many point chunks as the scratch holds; out->S = -1.
 * Every call on one GPU shares that GPU's scratch (held until the process
 * ends): calls on one context are serialised, but calls from different
 * contexts on the same GPU that overlap race.  Synchronous, like
 * ddks_distance.
 * Limits: those of ddks_distance, and the call's buffers (about N*d*4 bytes
 * of points, or the rank tables up to 65536 points, plus the partial counts)
 * within the 64 MiB.
 * Errors: DDKS_E_INVALID_ARG, DDKS_E_NONFINITE, DDKS_E_NOT_SUPPORTED,
 * DDKS_E_NOMEM (the input needs more scratch than the array holds; nothing is
 * launched), DDKS_E_DEVICE (also when the scratch is unavailable).
 */
int ddks_distance_noalloc(ddks_ctx *ctx, const float *P, int64_t n_p, const float *Q, int64_t n_q,
                          int32_t d, uint32_t flags, ddks_result *out, uint32_t *counts);

typedef struct ddks_perm_summary {
    int64_t B;          /* relabellings evaluated */
    uint64_t n_ge;      /* relabellings whose numerator is >= the observed one */
    double p_value;     /* (1 + n_ge) / (1 + B) */
    double fraction;    /* n_ge / B (0 when B == 0) */
} ddks_perm_summary;

/*
 * Permutation test (Sec. 3 and Sec. 4.2): the statistic for B relabellings
 * of the pooled sample Z (n x d).
 * labels: B rows of ceil(n/32) uint32 words; bit (i % 32) of word (i / 32)
 * set means point i is in the first sample.  Every row must hold exactly
 * n_p set bits (and none at or beyond n).  nums_out[B] receives each row's
 * numerator; all rows share den = n_p*(n - n_p).
 * observed (nullable): the statistic of the split "first n_p rows of Z are
 * the first sample", with its argmax, computed in the same launch sequence.
 * summary (nullable): the permutation p-value of the observed statistic;
 * ties count as at least as extreme (the paper gives no formula; this is
 * the add-one estimator).
 * Repeated calls with the same shapes replay one captured hipGraph.
 * Limits: 2 <= n <= 2^31 - 1, 1 <= n_p < n, n_p <= 65535, B >= 0.
 * Errors: as ddks_distance, plus DDKS_E_INVALID_ARG for a malformed row and
 * DDKS_E_NOT_SUPPORTED for n_p > 65535.
 */
int ddks_permutation_batch(ddks_ctx *ctx, const float *Z, int64_t n, int32_t d, int64_t n_p,
                           const uint32_t *labels, int32_t B, uint32_t flags, uint64_t *nums_out,
                           ddks_result *observed, ddks_perm_summary *summary);

/*
 * Permutation p-value of any statistic (Sec. 3 and Sec. 4.2, e.g. vdKS or
 * rdKS recomputed on relabelled samples): from the numerators nums[B] of the
 * relabellings (host memory) and the observed numerator num_obs, all over one
 * shared denominator, fills *summary as ddks_permutation_batch does (ties
 * count as at least as extreme; p = (1 + n_ge) / (1 + B)).  B = 0 gives
 * p = 1 and fraction 0.  Needs no context and no device.
 * Errors: DDKS_E_INVALID_ARG (null summary, B < 0, or null nums with B > 0).
 */
int ddks_perm_summary_of(const uint64_t *nums, int32_t B, uint64_t num_obs,
                         ddks_perm_summary *summary);

/*
 * Analytic significance S of a statistic num/(n_p*n_q) from its membership
 * counts (Sec. 3, Eq. ddks_significance):
 *   S = 1 - prod over origins k and orthants j of P(delta <= D | lambda_kj),
 *   lambda_kj = (c_Q[k][j] + 1) / (n_q + 2)   (Bayes estimator, uniform prior),
 * delta = |a/n_p - b/n_q| with a ~ Bi(n_p, lambda), b ~ Bi(n_q, lambda)
 * (Eq. abs_difference, Eq. binomial_probability).  flags DDKS_SIG_POISSON:
 * the large-sample approximation of Sec. 3, each binomial pmf replaced by the
 * Poisson pmf of the same mean over the same supports 0..n.  Computed on the
 * device in fp64.  counts: [n_p+n_q][2^d][2] as written by ddks_distance
 * (host memory unless DDKS_DEVICE_PTRS).
 * Errors: DDKS_E_INVALID_ARG, DDKS_E_NOMEM, DDKS_E_DEVICE.
 */
int ddks_significance(ddks_ctx *ctx, const uint32_t *counts, int64_t n_p, int64_t n_q, int32_t d,
                      uint64_t num, uint32_t flags, double *S_out);

/*
 * vdKS, the voxel approximation of the statistic (Sec. 2.2.2, Alg. 1): the
 * pooled points normalised per dimension onto [0, 1] (u = (x - lo)/(hi - lo),
 * u = 0 where hi == lo) and binned on a grid of voxels_per_dim^d voxels,
 * coordinate v_m = min(V - 1, floor(u_m V)) evaluated in fp64; around every
 * filled voxel the voxels split into orthants as points do around an origin
 * (Eq. g, >= per coordinate); out->num / out->den is the largest absolute
 * difference of the two samples' proportions in one orthant (Eq. d1).
 * out->argmax_origin receives the lowest maximising voxel's key
 * sum_m v_m V^m (not a point index), argmax_orthant its lowest code, S = -1.
 * n_filled (nullable): the number of voxels holding a point.
 * P, Q as in ddks_distance (host memory unless DDKS_DEVICE_PTRS).
 * Limits: 1 <= d <= 8, 1 <= voxels_per_dim <= 65535, voxels_per_dim^d < 4e18,
 * n_p + n_q < 2^30.
 * Errors: DDKS_E_INVALID_ARG, DDKS_E_NONFINITE, DDKS_E_NOMEM, DDKS_E_DEVICE.
 */
int ddks_vdks(ddks_ctx *ctx, const float *P, int64_t n_p, const float *Q, int64_t n_q, int32_t d,
              int32_t voxels_per_dim, uint32_t flags, ddks_result *out, int64_t *n_filled);

/*
 * rdKS, the radial approximation of the statistic (Sec. 2.2.3, Alg. 2): the
 * pooled points normalised per dimension onto [0, 1] as for ddks_vdks; for
 * each of the d + 1 corners of that space (0 = the origin, m + 1 = the unit
 * point e_m) the two-sample KS statistic of the samples' squared Euclidean
 * distances from the corner (fp32, summed over the dimensions in ascending
 * order, every operation rounded on its own), evaluated at the distinct
 * distances; out->num / out->den is the largest over the corners and
 * out->argmax_origin the lowest maximising corner (argmax_orthant 0, S -1).
 * corner_nums (nullable, host): d + 1 numerators, one per corner.
 * P, Q as in ddks_distance (host memory unless DDKS_DEVICE_PTRS).
 * Limits: 1 <= d <= 4096, (n_p + n_q) (d + 1) <= 2^34.
 * Errors: DDKS_E_INVALID_ARG, DDKS_E_NONFINITE, DDKS_E_NOMEM, DDKS_E_DEVICE.
 */
int ddks_rdks(ddks_ctx *ctx, const float *P, int64_t n_p, const float *Q, int64_t n_q, int32_t d,
              uint32_t flags, ddks_result *out, uint64_t *corner_nums);

/* ---------------------------------------------------------------- serving */

typedef struct ddks_request {
    const float *P; /* host, n_p x d */
    int64_t n_p;
    const float *Q; /* host, n_q x d */
    int64_t n_q;
    int32_t d;
    uint32_t flags; /* 0, or DDKS_WITH_SIGNIFICANCE (optionally | DDKS_SIG_POISSON): the
                       result's S receives the analytic significance (Sec. 3) */
} ddks_request;

typedef struct ddks_serve_stats {
    uint64_t submitted, completed, rejected_again, rejected_nomem;
    uint64_t launches;         /* launches issued (each packs one or more tests) */
    double p50_latency_us;     /* submit -> result ready, over completed requests */
    double p99_latency_us;
    double mean_batch;         /* tests per launch */
    uint64_t resident_bytes;   /* device bytes currently held by admitted requests */
    double busy_us;            /* device time covered by at least one retired launch
                                  (copies, encodings, sweeps, reductions) */
    uint64_t shifted_tests;    /* launched tests swept on shifted 16-bit codes plus
                                  corrections (more than 65536 points) */
} ddks_serve_stats;

/*
 * Submits one test to the context's serving loop (continuous batching:
 * requests that arrive while others run are admitted as device memory and
 * queue slots free up; tests below 16384 points are packed into shared
 * launches, larger ones are swept with the point-chunked plan of a plain
 * call on one of the serve_streams streams; compares on 16-bit codes from
 * 16384 up to 131072 points, else fp32).  The library copies P and Q
 * before returning; the caller may free them at once.  The first submit
 * starts the loop: per stream it holds a 16-bit rank-encoding scratch and a
 * 512 MB partial-count buffer, each only if the budget leaves a 64 MB
 * arena beside it (otherwise that path is not used), and an arena of what
 * the budget then leaves, up to 8 GB, for the admitted requests.
 * Thread-safe.  *ticket identifies the request for ddks_serve_poll.
 * Each test is swept by one block shape whose 16-bit per-sample counters
 * bound a sample to about 8 * 65535 points (4 * 65535 at d = 7, 2 * 65535
 * at d = 8); larger tests get DDKS_E_NOT_SUPPORTED (ddks_distance has no
 * such bound).  A test with DDKS_WITH_SIGNIFICANCE is swept on its own with
 * its membership counts kept in its arena space (N * 2^d * 8 bytes more),
 * and its S is computed on the device after the sweep, as ddks_distance does;
 * other request flags are rejected with DDKS_E_INVALID_ARG.
 * Errors: DDKS_E_AGAIN (queue full), DDKS_E_NOMEM (can never fit the
 * budget), DDKS_E_INVALID_ARG, DDKS_E_NONFINITE, DDKS_E_NOT_SUPPORTED,
 * DDKS_E_DEVICE.
 */
int ddks_serve_submit(ddks_ctx *ctx, const ddks_request *req, uint64_t *ticket);

/*
 * Waits up to timeout_us (0 = just check, < 0 = wait forever) for a
 * submitted test.  On DDKS_OK fills *out (identical to what ddks_distance
 * returns for the same inputs) and releases the ticket.  Thread-safe.
 * Errors: DDKS_E_PENDING, DDKS_E_UNKNOWN_TICKET, DDKS_E_DEVICE.
 */
int ddks_serve_poll(ddks_ctx *ctx, uint64_t ticket, int32_t timeout_us, ddks_result *out);

/* Counters and latency percentiles of the serving loop since the context was created
 * (or since the last reset when reset != 0). */
int ddks_serve_stats_get(ddks_ctx *ctx, ddks_serve_stats *out, int32_t reset);

/* ---------------------------------------------------------------- profiling */

typedef struct ddks_profile {
    uint64_t sweeps;      /* sweep launches timed */
    double sweep_ms;      /* summed device time of the orthant-counting sweep kernel */
    double score_ms;      /* summed device time of the partial-count scoring kernel */
    double batch_ms;      /* summed device time of whole permutation batches (graph launches) */
    uint64_t compares;    /* origin*point*dim compares those sweeps evaluated */
    uint64_t batches;     /* permutation batches timed */
    uint64_t graph_calls; /* ddks_distance calls run as a replayed captured graph */
    uint64_t shifted_calls; /* ddks_distance calls swept on shifted 16-bit codes plus
                               corrections (a dimension with more than 65536 distinct values) */
} ddks_profile;

/*
 * Device-time counters, recorded with HIP events on the context's stream
 * around each kernel launch when the context was created with
 * DDKS_PROFILE_KERNELS (all zero otherwise; shifted_calls is counted either
 * way).  reset != 0 clears them after
 * reading.  Errors: DDKS_E_INVALID_ARG.
 */
int ddks_profile_get(ddks_ctx *ctx, ddks_profile *out, int32_t reset);

/* ---------------------------------------------------------------- misc */

/* Static description of a status code. */
const char *ddks_status_string(int status);

/* Description of the last error on this context (empty string if none). */
const char *ddks_last_error(const ddks_ctx *ctx);

/* Library version string. */
const char *ddks_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DDKS_H */
