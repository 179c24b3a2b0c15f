// Host side of the permutation test (Sec. 3 / Sec. 4.2 of arXiv:2106.13706):
// ddks_permutation_batch.  The whole device pipeline of one call -- ingest,
// label checks, rank encoding, the observed split's sweep (which also gives
// the label-free totals) and the permutation kernel -- is captured once into
// a hipGraph and replayed while the shapes and buffers stay the same.
#include <string.h>

#include <algorithm>

#include "ddks_runtime.h"

using namespace ddks;

namespace {

struct BatchArgs {
    int64_t n, n_p;
    int d, B, path, pb, waves;
    const float *srcZ;
    const uint32_t *labels;
    unsigned long long *nums;
    SweepPlan plan;
};

// Enqueues the device pipeline of one batch on stream s (eager or captured).
int enqueue_batch(ddks_ctx *c, const BatchArgs &a, hipStream_t s)
{
    float *Z = (float *)c->z.ptr;
    int st = hip_check(c, launch_ingest_f32(a.srcZ, a.n_p, a.srcZ + a.n_p * a.d, a.n - a.n_p, a.d, Z,
                                            c->flags_dev, s), "ingest launch");
    if (st) return st;
    st = hip_check(c, launch_perm_prepare(a.labels, a.n, a.B, a.n_p, a.pb, (uint64_t *)c->inc.ptr,
                                          c->flags_dev, a.nums, s), "label preparation");
    if (st) return st;
    const void *zdata = Z;
    if (a.path == PATH_R16) {
        st = hip_check(c, launch_rank16(Z, a.n, a.d, (uint32_t *)c->zr.ptr, c->rank_scratch.ptr,
                                        c->rank_ctl_dev, s), "rank launch");
        if (st) return st;
        zdata = c->zr.ptr;
    }
    st = run_sweep(c, a.plan, zdata, a.n, a.n_p, a.n - a.n_p, (uint32_t *)c->obs.ptr, c->result_dev, s);
    if (st) return st;
    if (a.B == 0) return DDKS_OK;
    st = hip_check(c, launch_perm(a.path, a.d, a.pb, a.waves, zdata, a.n, a.n_p, (const uint64_t *)c->inc.ptr,
                                  a.B, (const uint32_t *)c->obs.ptr, a.nums, s), "permutation launch");
    if (st) return st;
    // number of relabellings at least as extreme as the observed split
    return hip_check(c, launch_count_ge(a.nums, a.B, c->result_dev, s), "count launch");
}

// Increments buffer of relabellings-per-block pb for B relabellings of n points.
size_t inc_bytes(int64_t n, int B, int pb)
{
    return (size_t)std::max<int64_t>((B + pb - 1) / pb, 1) * n * (pb / 4) * 8;
}

// Times every admissible (waves, relabellings per block) shape of the
// permutation kernel on this call's input, once per (path, d, log2 n) key,
// and records the fastest.  Runs the whole pipeline once eagerly first (the
// kernel reads the observed split's counts); each timed launch is preceded by
// the preparation of its increments and cleared numerators.
int tune_perm(ddks_ctx *c, const BatchArgs &a0, hipStream_t s)
{
    std::vector<std::pair<int, int>> cand;
    for (int pb : {4, 8})
        for (int w : {4, 8, 16})
            if (perm_shape_ok(a0.d, pb, w)) cand.emplace_back(w, pb);
    if (cand.size() < 2) return DDKS_OK;
    int st = enqueue_batch(c, a0, s);
    if (!st) st = hip_check(c, hipStreamSynchronize(s), "stream synchronize");
    if (st) return st;
    const void *zdata = a0.path == PATH_R16 ? c->zr.ptr : c->z.ptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    st = hip_check(c, hipEventCreate(&e0), "hipEventCreate");
    if (!st) st = hip_check(c, hipEventCreate(&e1), "hipEventCreate");
    float best_ms = 1e30f;
    std::pair<int, int> best = {a0.waves, a0.pb};
    for (const auto &wp : cand) {
        float ms_min = 1e30f;
        for (int rep = 0; rep < 2 && !st; ++rep) {
            st = hip_check(c, launch_perm_prepare(a0.labels, a0.n, a0.B, a0.n_p, wp.second, (uint64_t *)c->inc.ptr,
                                                  c->flags_dev, a0.nums, s), "label preparation");
            if (!st) st = hip_check(c, hipEventRecord(e0, s), "hipEventRecord");
            if (!st)
                st = hip_check(c, launch_perm(a0.path, a0.d, wp.second, wp.first, zdata, a0.n, a0.n_p,
                                              (const uint64_t *)c->inc.ptr, a0.B, (const uint32_t *)c->obs.ptr,
                                              a0.nums, s), "permutation launch");
            if (!st) st = hip_check(c, hipEventRecord(e1, s), "hipEventRecord");
            if (!st) st = hip_check(c, hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            if (!st) {
                if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ms_min = std::min(ms_min, ms);
                else (void)hipGetLastError();
            }
        }
        if (!st && ms_min < best_ms) {
            best_ms = ms_min;
            best = wp;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // the label check above may have flagged rows; the call itself reports them
    if (!st) st = hip_check(c, hipMemsetAsync(c->flags_dev, 0, sizeof(uint32_t), s), "flags reset");
    if (!st) st = hip_check(c, hipStreamSynchronize(s), "stream synchronize");
    if (st) return st;
    tuner_store_perm(c->tuner, a0.path, a0.d, a0.n, best.first, best.second);
    return DDKS_OK;
}

}  // namespace

// The permutation p-value of Sec. 3 / Sec. 4.2 from the count of relabellings
// at least as extreme (the paper gives no formula: the add-one estimator).
static void perm_summary_fill(int64_t B, uint64_t n_ge, ddks_perm_summary *out)
{
    out->B = B;
    out->n_ge = n_ge;
    out->p_value = (1.0 + (double)n_ge) / (1.0 + (double)B);
    out->fraction = B > 0 ? (double)n_ge / (double)B : 0.0;
}

extern "C" int ddks_permutation_batch(ddks_ctx *c, const float *Zin, int64_t n, int32_t d,
                                      int64_t n_p, const uint32_t *labels, int32_t B, uint32_t flags,
                                      uint64_t *nums_out, ddks_result *observed,
                                      ddks_perm_summary *summary)
{
    if (!c) return DDKS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->poisoned) return fail(c, DDKS_E_DEVICE, "context poisoned by an earlier device error");
    if (!Zin || (B > 0 && (!labels || !nums_out)))
        return fail(c, DDKS_E_INVALID_ARG, "null pointer argument");
    if (d < 1 || d > 8) return fail(c, DDKS_E_INVALID_ARG, "d must be in [1, 8]");
    if (n < 2 || n_p < 1 || n_p >= n) return fail(c, DDKS_E_INVALID_ARG, "need 1 <= n_p < n");
    if (n > 0x7fffffffLL || B < 0) return fail(c, DDKS_E_INVALID_ARG, "n or B out of range");
    if (n_p > 65535)
        return fail(c, DDKS_E_NOT_SUPPORTED, "permutation batch needs n_p <= 65535");
    if (hipSetDevice(c->device) != hipSuccess) return hip_check(c, hipGetLastError(), "hipSetDevice");
    const bool dev = (flags & DDKS_DEVICE_PTRS) != 0;
    hipStream_t s = c->stream;
    const int64_t words = (n + 31) / 32;
    const size_t bins = (size_t)1 << d;

    BatchArgs a;
    a.n = n;
    a.n_p = n_p;
    a.d = d;
    a.B = std::max<int32_t>(B, 0);
    a.path = choose_path(c, d, n, flags);
    if (a.path == PATH_R16 && n > 65536) a.path = PATH_F32;  // keep the pipeline free of host syncs
    a.plan = plan_for(c, a.path, d, n, n_p);
    // permutation kernel shape: forced (tests), tuned, or the default
    a.pb = perm_max_group(d);
    a.waves = PERM_DEFAULT_WAVES;
    bool tune = false;
    if (c->force_perm_waves && perm_shape_ok(d, c->force_perm_pb, c->force_perm_waves)) {
        a.waves = c->force_perm_waves;
        a.pb = c->force_perm_pb;
    } else if (!tuner_lookup_perm(c->tuner, a.path, d, n, &a.waves, &a.pb)) {
        a.pb = perm_max_group(d);
        a.waves = PERM_DEFAULT_WAVES;
        // tune once per key on sizeable batches (small ones are launch-bound)
        tune = c->tuner && !(c->opt_flags & DDKS_NO_AUTOTUNE) && a.B >= 64 && n >= 4096;
    }

    // every buffer the pipeline touches, allocated before any capture
    int st = ensure(c, c->z, (size_t)n * d * sizeof(float), "points");
    if (!st && a.B > 0)
        st = ensure(c, c->inc, std::max(inc_bytes(n, a.B, 4), inc_bytes(n, a.B, perm_max_group(d))), "increments");
    if (!st) st = ensure(c, c->obs, (size_t)n * bins * 2 * sizeof(uint32_t), "observed counts");
    if (!st && !dev && a.B > 0) st = ensure(c, c->labels, (size_t)a.B * words * sizeof(uint32_t), "labels");
    if (!st && !dev && a.B > 0) st = ensure(c, c->nums, (size_t)a.B * sizeof(uint64_t), "nums");
    if (!st && a.path == PATH_R16) {
        st = ensure(c, c->zr, (size_t)n * point_words(PATH_R16, d) * sizeof(uint32_t), "rank encoding");
        if (!st) st = ensure(c, c->rank_scratch, rank16_scratch_bytes(n, d), "rank scratch");
    }
    if (!st) st = ensure(c, c->block_best, (size_t)a.plan.groups * sizeof(BlockBest), "block results");
    if (!st && a.plan.chunks > 1) st = ensure(c, c->partial, partial_bytes(a.plan), "partial counts");
    if (st) return st;

    a.srcZ = dev ? Zin : (const float *)c->z.ptr;
    a.labels = a.B > 0 ? (dev ? labels : (const uint32_t *)c->labels.ptr) : nullptr;
    a.nums = a.B > 0 ? (unsigned long long *)(dev ? (void *)nums_out : c->nums.ptr) : nullptr;
    if (!dev) {
        st = hip_check(c, hipMemcpyAsync(c->z.ptr, Zin, (size_t)n * d * sizeof(float),
                                         hipMemcpyHostToDevice, s), "H2D points");
        if (!st && a.B > 0)
            st = hip_check(c, hipMemcpyAsync(c->labels.ptr, labels, (size_t)a.B * words * sizeof(uint32_t),
                                             hipMemcpyHostToDevice, s), "H2D labels");
        if (st) return st;
    }

    if (tune && a.B > 0) {
        st = tune_perm(c, a, s);
        if (st) return st;
        if (!tuner_lookup_perm(c->tuner, a.path, d, n, &a.waves, &a.pb)) {
            a.pb = perm_max_group(d);
            a.waves = PERM_DEFAULT_WAVES;
        }
    }
    if (a.B == 0) {
        st = enqueue_batch(c, a, s);  // observed split only (launch_perm_prepare is a no-op)
    } else {
        const std::vector<uint64_t> key = {
            (uint64_t)n, (uint64_t)n_p, (uint64_t)d, (uint64_t)a.B, (uint64_t)a.path, (uint64_t)a.pb,
            (uint64_t)(uintptr_t)a.srcZ, (uint64_t)(uintptr_t)a.labels, (uint64_t)(uintptr_t)a.nums,
            c->buf_gen, (uint64_t)a.plan.waves, (uint64_t)a.plan.chunks, (uint64_t)(uintptr_t)s,
            (uint64_t)a.waves};
        if (c->batch_exec && c->batch_key != key) {
            (void)hipGraphExecDestroy(c->batch_exec);
            c->batch_exec = nullptr;
        }
        if (!c->batch_exec) {
            hipGraph_t g = nullptr;
            c->batch_capturing = true;
            st = hip_check(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
            if (!st) {
                int st2 = enqueue_batch(c, a, s);
                hipError_t e = hipStreamEndCapture(s, &g);
                st = st2 ? st2 : hip_check(c, e, "end capture");
            }
            c->batch_capturing = false;
            if (!st) st = hip_check(c, hipGraphInstantiate(&c->batch_exec, g, nullptr, nullptr, 0),
                                    "graph instantiate");
            if (g) (void)hipGraphDestroy(g);
            if (st) return st;
            c->batch_key = key;
        }
        const bool prof = c->profile;
        if (prof) (void)hipEventRecord(c->ev[0], s);
        st = hip_check(c, hipGraphLaunch(c->batch_exec, s), "graph launch");
        if (!st && prof) {
            (void)hipEventRecord(c->ev[1], s);
            c->graph_pending = true;
        }
    }
    if (st) return st;
    st = hip_check(c, hipMemcpyAsync(c->result_host, c->result_dev, sizeof(ResultDev),
                                     hipMemcpyDeviceToHost, s), "D2H result");
    if (!st && !dev && a.B > 0)
        st = hip_check(c, hipMemcpyAsync(nums_out, c->nums.ptr, (size_t)a.B * sizeof(uint64_t),
                                         hipMemcpyDeviceToHost, s), "D2H nums");
    if (!st) st = hip_check(c, hipStreamSynchronize(s), "stream synchronize");
    if (st) return st;
    if (c->graph_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) c->prof.batch_ms += ms;
        else (void)hipGetLastError();
        c->prof.batches += 1;
        c->graph_pending = false;
    }
    c->ev_pending = false;  // the observed sweep inside a graph is not timed separately
    const ResultDev r = *c->result_host;
    if (r.flags & 2u) return fail(c, DDKS_E_INVALID_ARG, "a label row does not hold exactly n_p first-sample bits");
    if (r.flags & 1u) return fail(c, DDKS_E_NONFINITE, "input contains NaN or infinity");
    if (summary) {
        perm_summary_fill(a.B, a.B > 0 ? r.ge : 0, summary);
    }
    if (observed) {
        observed->num = r.num;
        observed->den = (uint64_t)n_p * (uint64_t)(n - n_p);
        observed->D = (double)r.num / (double)observed->den;
        observed->argmax_origin = r.origin;
        observed->argmax_orthant = r.code;
        observed->d = d;
        observed->n_p = n_p;
        observed->n_q = n - n_p;
        observed->S = -1.0;
    }
    return DDKS_OK;
}

extern "C" int ddks_perm_summary_of(const uint64_t *nums, int32_t B, uint64_t num_obs,
                                    ddks_perm_summary *out)
{
    if (!out || B < 0 || (B > 0 && !nums)) return DDKS_E_INVALID_ARG;
    uint64_t ge = 0;
    for (int32_t b = 0; b < B; ++b) ge += nums[b] >= num_obs ? 1 : 0;
    perm_summary_fill(B, ge, out);
    return DDKS_OK;
}
