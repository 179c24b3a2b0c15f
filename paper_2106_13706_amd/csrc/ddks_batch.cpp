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
    int d, B, path, pb;
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
    st = hip_check(c, launch_perm(a.path, a.d, a.pb, zdata, a.n, a.n_p, (const uint64_t *)c->inc.ptr,
                                  a.B, (const uint32_t *)c->obs.ptr, a.nums, s), "permutation launch");
    if (st) return st;
    // number of relabellings at least as extreme as the observed split
    return hip_check(c, launch_count_ge(a.nums, a.B, c->result_dev, s), "count launch");
}

}  // namespace

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
    a.pb = perm_max_group(d);
    a.path = choose_path(c, d, n, flags);
    if (a.path == PATH_R16 && n > 65536) a.path = PATH_F32;  // keep the pipeline free of host syncs
    a.plan = plan_for(c, a.path, d, n, n_p);

    // every buffer the pipeline touches, allocated before any capture
    const int64_t gq = (a.B + a.pb - 1) / a.pb;
    int st = ensure(c, c->z, (size_t)n * d * sizeof(float), "points");
    if (!st && a.B > 0) st = ensure(c, c->inc, (size_t)std::max<int64_t>(gq, 1) * n * (a.pb / 4) * 8, "increments");
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

    if (a.B == 0) {
        st = enqueue_batch(c, a, s);  // observed split only (launch_perm_prepare is a no-op)
    } else {
        const std::vector<uint64_t> key = {
            (uint64_t)n, (uint64_t)n_p, (uint64_t)d, (uint64_t)a.B, (uint64_t)a.path, (uint64_t)a.pb,
            (uint64_t)(uintptr_t)a.srcZ, (uint64_t)(uintptr_t)a.labels, (uint64_t)(uintptr_t)a.nums,
            c->buf_gen, (uint64_t)a.plan.waves, (uint64_t)a.plan.chunks, (uint64_t)(uintptr_t)s};
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
        summary->B = a.B;
        summary->n_ge = a.B > 0 ? r.ge : 0;
        summary->p_value = (1.0 + (double)summary->n_ge) / (1.0 + (double)a.B);
        summary->fraction = a.B > 0 ? (double)summary->n_ge / (double)a.B : 0.0;
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
