// Host side of vdKS (arXiv:2106.13706, Sec. 2.2.2, Alg. 1): ddks_vdks.
#include <math.h>

#include <algorithm>
#include <vector>

#include "ddks_runtime.h"

using namespace ddks;

namespace {

// Filled voxels from which the weighted sweep's shape is tuned (fewer are
// launch-bound: the default shape is as good).
constexpr int64_t VSWEEP_TUNE_MIN = 4096;

// Times every admissible (origin groups per block, waves, chunks) shape of the weighted sweep (the
// encoding, sweep, chunk scoring and reduction: everything that depends on
// the shape) twice and records the fastest for (d, log2 M) in the tuner.
int tune_vsweep(ddks_ctx *c, const uint64_t *keys, const uint64_t *inc, int64_t M, int d, int V, int64_t n_p,
                int64_t n_q, uint32_t *fit, uint32_t *scratch_flags, hipStream_t s, VSweepPlan *best)
{
    const int64_t groups = (M + 63) / 64;
    std::vector<VSweepPlan> cand;
    for (int g : {1, 2})
        for (int w : {4, 8, 16})
            for (int ch : {1, 2, 3, 4, 5, 6, 8, 10, 12, 16}) {
                VSweepPlan p;
                p.waves = w;
                p.chunks = ch;
                p.per_block = g;
                if (!vsweep_plan_ok(p, M, d) || M / ch < (int64_t)w * 64) continue;  // >= 64 voxels per wave
                if (groups * ch * w > 65536 * 4) continue;
                if (vsweep_partial_bytes(M, d, p) > (256ull << 20)) continue;
                cand.push_back(p);
            }
    if (cand.size() < 2) return DDKS_OK;
    size_t pmax = 0;
    for (const VSweepPlan &p : cand) pmax = std::max(pmax, vsweep_partial_bytes(M, d, p));
    int st = pmax ? ensure(c, c->partial, pmax, "voxel partial counts") : DDKS_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!st) st = hip_check(c, hipEventCreate(&e0), "hipEventCreate");
    if (!st) st = hip_check(c, hipEventCreate(&e1), "hipEventCreate");
    float best_ms = 1e30f;
    for (const VSweepPlan &p : cand) {
        float ms_min = 1e30f;
        for (int rep = 0; rep < 2 && !st; ++rep) {
            st = hip_check(c, hipEventRecord(e0, s), "hipEventRecord");
            if (!st)
                st = hip_check(c, launch_vsweep(keys, inc, M, d, V, n_p, n_q, p, (uint32_t *)c->zr.ptr, fit,
                                                c->block_best.ptr, c->partial.ptr, scratch_flags, c->result_dev, s),
                               "voxel sweep launch");
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
            *best = p;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) return st;
    tuner_store_vsweep(c->tuner, d, M, vsweep_uses_bytes(d, V), *best);
    return DDKS_OK;
}

constexpr uint32_t COUNT_PENDING = 0xffffffffu;  // above any count (N < 2^30)

// Waits until the filled-voxel count lands in count_host: polls it, checks
// the stream every 1024 polls (a failed stream ends the wait) and hands a long
// wait over to hipStreamSynchronize, so that it does not hold a host core.
int wait_count(ddks_ctx *c, hipStream_t s)
{
    for (uint32_t spin = 1; spin <= (1u << 16); ++spin) {
        if (__atomic_load_n(c->count_host, __ATOMIC_ACQUIRE) != COUNT_PENDING) return DDKS_OK;
        if ((spin & 1023u) == 0) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) return hip_check(c, q, "stream query");
        }
        __builtin_ia32_pause();
    }
    int st = hip_check(c, hipStreamSynchronize(s), "stream synchronize");
    if (!st && __atomic_load_n(c->count_host, __ATOMIC_ACQUIRE) == COUNT_PENDING)
        st = fail(c, DDKS_E_DEVICE, "the stream finished without the voxel count");
    return st;
}

}  // namespace

extern "C" int ddks_vdks(ddks_ctx *c, const float *P, int64_t n_p, const float *Q, int64_t n_q,
                         int32_t d, int32_t voxels_per_dim, uint32_t flags, ddks_result *out,
                         int64_t *n_filled)
{
    if (!c) return DDKS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->poisoned) return fail(c, DDKS_E_DEVICE, "context poisoned by an earlier device error");
    if (!P || !Q || !out) return fail(c, DDKS_E_INVALID_ARG, "null pointer argument");
    if (d < 1 || d > 8) return fail(c, DDKS_E_INVALID_ARG, "d must be in [1, 8]");
    if (n_p < 1 || n_q < 1) return fail(c, DDKS_E_INVALID_ARG, "each sample needs at least one point");
    const int64_t N = n_p + n_q;
    if (N > 0x3fffffffLL) return fail(c, DDKS_E_INVALID_ARG, "n_p + n_q exceeds 2^30 - 1");
    const int V = voxels_per_dim;
    if (V < 1 || V > 65535) return fail(c, DDKS_E_INVALID_ARG, "voxels_per_dim must be in [1, 65535]");
    if (pow((double)V, (double)d) > 4.0e18)
        return fail(c, DDKS_E_INVALID_ARG, "voxels_per_dim^d must stay below 4e18");
    if (hipSetDevice(c->device) != hipSuccess) return hip_check(c, hipGetLastError(), "hipSetDevice");
    const bool dev = (flags & DDKS_DEVICE_PTRS) != 0;
    hipStream_t s = c->stream;

    const int64_t slots = (int64_t)vdks_table_slots(N);
    const size_t pts = (size_t)N * d * sizeof(float);
    const size_t table = (size_t)slots * (sizeof(uint64_t) + 2 * sizeof(uint32_t));
    const size_t list = (size_t)N * 2 * sizeof(uint64_t);  // keys, increments
    const size_t r16 = (size_t)N * vox_words(d) * sizeof(uint32_t);
    const size_t best = vdks_best_bytes(N);
    int st = ensure(c, c->z, pts, "points");
    const size_t extents = 128 + (size_t)VOX_EXTENT_ROWS * 2 * d * sizeof(uint32_t) + VSWEEP_MAX_CHUNKS * 4;
    if (!st) st = ensure(c, c->vox, table + list + extents, "voxel table");  // + counter and extents
    if (!st) st = ensure(c, c->zr, r16, "voxel encoding");
    if (!st) st = ensure(c, c->block_best, best, "block results");
    if (st) return st;
    float *Z = (float *)c->z.ptr;
    uint64_t *tab_key = (uint64_t *)c->vox.ptr;
    uint32_t *tab_cnt = (uint32_t *)(tab_key + slots);
    uint64_t *keys = (uint64_t *)(tab_cnt + 2 * slots);
    uint64_t *inc = keys + N;
    uint32_t *counter = (uint32_t *)(inc + N);
    uint32_t *mm = counter + 4;     // 2 d words
    uint32_t *part = counter + 32;  // VOX_EXTENT_ROWS x 2 d words
    uint32_t *fit = part + (size_t)VOX_EXTENT_ROWS * 2 * d;  // VSWEEP_MAX_CHUNKS words

    const float *srcP = P, *srcQ = Q;
    if (!dev) {
        st = hip_check(c, hipMemcpyAsync(Z, P, (size_t)n_p * d * sizeof(float), hipMemcpyHostToDevice, s), "H2D P");
        if (!st) st = hip_check(c, hipMemcpyAsync(Z + n_p * d, Q, (size_t)n_q * d * sizeof(float), hipMemcpyHostToDevice, s), "H2D Q");
        if (st) return st;
        srcP = Z;
        srcQ = Z + n_p * d;
    }
    auto front = [&]() {
        int r = hip_check(c, launch_ingest_f32(srcP, n_p, srcQ, n_q, d, Z, c->flags_dev, s), "ingest launch");
        if (!r) r = hip_check(c, launch_vox_front(Z, N, n_p, d, V, mm, part, tab_key, tab_cnt, slots, counter, keys,
                                                 inc, s), "voxel launch");
        return r;
    };
    // with device-resident inputs the launches up to the voxel count form one
    // captured graph, replayed while (inputs, sizes, buffers, stream) match
    const std::vector<uint64_t> fkey = {(uint64_t)(uintptr_t)P, (uint64_t)(uintptr_t)Q, (uint64_t)n_p,
                                        (uint64_t)n_q, (uint64_t)d, (uint64_t)V, c->buf_gen,
                                        (uint64_t)(uintptr_t)s};
    st = dev ? replay_or_capture(c, &c->vdks_graphs, &c->vdks_front_exec, &c->vdks_front_key, fkey, s, front) : front();
    // the number of filled voxels sizes the sweep: copied into a coherent
    // pinned word that the host polls (it lands well before the runtime would
    // report the stream idle), with a sentinel no count can take
    __atomic_store_n(c->count_host, COUNT_PENDING, __ATOMIC_RELEASE);
    if (!st) st = hip_check(c, hipMemcpyAsync(c->count_host, counter, sizeof(uint32_t), hipMemcpyDeviceToHost, s),
                            "D2H voxel count");
    if (!st) st = wait_count(c, s);
    if (st) return st;
    const int64_t M = __atomic_load_n(c->count_host, __ATOMIC_ACQUIRE);
    if (M < 1 || M > N) return fail(c, DDKS_E_DEVICE, "voxel compaction produced an invalid count");
    VSweepPlan plan = vsweep_default_plan(M);
    if (c->force_vsweep.waves) {
        VSweepPlan f = c->force_vsweep;
        f.chunks = (int)std::min<int64_t>(f.chunks, M);
        if (vsweep_plan_ok(f, M, d)) plan = f;
    } else if (!tuner_lookup_vsweep(c->tuner, d, M, vsweep_uses_bytes(d, V), &plan) || !vsweep_plan_ok(plan, M, d)) {
        plan = vsweep_default_plan(M);
        if (c->tuner && !(c->opt_flags & DDKS_NO_AUTOTUNE) && M >= VSWEEP_TUNE_MIN) {
            // time the admissible shapes on this input once per (d, log2 M);
            // the timed runs report into a scratch flags word so that the
            // call's own flags survive them
            st = tune_vsweep(c, keys, inc, M, d, V, n_p, n_q, fit, counter + 2, s, &plan);
            if (st) return st;
        }
    }
    const size_t pb = vsweep_partial_bytes(M, d, plan);
    if (pb && (st = ensure(c, c->partial, pb, "voxel partial counts"))) return st;
    auto back = [&]() {
        return hip_check(c, launch_vsweep(keys, inc, M, d, V, n_p, n_q, plan, (uint32_t *)c->zr.ptr, fit,
                                          c->block_best.ptr, pb ? c->partial.ptr : nullptr, c->flags_dev,
                                          c->result_host, s),
                         "voxel sweep launch");
    };
    if (dev) {
        // the launches after the count: a second graph, keyed also by the
        // count and the shape (a partial-count buffer grown above bumps buf_gen)
        std::vector<uint64_t> bkey = fkey;
        bkey[6] = c->buf_gen;
        bkey.insert(bkey.end(), {(uint64_t)M, (uint64_t)plan.waves, (uint64_t)plan.chunks,
                                 (uint64_t)plan.per_block});
        st = replay_or_capture(c, &c->vdks_graphs, &c->vdks_back_exec, &c->vdks_back_key, bkey, s, back);
    } else {
        st = back();
    }
    if (!st) st = hip_check(c, hipStreamSynchronize(s), "stream synchronize");
    if (st) return st;
    const ResultDev r = *c->result_host;
    if (r.flags & 1u) return fail(c, DDKS_E_NONFINITE, "input contains NaN or infinity");
    out->num = r.num;
    out->den = (uint64_t)n_p * (uint64_t)n_q;
    out->D = (double)r.num / (double)out->den;
    out->argmax_origin = r.origin;
    out->argmax_orthant = r.code;
    out->d = d;
    out->n_p = n_p;
    out->n_q = n_q;
    out->S = -1.0;
    if (n_filled) *n_filled = M;
    return DDKS_OK;
}
