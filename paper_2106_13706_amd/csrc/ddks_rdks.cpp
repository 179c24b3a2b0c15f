// Host side of rdKS (arXiv:2106.13706, Sec. 2.2.3, Alg. 2): ddks_rdks.
#include "ddks_runtime.h"

using namespace ddks;

extern "C" int ddks_rdks(ddks_ctx *c, const float *P, int64_t n_p, const float *Q, int64_t n_q, int32_t d,
                         uint32_t flags, ddks_result *out, uint64_t *corner_nums)
{
    if (!c) return DDKS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->poisoned) return fail(c, DDKS_E_DEVICE, "context poisoned by an earlier device error");
    if (!P || !Q || !out) return fail(c, DDKS_E_INVALID_ARG, "null pointer argument");
    if (d < 1 || d > 4096) return fail(c, DDKS_E_INVALID_ARG, "d must be in [1, 4096]");
    if (n_p < 1 || n_q < 1) return fail(c, DDKS_E_INVALID_ARG, "each sample needs at least one point");
    const int64_t N = n_p + n_q;
    if (N > 0x7fffffffLL || N * (int64_t)(d + 1) > (1LL << 34))
        return fail(c, DDKS_E_INVALID_ARG, "(n_p + n_q) * (d + 1) exceeds 2^34");
    if (hipSetDevice(c->device) != hipSuccess) return hip_check(c, hipGetLastError(), "hipSetDevice");
    const bool dev = (flags & DDKS_DEVICE_PTRS) != 0;
    hipStream_t s = c->stream;
    const int C = d + 1;

    int st = ensure(c, c->z, (size_t)N * d * sizeof(float), "points");
    if (!st) st = ensure(c, c->rank_scratch, rdks_scratch_bytes(N, d), "rdks scratch");
    if (!st) st = ensure(c, c->nums, (size_t)C * sizeof(uint64_t), "corner numerators");
    if (st) return st;
    float *Z = (float *)c->z.ptr;
    const float *srcP = P, *srcQ = Q;
    if (!dev) {
        st = hip_check(c, hipMemcpyAsync(Z, P, (size_t)n_p * d * sizeof(float), hipMemcpyHostToDevice, s), "H2D P");
        if (!st) st = hip_check(c, hipMemcpyAsync(Z + n_p * d, Q, (size_t)n_q * d * sizeof(float), hipMemcpyHostToDevice, s), "H2D Q");
        if (st) return st;
        srcP = Z;
        srcQ = Z + n_p * d;
    }
    unsigned long long *cn = (unsigned long long *)c->nums.ptr;
    auto enqueue = [&]() {
        int r = hip_check(c, launch_ingest_f32(srcP, n_p, srcQ, n_q, d, Z, c->flags_dev, s), "ingest launch");
        if (!r) r = hip_check(c, launch_rdks(Z, N, n_p, d, c->rank_scratch.ptr, cn, c->flags_dev, c->result_host, s),
                              "rdks launch");
        return r;
    };
    if (dev) {
        // device-resident inputs: the call's launches form one captured graph,
        // replayed while (inputs, sizes, buffers, stream) match
        const std::vector<uint64_t> key = {(uint64_t)(uintptr_t)P, (uint64_t)(uintptr_t)Q, (uint64_t)n_p,
                                           (uint64_t)n_q, (uint64_t)d, c->buf_gen, (uint64_t)(uintptr_t)s};
        st = replay_or_capture(c, &c->rdks_graphs, &c->rdks_exec, &c->rdks_key, key, s, enqueue);
    } else {
        st = enqueue();
    }
    if (!st && corner_nums)
        st = hip_check(c, hipMemcpyAsync(corner_nums, cn, (size_t)C * sizeof(uint64_t), hipMemcpyDeviceToHost, s),
                       "D2H corner numerators");
    if (!st) st = hip_check(c, hipStreamSynchronize(s), "stream synchronize");
    if (st) return st;
    const ResultDev r = *c->result_host;
    if (r.flags & 1u) return fail(c, DDKS_E_NONFINITE, "input contains NaN or infinity");
    out->num = r.num;
    out->den = (uint64_t)n_p * (uint64_t)n_q;
    out->D = (double)r.num / (double)out->den;
    out->argmax_origin = r.origin;
    out->argmax_orthant = 0;
    out->d = d;
    out->n_p = n_p;
    out->n_q = n_q;
    out->S = -1.0;
    return DDKS_OK;
}
