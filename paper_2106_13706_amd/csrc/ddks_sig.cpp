// Host side of the analytic significance (arXiv:2106.13706, Sec. 3,
// Eq. ddks_significance): ddks_significance.
#include <algorithm>

#include "ddks_runtime.h"

using namespace ddks;

extern "C" int ddks_significance(ddks_ctx *c, const uint32_t *counts, int64_t n_p, int64_t n_q,
                                 int32_t d, uint64_t num, uint32_t flags, double *S_out)
{
    if (!c) return DDKS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->poisoned) return fail(c, DDKS_E_DEVICE, "context poisoned by an earlier device error");
    if (!counts || !S_out) return fail(c, DDKS_E_INVALID_ARG, "null pointer argument");
    if (d < 1 || d > 8) return fail(c, DDKS_E_INVALID_ARG, "d must be in [1, 8]");
    if (n_p < 1 || n_q < 1 || n_p + n_q > 0x7fffffffLL)
        return fail(c, DDKS_E_INVALID_ARG, "sample sizes out of range");
    if (num > (uint64_t)n_p * (uint64_t)n_q)
        return fail(c, DDKS_E_INVALID_ARG, "num exceeds n_p * n_q");
    if (hipSetDevice(c->device) != hipSuccess) return hip_check(c, hipGetLastError(), "hipSetDevice");
    const bool dev = (flags & DDKS_DEVICE_PTRS) != 0;
    hipStream_t s = c->stream;
    const int64_t N = n_p + n_q;
    const size_t cbytes = (size_t)N * ((size_t)1 << d) * 2 * sizeof(uint32_t);
    const int model = (flags & DDKS_SIG_POISSON) ? SIG_MODEL_POISSON : SIG_MODEL_BINOMIAL;
    const int rows = significance_rows(n_q, model);
    int st = ensure(c, c->sig, significance_scratch_bytes(n_p, n_q, rows, model) + 64, "significance scratch");
    if (st) return st;
    const uint32_t *cd = counts;
    if (!dev) {
        st = ensure(c, c->counts, cbytes, "counts");
        if (st) return st;
        st = hip_check(c, hipMemcpyAsync(c->counts.ptr, counts, cbytes, hipMemcpyHostToDevice, s), "H2D counts");
        if (st) return st;
        cd = (const uint32_t *)c->counts.ptr;
    }
    double *Sdev = (double *)((char *)c->sig.ptr + significance_scratch_bytes(n_p, n_q, rows, model));
    st = hip_check(c, launch_significance(cd, N, d, n_p, n_q, num, nullptr, model, c->sig.ptr, rows,
                                          c->flags_dev, Sdev, s), "significance launch");
    if (st) return st;
    double S = 0.0;
    uint32_t fl = 0;
    st = hip_check(c, hipMemcpyAsync(c->sig_host, Sdev, sizeof(double), hipMemcpyDeviceToHost, s), "D2H S");
    if (!st) st = hip_check(c, hipMemcpyAsync(c->sig_host + 1, c->flags_dev, sizeof(uint32_t),
                                              hipMemcpyDeviceToHost, s), "D2H flags");
    if (!st) st = hip_check(c, hipStreamSynchronize(s), "stream synchronize");
    if (st) return st;
    S = c->sig_host[0];
    fl = *(const uint32_t *)(c->sig_host + 1);
    if (fl) {
        // clear the flags word for the next call (the sweeps clear it on their own)
        (void)hipMemsetAsync(c->flags_dev, 0, sizeof(uint32_t), s);
        (void)hipStreamSynchronize(s);
        if (fl & 4u) return fail(c, DDKS_E_INVALID_ARG, "a second-sample count exceeds n_q");
    }
    *S_out = S;
    return DDKS_OK;
}
