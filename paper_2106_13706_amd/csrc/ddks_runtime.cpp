// libddks host runtime: context, device buffers under a budget, and the
// single-test entry point ddks_distance (arXiv:2106.13706, Sec. 2.1
// Eq. ddks_tensor_definition).
#include "ddks_runtime.h"

#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <new>

using namespace ddks;

namespace ddks {

int fail(ddks_ctx *c, int status, const std::string &msg)
{
    if (c) c->last_error = msg;
    return status;
}

bool fault_injected(ddks_ctx *c, int site)
{
    if (!c || c->fault_site == FAULT_NONE || c->fault_site != site) return false;
    return c->fault_countdown.fetch_sub(1) == 1;
}

static void parse_fault_injection(ddks_ctx *c)
{
    const char *e = getenv("DDKS_FAULT_INJECT");
    if (!e) return;
    static const struct {
        const char *name;
        int site;
    } sites[] = {{"call:", FAULT_CALL}, {"serve_launch:", FAULT_SERVE_LAUNCH}, {"serve_event:", FAULT_SERVE_EVENT}};
    for (const auto &x : sites) {
        const size_t n = strlen(x.name);
        if (strncmp(e, x.name, n) == 0) {
            const long long k = atoll(e + n);
            if (k >= 1) {
                c->fault_site = x.site;
                c->fault_countdown = k;
            }
        }
    }
}

int hip_check(ddks_ctx *c, hipError_t e, const char *what)
{
    if (e == hipSuccess) return DDKS_OK;
    if (c) {
        c->poisoned = true;
        c->last_error = std::string(what) + ": " + hipGetErrorString(e);
    }
    return DDKS_E_DEVICE;
}

int ensure(ddks_ctx *c, DevBuf &b, size_t bytes, const char *what)
{
    // 256 bytes of slack past every buffer: the sweep's wave-uniform point
    // reads are merged into wide scalar loads, which may run up to 128 bytes
    // past the last point they use.
    bytes += 256;
    if (b.bytes >= bytes) return DDKS_OK;
    // grow geometrically to limit reallocations across calls of rising size
    size_t want = std::max(bytes, b.bytes + b.bytes / 2);
    want = (want + 4095) & ~(size_t)4095;
    uint64_t others = c->used.load() - b.bytes;
    if (others + want > c->budget) {
        want = (bytes + 4095) & ~(size_t)4095;
        if (others + want > c->budget)
            return fail(c, DDKS_E_NOMEM,
                        std::string("device memory budget exceeded allocating ") + what);
    }
    if (b.ptr) {
        hipError_t e = hipFree(b.ptr);
        c->used -= b.bytes;
        b.ptr = nullptr;
        b.bytes = 0;
        if (e != hipSuccess) return hip_check(c, e, "hipFree");
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return fail(c, DDKS_E_NOMEM, std::string("hipMalloc out of memory for ") + what);
    }
    if (e != hipSuccess) return hip_check(c, e, "hipMalloc");
    b.ptr = p;
    b.bytes = want;
    c->used += want;
    c->buf_gen += 1;
    return DDKS_OK;
}

void release(ddks_ctx *c, DevBuf &b)
{
    if (b.ptr) {
        (void)hipFree(b.ptr);
        c->used -= b.bytes;
    }
    b.ptr = nullptr;
    b.bytes = 0;
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool plan_complete(SweepPlan &p, int64_t N, int64_t n_p)
{
    if (p.waves != 1 && p.waves != 2 && p.waves != 4 && p.waves != 8 && p.waves != 12 &&
        p.waves != 16)
        return false;
    p.groups = cdiv(N, 64);
    p.chunks = std::max<int64_t>(1, std::min<int64_t>({p.chunks, N, 65535}));
    p.chunk_len = cdiv(N, p.chunks);
    p.hists = sweep_hists(p.d, p.waves, p.chunk_len, n_p, N - n_p);
    return p.hists > 0;
}

SweepPlan plan_for(ddks_ctx *c, int path, int d, int64_t N, int64_t n_p)
{
    SweepPlan p;
    p.path = path;
    p.d = d;
    if (c && c->tuner && !(c->opt_flags & DDKS_NO_AUTOTUNE) && tuner_lookup(c->tuner, path, d, N, &p)) {
        p.path = path;
        p.d = d;
        if (plan_complete(p, N, n_p)) return p;
    }
    // 4 waves per block; 8 from d = 4 on, where LDS (the 68 KB pair table at
    // d = 4, 2^d 256-byte bins above) admits few blocks per CU.  At d = 4 the
    // table admits two blocks per CU whatever their size, so from 6144 points
    // on the blocks take 12 waves.  From 32768 points on every d takes 16: two
    // such blocks fill a CU's 8 waves per SIMD (the sweep's 80 SGPRs allow
    // that many).  Kernel times with the default chunks, 8 / 12 / 16 waves, at
    // 32768 and 131072 points: d = 4 168 / 162 / 157 us and 2.80 / 2.51 / 2.39
    // ms; d = 6 251 / 251 / 244 us and 3.72 / 3.59 / 3.49 ms; d = 8 313 / 298 /
    // 289 us and 6.20 / 5.48 / 5.26 ms; d = 2, 3, 5, 7 alike or within 1%.
    p.waves = d >= 4 ? 8 : 4;
    if (d == 4 && N >= 6144) p.waves = 12;
    if (N >= 32768) p.waves = 16;
    if (c && (c->force_waves == 1 || c->force_waves == 2 || c->force_waves == 4 ||
              c->force_waves == 8 || c->force_waves == 12 || c->force_waves == 16))
        p.waves = c->force_waves;
    p.groups = cdiv(N, 64);
    // about 8 waves per SIMD over the 1024 SIMDs (16 at d = 5..7, where more
    // point chunks measured faster, and with 16-wave blocks at d = 4, whose
    // 2 x 20000 sweep measured 214 us in two chunks against 256 in one; 2 at
    // d = 8, whose 256-bin partial counts cost more than the extra waves
    // gain), each sweeping >= 128 points (a longer chain of point blocks per
    // wave is latency-bound at small N)
    const int64_t target_waves = d == 8 ? 2048 : (d >= 5 || p.waves == 16 ? 16384 : 8192);
    int64_t chunks = cdiv(target_waves, p.groups * p.waves);
    int64_t max_chunks = std::max<int64_t>(1, N / ((int64_t)p.waves * 128));
    chunks = std::min(chunks, max_chunks);
    if (c && c->force_chunks > 0) chunks = c->force_chunks;
    p.chunks = chunks;
    // more chunks until the histograms of a block fit (16-bit counters, LDS)
    while (!plan_complete(p, N, n_p) && p.chunks < std::min<int64_t>(N, 65535)) ++p.chunks;
    return p;
}

int choose_path(ddks_ctx * /*c*/, int /*d*/, int64_t N, uint32_t flags)
{
    if (flags & DDKS_FORCE_F32) return PATH_F32;
    if (flags & DDKS_FORCE_RANK16) return PATH_R16;
    // The encoding costs a few small launches; it pays once the O(N^2) sweep
    // dominates.
    return N >= 8192 ? PATH_R16 : PATH_F32;
}

int rank_position_shift(int64_t N)
{
    int sh = 0;
    while (sh <= RANK_MAX_SHIFT && (uint64_t)N > (65536ull << sh)) ++sh;
    return sh <= RANK_MAX_SHIFT ? sh : -1;
}

uint32_t shifts_all(int shift, int d)
{
    uint32_t packed = 0;
    for (int m = 0; m < d; ++m) packed |= (uint32_t)shift << (4 * m);
    return packed;
}

int encode_rank16(ddks_ctx *c, int64_t N, int d, bool *ok, uint32_t *shifts)
{
    *ok = false;
    *shifts = 0;
    const int pw = point_words(PATH_R16, d);
    int st = ensure(c, c->zr, (size_t)N * pw * sizeof(uint32_t), "rank encoding");
    if (st) return st;
    st = ensure(c, c->rank_scratch, rank16_scratch_bytes(N, d), "rank scratch");
    if (st) return st;
    st = hip_check(c, launch_rank16((const float *)c->z.ptr, N, d, (uint32_t *)c->zr.ptr,
                                    c->rank_scratch.ptr, c->rank_ctl_dev, c->stream),
                   "rank launch");
    if (st) return st;
    if (N <= 65536) {
        *ok = true;  // at most N distinct values per dimension
        return DDKS_OK;
    }
    st = hip_check(c, hipMemcpyAsync(c->rank_distinct_host, c->rank_ctl_dev, (size_t)(1 + d) * sizeof(uint32_t),
                                     hipMemcpyDeviceToHost, c->stream), "D2H distinct counts");
    if (!st) st = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
    if (st) return st;
    // a dimension whose dense ranks fit keeps them (nothing to correct there)
    uint32_t packed = 0;
    for (int m = 0; m < d; ++m) {
        if (c->rank_distinct_host[1 + m] <= 65536u) continue;
        const int sh = rank_position_shift(N);
        if (sh < 0) return DDKS_OK;  // fp32 compares
        packed |= (uint32_t)sh << (4 * m);
    }
    if (packed) {
        st = hip_check(c, launch_rank16_shift(N, d, (uint32_t *)c->zr.ptr, c->rank_scratch.ptr, packed, c->stream),
                       "rank shift launch");
        if (st) return st;
    }
    *ok = true;
    *shifts = packed;
    return DDKS_OK;
}

int run_sweep(ddks_ctx *c, const SweepPlan &plan, const void *zdata, int64_t N, int64_t n_p,
              int64_t n_q, uint32_t *counts_dev, ResultDev *res, hipStream_t s, uint32_t shifts)
{
    if (shifts && plan.chunks < 2) return fail(c, DDKS_E_DEVICE, "shifted ranks need a chunked plan");
    int st = ensure(c, c->block_best, (size_t)plan.groups * sizeof(BlockBest), "block results");
    if (st) return st;
    void *partial = nullptr;
    if (plan.chunks > 1) {
        st = ensure(c, c->partial, partial_bytes(plan), "partial counts");
        if (st) return st;
        partial = c->partial.ptr;
    }
    const bool prof = c->profile && s == c->stream && !c->batch_capturing;
    return sweep_into(c, plan, zdata, N, n_p, n_q, counts_dev, res, s, shifts, (BlockBest *)c->block_best.ptr,
                      partial, shifts ? c->rank_scratch.ptr : nullptr, prof);
}

int sweep_into(ddks_ctx *c, const SweepPlan &plan, const void *zdata, int64_t N, int64_t n_p, int64_t n_q,
               uint32_t *counts_dev, ResultDev *res, hipStream_t s, uint32_t shifts, BlockBest *bb,
               void *partial, void *rank_scratch, bool prof)
{
    if (shifts && plan.chunks < 2) return fail(c, DDKS_E_DEVICE, "shifted ranks need a chunked plan");
    if (prof) (void)hipEventRecord(c->ev[0], s);
    int st = hip_check(c, launch_sweep(plan, zdata, N, n_p, n_q, partial, bb, counts_dev, s), "sweep launch");
    if (st) return st;
    if (prof) (void)hipEventRecord(c->ev[1], s);
    if (shifts) {
        st = hip_check(c, launch_rank_fixups(plan, rank16_tables(rank_scratch, N, plan.d), N, n_p, shifts,
                                             partial, s),
                       "rank fixup launch");
        if (st) return st;
    }
    if (plan.chunks > 1) {
        st = hip_check(c, launch_score(plan, N, n_p, n_q, partial, bb, counts_dev, s), "score launch");
        if (st) return st;
        if (prof) (void)hipEventRecord(c->ev[2], s);
    }
    if (prof) {
        c->ev_pending = true;
        c->ev_score = plan.chunks > 1;
        c->ev_compares = N * N * plan.d;
    }
    return hip_check(c, launch_reduce(bb, plan.groups, c->flags_dev, res, s,
                                      res == c->result_host ? c->done_host : nullptr),
                     "reduce launch");
}

void profile_collect(ddks_ctx *c)
{
    if (!c->ev_pending) return;
    float ms = 0.f;
    // a failed query must not leave its error for the next launch check
    if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) c->prof.sweep_ms += ms;
    else (void)hipGetLastError();
    if (c->ev_score) {
        if (hipEventElapsedTime(&ms, c->ev[1], c->ev[2]) == hipSuccess) c->prof.score_ms += ms;
        else (void)hipGetLastError();
    }
    c->prof.sweeps += 1;
    c->prof.compares += (uint64_t)c->ev_compares;
    c->ev_pending = false;
}

}  // namespace ddks

// ==================================================================== C ABI

// Everything one single-test call enqueues after its buffers exist.
struct DistArgs {
    const float *P, *Q;
    int64_t n_p, n_q;
    int d, path;
    uint32_t shifts;  // rank path past 65536 points: shifted codes in every dimension
    uint32_t *counts;
    SweepPlan plan;
};

// Allocates (outside any capture) every buffer enqueue_distance uses.
static int prepare_distance(ddks_ctx *c, const DistArgs &a)
{
    const int64_t N = a.n_p + a.n_q;
    int st = DDKS_OK;
    if (a.path == PATH_R16) {
        st = ensure(c, c->zr, (size_t)N * point_words(PATH_R16, a.d) * sizeof(uint32_t), "rank encoding");
        if (!st) st = ensure(c, c->rank_scratch, rank16_scratch_bytes(N, a.d), "rank scratch");
    }
    if (!st) st = ensure(c, c->block_best, (size_t)a.plan.groups * sizeof(BlockBest), "block results");
    if (!st && a.plan.chunks > 1) st = ensure(c, c->partial, partial_bytes(a.plan), "partial counts");
    return st;
}

// Ingest, rank encoding (no host decision: past 65536 points every dimension
// takes the shifted codes) and, if with_sweep, the sweep of device-resident P
// and Q; the result lands in the pinned c->result_host.  Up to 65536 points
// on the rank path the encoding reads P and Q itself and there is no ingest.
static int enqueue_distance(ddks_ctx *c, const DistArgs &a, hipStream_t s, bool with_sweep)
{
    const int64_t N = a.n_p + a.n_q;
    float *Z = (float *)c->z.ptr;
    int st = DDKS_OK;
    if (a.path == PATH_R16 && N <= 65536) {
        // the sweep reads only the encoding, which reads P and Q itself (and
        // checks their values), so no ingested copy is made
        st = hip_check(c, launch_rank16_pq(a.P, a.n_p, a.Q, a.n_q, a.d, (uint32_t *)c->zr.ptr,
                                           c->rank_scratch.ptr, c->flags_dev, s), "rank launch");
        if (st) return st;
        if (!with_sweep) return DDKS_OK;
        return run_sweep(c, a.plan, c->zr.ptr, N, a.n_p, a.n_q, a.counts, c->result_host, s, 0);
    }
    st = hip_check(c, launch_ingest_f32(a.P, a.n_p, a.Q, a.n_q, a.d, Z, c->flags_dev, s), "ingest launch");
    if (st) return st;
    const void *zdata = Z;
    if (a.path == PATH_R16) {
        st = hip_check(c, launch_rank16(Z, N, a.d, (uint32_t *)c->zr.ptr, c->rank_scratch.ptr,
                                        c->rank_ctl_dev, s), "rank launch");
        if (!st && a.shifts)
            st = hip_check(c, launch_rank16_shift(N, a.d, (uint32_t *)c->zr.ptr, c->rank_scratch.ptr, a.shifts, s),
                           "rank shift launch");
        if (st) return st;
        zdata = c->zr.ptr;
    }
    if (!with_sweep) return DDKS_OK;
    return run_sweep(c, a.plan, zdata, N, a.n_p, a.n_q, a.counts, c->result_host, s, a.shifts);
}

// Waits for the call's work, copies host counts if asked, fills *out.
// Waits for a call whose only output is the result the reduction writes to
// result_host: polls the done word the reduction sets after it, which returns
// as soon as that write lands rather than when the runtime has processed the
// stream's completion.  Checks the stream every 1024 polls (a failed stream
// ends the wait) and hands a long call over to hipStreamSynchronize, so that
// it does not hold a host core.
static int wait_result(ddks_ctx *c, hipStream_t s)
{
    for (uint32_t spin = 1; spin <= (1u << 16); ++spin) {
        if (__atomic_load_n(c->done_host, __ATOMIC_ACQUIRE) == 1u) return DDKS_OK;
        if ((spin & 1023u) == 0) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) return hip_check(c, q, "stream query");
        }
        __builtin_ia32_pause();
    }
    int st = hip_check(c, hipStreamSynchronize(s), "stream synchronize");
    if (!st && __atomic_load_n(c->done_host, __ATOMIC_ACQUIRE) != 1u)
        st = fail(c, DDKS_E_DEVICE, "the stream finished without a result");
    return st;
}

static int finish_distance(ddks_ctx *c, int64_t n_p, int64_t n_q, int d, ddks_result *out,
                           uint32_t *counts_host, const uint32_t *counts_dev, size_t counts_bytes,
                           bool with_S)
{
    hipStream_t s = c->stream;
    int st = DDKS_OK;
    if (counts_host)
        st = hip_check(c, hipMemcpyAsync(counts_host, counts_dev, counts_bytes, hipMemcpyDeviceToHost, s),
                       "D2H counts");
    if (st) return st;
    // Timing events, a copy of the counts or the significance still need the
    // whole stream; otherwise the result word is enough.
    st = (counts_host || with_S || c->ev_pending) ? hip_check(c, hipStreamSynchronize(s), "stream synchronize")
                                                  : wait_result(c, s);
    if (st) return st;
    profile_collect(c);
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
    out->S = with_S ? c->sig_host[0] : -1.0;
    return DDKS_OK;
}

// ------------------------------------------------ scratch of the no-allocation call
// ddks_distance_noalloc works in this array instead of buffers it would
// allocate: one copy per GPU the library runs on, held until the process
// ends.  In host code `scratch` names a host-side stand-in, not device
// memory: the per-device address comes from hipGetSymbolAddress at context
// creation, and only that address is handed to kernels.  Calls on one GPU
// share its copy, so calls that overlap on one GPU (from different contexts)
// race; the kernels write every part of it they later read, so nothing needs
// to start at zero.
static constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// With c->device current: looks up this device's copy of `scratch` once.
static void noalloc_setup(ddks_ctx *c)
{
    if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[c->device]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();  // the no-allocation call reports it; other calls are unaffected
        return;
    }
    g_scratch_ptr[c->device] = p;
}

static void *noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of one call's buffers in the scratch.
struct NoallocLayout {
    size_t pts = 0, rank = 0, bb = 0, partial = 0, total = 0;
};

static NoallocLayout noalloc_layout(const SweepPlan &p, int64_t N, int d)
{
    NoallocLayout L;
    size_t off = 0;
    L.pts = off;
    off += al256((size_t)N * point_words(p.path, d) * sizeof(uint32_t));
    L.rank = off;
    if (p.path == PATH_R16) off += al256(rank16_scratch_bytes(N, d));
    L.bb = off;
    off += al256((size_t)p.groups * sizeof(BlockBest));
    L.partial = off;
    if (p.chunks > 1) off += al256(partial_bytes(p));
    L.total = off + 256;  // the sweep's wide point loads may read up to 128 bytes past the points
    return L;
}

extern "C" {

const char *ddks_version(void) { return "libddks 0.1 (gfx950)"; }

const char *ddks_status_string(int s)
{
    switch (s) {
    case DDKS_OK: return "ok";
    case DDKS_E_INVALID_ARG: return "invalid argument";
    case DDKS_E_NO_DEVICE: return "no usable device";
    case DDKS_E_DEVICE: return "device error";
    case DDKS_E_NOMEM: return "out of device memory budget";
    case DDKS_E_NONFINITE: return "non-finite input value";
    case DDKS_E_AGAIN: return "queue full, try again";
    case DDKS_E_PENDING: return "result pending";
    case DDKS_E_UNKNOWN_TICKET: return "unknown ticket";
    case DDKS_E_NOT_SUPPORTED: return "not supported";
    default: return "unknown status";
    }
}

const char *ddks_last_error(const ddks_ctx *c) { return c ? c->last_error.c_str() : ""; }

void ddks_default_options(ddks_options *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
}

int ddks_create(const ddks_options *opt, ddks_ctx **out)
{
    if (!out) return DDKS_E_INVALID_ARG;
    *out = nullptr;
    ddks_options o;
    ddks_default_options(&o);
    if (opt) o = *opt;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return DDKS_E_NO_DEVICE;
    }
    if (o.device < 0 || o.device >= ndev) return DDKS_E_NO_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, o.device) != hipSuccess) return DDKS_E_NO_DEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return DDKS_E_NO_DEVICE;
    if (hipSetDevice(o.device) != hipSuccess) return DDKS_E_DEVICE;

    ddks_ctx *c = new (std::nothrow) ddks_ctx();
    if (!c) return DDKS_E_NOMEM;
    c->device = o.device;
    c->opt_flags = o.flags;
    c->serve_streams = o.serve_streams > 0 ? o.serve_streams : 4;
    c->serve_queue_depth = o.serve_queue_depth > 0 ? o.serve_queue_depth : 65536;
    if (o.tune_cache) c->tune_cache = o.tune_cache;
    if (const char *e = getenv("DDKS_FORCE_WAVES")) c->force_waves = atoi(e);
    if (const char *e = getenv("DDKS_FORCE_CHUNKS")) c->force_chunks = atoll(e);
    if (const char *e = getenv("DDKS_FORCE_PERM")) {
        int w = 0, pb = 0;
        if (sscanf(e, "%d:%d", &w, &pb) == 2) {
            c->force_perm_waves = w;
            c->force_perm_pb = pb;
        }
    }
    if (const char *e = getenv("DDKS_FORCE_PACKED_WAVES")) c->force_packed_waves = atoi(e);
    if (const char *e = getenv("DDKS_SERVE_HOLD")) c->serve_hold = atoll(e);
    if (const char *e = getenv("DDKS_FORCE_VSWEEP")) {
        int w = 0, ch = 0, g = 1;
        if (sscanf(e, "%d:%d:%d", &w, &ch, &g) >= 2) {
            c->force_vsweep.waves = w;
            c->force_vsweep.chunks = ch;
            c->force_vsweep.per_block = g;
        }
    }
    parse_fault_injection(c);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        delete c;
        return DDKS_E_DEVICE;
    }
    c->budget = o.mem_budget ? o.mem_budget : (uint64_t)(free_b * 0.9);
    int st = DDKS_OK;
    if (o.stream) {
        c->stream = (hipStream_t)o.stream;
    } else {
        st = hip_check(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "stream");
        c->own_stream = (st == DDKS_OK);
    }
    if (!st) st = hip_check(c, hipMalloc((void **)&c->result_dev, sizeof(ResultDev)), "hipMalloc");
    if (!st) st = hip_check(c, hipMalloc((void **)&c->flags_dev, 2 * sizeof(uint32_t)), "hipMalloc");
    if (!st) st = hip_check(c, hipMemset(c->flags_dev, 0, 2 * sizeof(uint32_t)), "hipMemset");
    if (!st) st = hip_check(c, hipHostMalloc((void **)&c->done_host, 64, hipHostMallocCoherent), "hipHostMalloc");
    if (!st) *c->done_host = 0u;
    if (!st) st = hip_check(c, hipMalloc((void **)&c->rank_ctl_dev, RANK_CTL_WORDS * sizeof(uint32_t)), "hipMalloc");
    if (!st) st = hip_check(c, hipMemset(c->rank_ctl_dev, 0, RANK_CTL_WORDS * sizeof(uint32_t)), "hipMemset");
    if (!st) st = hip_check(c, hipHostMalloc((void **)&c->result_host, sizeof(ResultDev), 0), "hipHostMalloc");
    if (!st) st = hip_check(c, hipHostMalloc((void **)&c->rank_distinct_host, 16 * sizeof(uint32_t), 0), "hipHostMalloc");
    if (!st) st = hip_check(c, hipHostMalloc((void **)&c->count_host, 64, hipHostMallocCoherent), "hipHostMalloc");
    if (!st) st = hip_check(c, hipHostMalloc((void **)&c->sig_host, 2 * sizeof(double), 0), "hipHostMalloc");
    if (!st) c->used += sizeof(ResultDev) + 2 * sizeof(uint32_t) + 16 * sizeof(uint32_t);
    c->profile = (o.flags & DDKS_PROFILE_KERNELS) != 0;
    for (int i = 0; i < 4 && !st && c->profile; ++i)
        st = hip_check(c, hipEventCreate(&c->ev[i]), "hipEventCreate");
    if (!st) c->tuner = tuner_create(c->tune_cache.empty() ? nullptr : c->tune_cache.c_str());
    if (!st) noalloc_setup(c);
    if (st) {
        ddks_destroy(c);
        return st;
    }
    *out = c;
    return DDKS_OK;
}

int ddks_destroy(ddks_ctx *c)
{
    if (!c) return DDKS_OK;
    (void)hipSetDevice(c->device);
    serve_stop(c);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->batch_exec) (void)hipGraphExecDestroy(c->batch_exec);
    DevBuf *bufs[] = {&c->z, &c->zr, &c->vox, &c->partial, &c->block_best, &c->counts, &c->rank_scratch,
                      &c->labels, &c->nums, &c->sig, &c->inc, &c->obs};
    for (DevBuf *b : bufs) release(c, *b);
    if (c->result_dev) (void)hipFree(c->result_dev);
    if (c->flags_dev) (void)hipFree(c->flags_dev);
    if (c->rank_ctl_dev) (void)hipFree(c->rank_ctl_dev);
    if (c->result_host) (void)hipHostFree(c->result_host);
    if (c->done_host) (void)hipHostFree(c->done_host);
    if (c->rank_distinct_host) (void)hipHostFree(c->rank_distinct_host);
    if (c->count_host) (void)hipHostFree(c->count_host);
    if (c->sig_host) (void)hipHostFree(c->sig_host);
    for (int i = 0; i < 4; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->dist_exec) (void)hipGraphExecDestroy(c->dist_exec);
    if (c->vdks_front_exec) (void)hipGraphExecDestroy(c->vdks_front_exec);
    if (c->vdks_back_exec) (void)hipGraphExecDestroy(c->vdks_back_exec);
    if (c->rdks_exec) (void)hipGraphExecDestroy(c->rdks_exec);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    tuner_destroy(c->tuner);
    delete c;
    return DDKS_OK;
}

int ddks_distance(ddks_ctx *c, const float *P, int64_t n_p, const float *Q, int64_t n_q,
                  int32_t d, uint32_t flags, ddks_result *out, uint32_t *counts)
{
    if (!c) return DDKS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->poisoned) return fail(c, DDKS_E_DEVICE, "context poisoned by an earlier device error");
    if (!P || !Q || !out) return fail(c, DDKS_E_INVALID_ARG, "null pointer argument");
    if (d < 1 || d > 8) return fail(c, DDKS_E_INVALID_ARG, "d must be in [1, 8]");
    if (n_p < 1 || n_q < 1) return fail(c, DDKS_E_INVALID_ARG, "each sample needs at least one point");
    const int64_t N = n_p + n_q;
    if (N > 0x7fffffffLL) return fail(c, DDKS_E_INVALID_ARG, "n_p + n_q exceeds 2^31 - 1");
    if (hipSetDevice(c->device) != hipSuccess) return hip_check(c, hipGetLastError(), "hipSetDevice");
    if (fault_injected(c, FAULT_CALL))
        return hip_check(c, hipErrorLaunchFailure, "injected launch failure (DDKS_FAULT_INJECT)");
    const bool dev = (flags & DDKS_DEVICE_PTRS) != 0;
    hipStream_t s = c->stream;
    const size_t bins = (size_t)1 << d;
    __atomic_store_n(c->done_host, 0u, __ATOMIC_RELEASE);  // set again by this call's reduction

    int st = ensure(c, c->z, (size_t)N * d * sizeof(float), "points");
    if (st) return st;
    float *Z = (float *)c->z.ptr;
    uint32_t *counts_dev = nullptr;
    if (counts) {
        if (dev) {
            counts_dev = counts;
        } else {
            st = ensure(c, c->counts, (size_t)N * bins * 2 * sizeof(uint32_t), "counts");
            if (st) return st;
            counts_dev = (uint32_t *)c->counts.ptr;
        }
    }
    int path = choose_path(c, d, N, flags);
    const bool with_S = (flags & DDKS_WITH_SIGNIFICANCE) != 0;

    // Device-resident inputs and outputs and a launch shape already known:
    // the whole call is one captured graph, replayed while its key matches.
    // No decision may wait on the host halfway, so past 65536 points the rank
    // path codes every dimension by shifted positions (an eager call reads the
    // distinct counts first and keeps the dense ranks where they fit).  With
    // kernel profiling the graph stops before the sweep, which is launched
    // between timing events (events recorded inside a graph cannot be timed).
    const bool graphable = c->dist_graphs && dev && !with_S &&
                           (path == PATH_F32 || rank_position_shift(N) >= 0) && !tune_pending(c, path, d, N);
    if (graphable) {
        DistArgs a;
        a.P = P;
        a.Q = Q;
        a.n_p = n_p;
        a.n_q = n_q;
        a.d = d;
        a.path = path;
        a.shifts = path == PATH_R16 && N > 65536 ? shifts_all(rank_position_shift(N), d) : 0;
        a.counts = counts_dev;
        a.plan = plan_for(c, path, d, N, n_p);
        if (a.shifts && a.plan.chunks < 2) {
            a.plan.chunks = 2;  // the corrections go into the chunks' partial counts
            if (!plan_complete(a.plan, N, n_p)) return fail(c, DDKS_E_DEVICE, "no launch shape for shifted codes");
        }
        st = prepare_distance(c, a);
        if (st) return st;
        const std::vector<uint64_t> key = {
            (uint64_t)(uintptr_t)P, (uint64_t)(uintptr_t)Q, (uint64_t)n_p, (uint64_t)n_q,
            (uint64_t)d, (uint64_t)path, (uint64_t)(uintptr_t)counts_dev, (uint64_t)a.plan.waves,
            (uint64_t)a.plan.chunks, (uint64_t)a.plan.hists, c->buf_gen, (uint64_t)(uintptr_t)s,
            (uint64_t)c->profile};
        if (c->dist_exec && c->dist_key != key) {
            (void)hipGraphExecDestroy(c->dist_exec);
            c->dist_exec = nullptr;
        }
        if (!c->dist_exec) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ex = nullptr;
            bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
            int st2 = DDKS_OK;
            if (ok) {
                st2 = enqueue_distance(c, a, s, !c->profile);
                ok = hipStreamEndCapture(s, &g) == hipSuccess && st2 == DDKS_OK;
            }
            ok = ok && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
            if (!ok) {
                // Capture is an optimisation: fall back to eager launches for
                // good.  Launches refused inside a failed capture are not
                // device errors, so they do not poison the context; a real
                // fault shows again on the eager path.
                (void)hipGetLastError();
                if (ex) (void)hipGraphExecDestroy(ex);
                c->dist_graphs = false;
                c->ev_pending = false;
                c->poisoned = false;
            } else {
                c->dist_exec = ex;
                c->dist_key = key;
            }
        }
        if (c->dist_exec) {
            st = hip_check(c, hipGraphLaunch(c->dist_exec, s), "graph launch");
            if (st) return st;
            if (a.shifts) c->prof.shifted_calls += 1;
            if (c->profile) {
                c->prof.graph_calls += 1;
                const void *zdata = path == PATH_R16 ? c->zr.ptr : c->z.ptr;
                st = run_sweep(c, a.plan, zdata, N, n_p, n_q, counts_dev, c->result_host, s, a.shifts);
                if (st) return st;
            }
            return finish_distance(c, n_p, n_q, d, out, nullptr, nullptr, 0, false);
        }
    }

    // The significance reads the counts on the device; they stay there unless
    // the caller asked for them.
    const int sig_model = (flags & DDKS_SIG_POISSON) ? SIG_MODEL_POISSON : SIG_MODEL_BINOMIAL;
    const int sig_rows = with_S ? significance_rows(n_q, sig_model) : 0;
    if (with_S) {
        if (!counts_dev) {
            st = ensure(c, c->counts, (size_t)N * bins * 2 * sizeof(uint32_t), "counts");
            if (st) return st;
            counts_dev = (uint32_t *)c->counts.ptr;
        }
        st = ensure(c, c->sig, significance_scratch_bytes(n_p, n_q, sig_rows, sig_model) + 64,
                    "significance scratch");
        if (st) return st;
    }
    const float *srcP = P, *srcQ = Q;
    if (!dev) {
        st = hip_check(c, hipMemcpyAsync(Z, P, (size_t)n_p * d * sizeof(float), hipMemcpyHostToDevice, s), "H2D P");
        if (!st) st = hip_check(c, hipMemcpyAsync(Z + n_p * d, Q, (size_t)n_q * d * sizeof(float), hipMemcpyHostToDevice, s), "H2D Q");
        if (st) return st;
        srcP = Z;
        srcQ = Z + n_p * d;
    }
    st = hip_check(c, launch_ingest_f32(srcP, n_p, srcQ, n_q, d, Z, c->flags_dev, s), "ingest launch");
    if (st) return st;
    const void *zdata = Z;
    uint32_t shifts = 0;  // per-dimension shifts, 4 bits each
    if (path == PATH_R16) {
        bool ok = false;
        st = encode_rank16(c, N, d, &ok, &shifts);
        if (st) return st;
        if (ok) zdata = c->zr.ptr;
        else path = PATH_F32;
    }
    st = tune_sweep(c, path, d, N, n_p, n_q, zdata);
    if (st) return st;
    SweepPlan plan = plan_for(c, path, d, N, n_p);
    if (shifts && plan.chunks < 2) {
        // the corrections go into the chunks' partial counts
        plan.chunks = 2;
        if (!plan_complete(plan, N, n_p)) return fail(c, DDKS_E_DEVICE, "no launch shape for shifted codes");
    }
    if (shifts) c->prof.shifted_calls += 1;
    st = run_sweep(c, plan, zdata, N, n_p, n_q, counts_dev, with_S ? c->result_dev : c->result_host, s, shifts);
    if (st) return st;
    if (with_S) {
        // S of the statistic just found: num is read on the device
        double *Sdev = (double *)((char *)c->sig.ptr + significance_scratch_bytes(n_p, n_q, sig_rows, sig_model));
        st = hip_check(c, launch_significance(counts_dev, N, d, n_p, n_q, 0, &c->result_dev->num, sig_model,
                                              c->sig.ptr, sig_rows, c->flags_dev, Sdev, s),
                       "significance launch");
        if (!st) st = hip_check(c, hipMemcpyAsync(c->result_host, c->result_dev, sizeof(ResultDev),
                                                  hipMemcpyDeviceToHost, s), "D2H result");
        if (!st) st = hip_check(c, hipMemcpyAsync(c->sig_host, Sdev, sizeof(double), hipMemcpyDeviceToHost, s),
                                "D2H S");
        if (st) return st;
    }
    return finish_distance(c, n_p, n_q, d, out, counts && !dev ? counts : nullptr, counts_dev,
                           (size_t)N * bins * 2 * sizeof(uint32_t), with_S);
}

int ddks_distance_noalloc(ddks_ctx *c, const float *P, int64_t n_p, const float *Q, int64_t n_q,
                          int32_t d, uint32_t flags, ddks_result *out, uint32_t *counts)
{
    if (!c) return DDKS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->poisoned) return fail(c, DDKS_E_DEVICE, "context poisoned by an earlier device error");
    if (!P || !Q || !out) return fail(c, DDKS_E_INVALID_ARG, "null pointer argument");
    if (d < 1 || d > 8) return fail(c, DDKS_E_INVALID_ARG, "d must be in [1, 8]");
    if (n_p < 1 || n_q < 1) return fail(c, DDKS_E_INVALID_ARG, "each sample needs at least one point");
    if (flags & DDKS_WITH_SIGNIFICANCE)
        return fail(c, DDKS_E_NOT_SUPPORTED, "the no-allocation call does not compute the significance");
    const int64_t N = n_p + n_q;
    if (N > 0x7fffffffLL) return fail(c, DDKS_E_INVALID_ARG, "n_p + n_q exceeds 2^31 - 1");
    if (hipSetDevice(c->device) != hipSuccess) return hip_check(c, hipGetLastError(), "hipSetDevice");
    char *base = (char *)noalloc_scratch(c->device);
    if (!base) return fail(c, DDKS_E_DEVICE, "the no-allocation scratch is not available on this device");
    // Rank codes up to 65536 points, read straight from P and Q; beyond that
    // fp32 compares (shifted codes would need the larger tables of the
    // position coding).
    int path = choose_path(c, d, N, flags);
    if (path == PATH_R16 && N > 65536) path = PATH_F32;
    // The context's launch shape (tuned if known; no tuning launches here),
    // with as many of its point chunks as the scratch holds.
    const SweepPlan want = plan_for(c, path, d, N, n_p);
    SweepPlan plan;
    bool fits = false;
    for (int64_t k = want.chunks; k >= 1 && !fits; --k) {
        plan = want;
        plan.chunks = k;
        fits = plan_complete(plan, N, n_p) && noalloc_layout(plan, N, d).total <= NOALLOC_SCRATCH_BYTES;
    }
    if (!fits) {
        plan = want;
        plan.chunks = 1;
        (void)plan_complete(plan, N, n_p);
        char msg[160];
        snprintf(msg, sizeof msg, "input needs %zu bytes of scratch; the no-allocation call has %zu",
                 noalloc_layout(plan, N, d).total, NOALLOC_SCRATCH_BYTES);
        return fail(c, DDKS_E_NOMEM, msg);
    }
    const NoallocLayout L = noalloc_layout(plan, N, d);
    hipStream_t s = c->stream;
    __atomic_store_n(c->done_host, 0u, __ATOMIC_RELEASE);  // set again by this call's reduction
    void *pts = base + L.pts;
    int st;
    if (path == PATH_R16)
        st = hip_check(c, launch_rank16_pq(P, n_p, Q, n_q, d, (uint32_t *)pts, base + L.rank, c->flags_dev, s),
                       "rank launch");
    else
        st = hip_check(c, launch_ingest_f32(P, n_p, Q, n_q, d, (float *)pts, c->flags_dev, s), "ingest launch");
    if (st) return st;
    st = sweep_into(c, plan, pts, N, n_p, n_q, counts, c->result_host, s, 0, (BlockBest *)(base + L.bb),
                    plan.chunks > 1 ? base + L.partial : nullptr, nullptr, false);
    if (st) return st;
    return finish_distance(c, n_p, n_q, d, out, nullptr, nullptr, 0, false);
}

int ddks_profile_get(ddks_ctx *c, ddks_profile *out, int32_t reset)
{
    if (!c || !out) return DDKS_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(c->mu);
    *out = c->prof;
    if (reset) c->prof = ddks_profile{};
    return DDKS_OK;
}

}  // extern "C"
