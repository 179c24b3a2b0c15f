// Serving loop of libddks: continuous batching of many exact ddKS tests
// (arXiv:2106.13706, Sec. 2.1) of mixed dimension and size on one GPU.
//
//   submit  copies the request (mapping -0 to +0, rejecting non-finite
//           values) and queues it;
//   admit   a scheduler thread moves queued requests, oldest first, into a
//           device arena while it has room (the arena is charged to the
//           context's memory budget);
//   launch  admitted tests are packed, per dimension and compare path, into
//           one launch whose blocks are (test, origin group) work items, on
//           one of several streams, so launches overlap on the device and
//           requests that arrive while others run join the next launch;
//           large tests (SERVE_SOLO_MIN <= N) are swept on their own with
//           the point-chunked plan of a plain call instead: a packed block
//           sweeps all N points for its 64 origins, too coarse a unit to keep
//           every CU busy to the end of a large test;
//           mid-size tests (SERVE_R16_MIN <= N <= 65536) are first rank
//           encoded on the device for the 16-bit compare path (at most N
//           distinct values per dimension, so the ranks always fit); larger
//           solo tests up to SERVE_R16_MAX points take shifted position codes
//           in every dimension, encoded, swept and corrected one after
//           another on the slot's stream (the corrections read the slot's
//           rank tables);
//   retire  finished launches (HIP events) hand their results to the
//           tickets, free their arena space and wake pollers.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "ddks_runtime.h"

namespace ddks {

using Clock = std::chrono::steady_clock;

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with coalescing.
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t n)
    {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    int64_t alloc(size_t n)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                return (int64_t)off;
            }
        }
        return -1;
    }
    void release(size_t off, size_t n)
    {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Smallest test swept on the rank-encoded path: below it the two encoding
// launches cost about what the 16-bit compares save.
static constexpr int64_t SERVE_R16_MIN = 16384;

// Smallest test swept on its own with a chunked plan, and the per-slot
// buffer for the partial counts of its chunks (they grow with 2^d; two chunks
// of a d = 8 test of SERVE_R16_MAX points fill it).
static constexpr int64_t SERVE_SOLO_MIN = 16384;
static constexpr size_t SERVE_SOLO_PARTIAL = 512ull << 20;
// Largest test on the 16-bit compare path (the per-slot rank scratch is sized
// for it); past 65536 points with shifted codes, solo sweeps only.
static constexpr int64_t SERVE_R16_MAX = 131072;

struct Req {
    uint64_t ticket = 0;
    int d = 0;
    int64_t n_p = 0, n_q = 0, N = 0;
    int hists = 1;            // LDS histograms per block of its packed sweep
    int path = PATH_F32;      // compare path of its sweep
    uint32_t shifts = 0;      // shifted position codes (PATH_R16 past 65536 points)
    bool solo = false;        // swept on its own with `plan` (not packed)
    SweepPlan plan;
    int sig_model = -1;       // analytic significance asked for: SIG_MODEL_*, else -1
    int sig_rows = 0;         // its tail kernel's waves in flight
    std::vector<float> data;  // P then Q
    // arena layout: fp32 points | rank-encoded points (PATH_R16) | block results
    // | (with the significance) counts [N][2^d][2] | significance scratch
    size_t pts_bytes = 0, r16_bytes = 0, bb_bytes = 0, counts_bytes = 0, sig_bytes = 0, bytes = 0;
    int64_t off = -1;
    bool done = false;
    int status = DDKS_OK;
    ddks_result result{};
    Clock::time_point t_submit, t_done;
};

// One stream with the buffers of the launch in flight on it.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;  // timing events around the launch in flight
    bool busy = false;
    std::vector<Req *> reqs;
    // pinned staging and device copies of the launch's tables and results
    PackedTest *tests_h = nullptr, *tests_d = nullptr;
    int2 *items_h = nullptr, *items_d = nullptr;
    ResultDev *res_h = nullptr, *res_d = nullptr;
    double *S_h = nullptr, *S_d = nullptr;  // significance of each test that asked for it
    size_t cap_tests = 0, cap_items = 0;
    // rank encoding of this slot's requests, one after another on its stream
    void *rank_scratch = nullptr;
    uint32_t *rank_ctl = nullptr;  // launch_rank16 control block
    // partial counts and the (always zero) flags word of solo sweeps
    void *partial = nullptr;
    uint32_t *flags_d = nullptr;
};

// Packed launches of one batch: tests [i0, i1) share a dimension and a path.
struct PackedRun {
    size_t i0 = 0, i1 = 0, items = 0;
    int waves = PACKED_WAVES;
    int64_t maxN = 0;
    bool tune = false;
    std::vector<int> cand;  // waves to time when tuning
};

// Work items a packed launch needs before its timing is worth recording
// (fewer leave the GPU mostly idle and time the launch, not the shape).
static constexpr size_t PACKED_TUNE_MIN_ITEMS = 1024;

struct Serve {
    ddks_ctx *c = nullptr;
    std::mutex m;
    std::condition_variable cv_sched, cv_done;
    std::deque<Req *> pending;
    std::deque<Req *> ready;  // admitted, not yet launched
    std::unordered_map<uint64_t, Req *> table;
    uint64_t next_ticket = 1;
    size_t held = 0;  // requests submitted and not yet collected
    Arena arena;
    void *arena_base = nullptr;
    size_t slot_bytes = 0;  // per-slot device scratch charged to the budget
    bool use_r16 = false;   // rank-encoded path available (set once at start)
    bool use_solo = false;  // chunked solo sweeps available (set once at start)
    std::vector<Slot> slots;
    std::thread th;
    bool stop = false;
    bool failed = false;
    std::string error;
    // stats
    uint64_t submitted = 0, completed = 0, rej_again = 0, rej_nomem = 0, launches = 0,
             launched_tests = 0, shifted_tests = 0;
    std::vector<double> lat_us;
    // device time: [start, end) of every retired launch in ms after `ref`
    hipEvent_t ref = nullptr;
    std::vector<std::pair<float, float>> spans;

    hipEvent_t tune_e0 = nullptr, tune_e1 = nullptr;  // timing of packed-sweep shapes

    int grow_slot(Slot &s, size_t tests, size_t items);
    bool launch_batch(Slot &s, std::vector<Req *> &batch);
    void fail_req(Req *r);
    void retire(Slot &s);
    void loop();
};

int Serve::grow_slot(Slot &s, size_t tests, size_t items)
{
    if (tests > s.cap_tests) {
        size_t n = std::max(tests, s.cap_tests * 2);
        if (s.tests_h) (void)hipHostFree(s.tests_h);
        if (s.tests_d) (void)hipFree(s.tests_d);
        if (s.res_h) (void)hipHostFree(s.res_h);
        if (s.res_d) (void)hipFree(s.res_d);
        if (s.S_h) (void)hipHostFree(s.S_h);
        if (s.S_d) (void)hipFree(s.S_d);
        s.tests_h = nullptr;
        s.tests_d = nullptr;
        s.res_h = nullptr;
        s.res_d = nullptr;
        s.S_h = nullptr;
        s.S_d = nullptr;
        if (hipHostMalloc((void **)&s.tests_h, n * sizeof(PackedTest), 0) != hipSuccess ||
            hipMalloc((void **)&s.tests_d, n * sizeof(PackedTest)) != hipSuccess ||
            hipHostMalloc((void **)&s.res_h, n * sizeof(ResultDev), 0) != hipSuccess ||
            hipMalloc((void **)&s.res_d, n * sizeof(ResultDev)) != hipSuccess ||
            hipHostMalloc((void **)&s.S_h, n * sizeof(double), 0) != hipSuccess ||
            hipMalloc((void **)&s.S_d, n * sizeof(double)) != hipSuccess)
            return DDKS_E_DEVICE;
        s.cap_tests = n;
    }
    if (items > s.cap_items) {
        size_t n = std::max(items, s.cap_items * 2);
        if (s.items_h) (void)hipHostFree(s.items_h);
        if (s.items_d) (void)hipFree(s.items_d);
        s.items_h = nullptr;
        s.items_d = nullptr;
        if (hipHostMalloc((void **)&s.items_h, n * sizeof(int2), 0) != hipSuccess ||
            hipMalloc((void **)&s.items_d, n * sizeof(int2)) != hipSuccess)
            return DDKS_E_DEVICE;
        s.cap_items = n;
    }
    return DDKS_OK;
}

// Uploads the batch's points and tables and enqueues one packed launch per
// dimension present, then the per-test reductions and the result copy.
bool Serve::launch_batch(Slot &s, std::vector<Req *> &batch)
{
    if (fault_injected(c, FAULT_SERVE_LAUNCH)) {
        error = "injected serving launch failure (DDKS_FAULT_INJECT)";
        return false;
    }
    // packed tests first (sorted by dimension and path), then the solo ones
    std::stable_sort(batch.begin(), batch.end(), [](const Req *a, const Req *b) {
        if (a->solo != b->solo) return !a->solo;
        return a->d != b->d ? a->d < b->d : a->path < b->path;
    });
    size_t nitems = 0, npacked = 0;
    for (Req *r : batch)
        if (!r->solo) {
            nitems += (size_t)((r->N + 63) / 64);
            ++npacked;
        }
    // one packed launch per run of equal dimension and path; its waves per
    // block: forced (tests), tuned for (path, d, log2 of the run's largest
    // test), or the default, and timed on this launch when not yet tuned
    std::vector<PackedRun> runs;
    std::vector<int> hists(batch.size(), 1);
    for (size_t i0 = 0; i0 < npacked;) {
        PackedRun run;
        run.i0 = i0;
        run.i1 = i0;
        int64_t maxN = 0;
        while (run.i1 < npacked && batch[run.i1]->d == batch[i0]->d && batch[run.i1]->path == batch[i0]->path) {
            maxN = std::max(maxN, batch[run.i1]->N);
            run.items += (size_t)((batch[run.i1]->N + 63) / 64);
            ++run.i1;
        }
        const int d = batch[i0]->d, path = batch[i0]->path;
        // waves w serve the run if every test has histograms for it, as many
        // as for the default (the test table holds one count per test)
        auto serves = [&](int w) {
            if (!packed_waves_ok(w)) return false;
            for (size_t k = run.i0; k < run.i1; ++k) {
                const Req *r = batch[k];
                const int h = sweep_hists(d, w, r->N, r->n_p, r->n_q);
                if (h == 0 || h != sweep_hists(d, PACKED_WAVES, r->N, r->n_p, r->n_q)) return false;
            }
            return true;
        };
        int w = 0;
        if (c->force_packed_waves && serves(c->force_packed_waves)) {
            w = c->force_packed_waves;
        } else if (!(tuner_lookup_packed(c->tuner, path, d, maxN, &w) && serves(w))) {
            w = PACKED_WAVES;
            run.tune = c->tuner && !(c->opt_flags & DDKS_NO_AUTOTUNE) && run.items >= PACKED_TUNE_MIN_ITEMS;
            for (int cw : {4, 8, 16})
                if (run.tune && serves(cw)) run.cand.push_back(cw);
            run.tune = run.cand.size() >= 2;
        }
        run.waves = w;
        run.maxN = maxN;
        for (size_t k = run.i0; k < run.i1; ++k)
            hists[k] = sweep_hists(d, w, batch[k]->N, batch[k]->n_p, batch[k]->n_q);
        runs.push_back(run);
        i0 = run.i1;
    }
    if (grow_slot(s, batch.size(), nitems) != DDKS_OK) {
        error = "serving buffer allocation failed";
        return false;
    }
    char *base = (char *)arena_base;
    BlockBest *bb = (BlockBest *)arena_base;
    size_t it = 0;
    if (hipEventRecord(s.t0, s.stream) != hipSuccess) {
        error = "event record failed";
        return false;
    }
    for (size_t i = 0; i < batch.size(); ++i) {
        Req *r = batch[i];
        PackedTest &t = s.tests_h[i];
        char *zf = base + r->off, *zr = zf + r->pts_bytes;
        t.Z = r->path == PATH_R16 ? (const void *)zr : (const void *)zf;
        t.N = r->N;
        t.n_p = r->n_p;
        t.n_q = r->n_q;
        t.groups = (r->N + 63) / 64;
        t.bb_offset = (int64_t)((r->off + r->pts_bytes + r->r16_bytes) / sizeof(BlockBest));
        t.hists = r->solo ? r->hists : hists[i];
        t.path = r->path;
        if (!r->solo)
            for (int64_t g = 0; g < t.groups; ++g) s.items_h[it++] = make_int2((int)i, (int)g);
        if (hipMemcpyAsync(zf, r->data.data(), r->data.size() * sizeof(float),
                           hipMemcpyHostToDevice, s.stream) != hipSuccess) {
            error = "H2D request copy failed";
            return false;
        }
        if (r->path == PATH_R16 && !r->shifts &&
            launch_rank16((const float *)zf, r->N, r->d, (uint32_t *)zr, s.rank_scratch,
                          s.rank_ctl, s.stream) != hipSuccess) {
            error = "rank encoding launch failed";
            return false;
        }
    }
    if (npacked &&
        (hipMemcpyAsync(s.tests_d, s.tests_h, npacked * sizeof(PackedTest), hipMemcpyHostToDevice,
                        s.stream) != hipSuccess ||
         hipMemcpyAsync(s.items_d, s.items_h, nitems * sizeof(int2), hipMemcpyHostToDevice,
                        s.stream) != hipSuccess)) {
        error = "H2D table copy failed";
        return false;
    }
    // one launch per run of equal dimension and path (the batch is sorted so)
    size_t item0 = 0;
    for (PackedRun &run : runs) {
        const int d = batch[run.i0]->d, path = batch[run.i0]->path;
        int max_hists = 1;
        for (size_t k = run.i0; k < run.i1; ++k) max_hists = std::max(max_hists, hists[k]);
        auto launch = [&](int w) {
            return launch_sweep_packed(path, d, w, s.tests_d, s.items_d + item0, (int64_t)run.items, max_hists,
                                       bb, s.stream);
        };
        if (run.tune) {
            // time each candidate on this launch's own tests (the sweep only
            // writes its block results, so repeating it is harmless); the
            // first timing also waits for the uploads queued before it
            float best_ms = 1e30f;
            int best = run.waves;
            for (int w : run.cand) {
                float ms_min = 1e30f;
                for (int rep = 0; rep < 2; ++rep) {
                    if (hipEventRecord(tune_e0, s.stream) != hipSuccess || launch(w) != hipSuccess ||
                        hipEventRecord(tune_e1, s.stream) != hipSuccess || hipEventSynchronize(tune_e1) != hipSuccess) {
                        error = "packed sweep tuning failed";
                        return false;
                    }
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, tune_e0, tune_e1) == hipSuccess) ms_min = std::min(ms_min, ms);
                    else (void)hipGetLastError();
                }
                if (ms_min < best_ms) {
                    best_ms = ms_min;
                    best = w;
                }
            }
            tuner_store_packed(c->tuner, path, d, run.maxN, best);
            run.waves = best;
        }
        if (launch(run.waves) != hipSuccess) {
            error = "packed sweep launch failed";
            return false;
        }
        item0 += run.items;
    }
    if (npacked && launch_reduce_packed(s.tests_d, (int64_t)npacked, bb, s.res_d, s.stream) != hipSuccess) {
        error = "packed reduction launch failed";
        return false;
    }
    // solo tests: (shifted encoding +) sweep (+ corrections) (+ score of the
    // chunks' partial counts) + reduce
    for (size_t i = npacked; i < batch.size(); ++i) {
        Req *r = batch[i];
        const PackedTest &t = s.tests_h[i];
        BlockBest *tbb = bb + t.bb_offset;
        void *part = r->plan.chunks > 1 ? s.partial : nullptr;
        if (r->shifts) {
            const float *zf = (const float *)(base + r->off);
            if (launch_rank16(zf, r->N, r->d, (uint32_t *)t.Z, s.rank_scratch, s.rank_ctl, s.stream) != hipSuccess ||
                launch_rank16_shift(r->N, r->d, (uint32_t *)t.Z, s.rank_scratch, r->shifts, s.stream) !=
                    hipSuccess) {
                error = "rank encoding launch failed";
                return false;
            }
        }
        uint32_t *counts = r->sig_model >= 0 ? (uint32_t *)((char *)tbb + r->bb_bytes) : nullptr;
        if (launch_sweep(r->plan, t.Z, r->N, r->n_p, r->n_q, part, tbb, counts, s.stream) != hipSuccess ||
            (r->shifts && launch_rank_fixups(r->plan, rank16_tables(s.rank_scratch, r->N, r->d), r->N, r->n_p,
                                             r->shifts, part, s.stream) != hipSuccess) ||
            (part && launch_score(r->plan, r->N, r->n_p, r->n_q, part, tbb, counts, s.stream) != hipSuccess) ||
            launch_reduce(tbb, r->plan.groups, s.flags_d, s.res_d + i, s.stream) != hipSuccess) {
            error = "solo sweep launch failed";
            return false;
        }
        // the analytic significance (Sec. 3) of the statistic just found, from
        // the counts on the device (num read there too)
        if (counts && launch_significance(counts, r->N, r->d, r->n_p, r->n_q, 0, &s.res_d[i].num, r->sig_model,
                                          (char *)counts + r->counts_bytes, r->sig_rows, s.flags_d, s.S_d + i,
                                          s.stream) != hipSuccess) {
            error = "significance launch failed";
            return false;
        }
    }
    if (hipMemcpyAsync(s.res_h, s.res_d, batch.size() * sizeof(ResultDev), hipMemcpyDeviceToHost,
                       s.stream) != hipSuccess ||
        hipMemcpyAsync(s.S_h, s.S_d, batch.size() * sizeof(double), hipMemcpyDeviceToHost, s.stream) !=
            hipSuccess ||
        hipEventRecord(s.t1, s.stream) != hipSuccess ||
        hipEventRecord(s.done, s.stream) != hipSuccess) {
        error = "packed reduction launch failed";
        return false;
    }
    s.reqs = batch;
    s.busy = true;
    launches += 1;
    launched_tests += batch.size();
    for (const Req *r : batch) shifted_tests += r->shifts ? 1 : 0;
    return true;
}

// Called with m held: ends a request with a device error and returns its
// arena space (nothing runs on it any more: the failed loop launches no more
// work, and a slot's stream has been waited for before its requests get here).
void Serve::fail_req(Req *r)
{
    if (r->done) return;
    r->status = DDKS_E_DEVICE;
    r->done = true;
    if (r->off >= 0) {
        arena.release((size_t)r->off, r->bytes);
        r->off = -1;
    }
}

// Called with m held, after s.done completed.
void Serve::retire(Slot &s)
{
    const auto now = Clock::now();
    float a = 0.f, b = 0.f;
    if (hipEventElapsedTime(&a, ref, s.t0) == hipSuccess && hipEventElapsedTime(&b, ref, s.t1) == hipSuccess)
        spans.emplace_back(a, b);
    else
        (void)hipGetLastError();
    for (size_t i = 0; i < s.reqs.size(); ++i) {
        Req *r = s.reqs[i];
        const ResultDev &x = s.res_h[i];
        r->result.num = x.num;
        r->result.den = (uint64_t)r->n_p * (uint64_t)r->n_q;
        r->result.D = (double)x.num / (double)r->result.den;
        r->result.argmax_origin = x.origin;
        r->result.argmax_orthant = x.code;
        r->result.d = r->d;
        r->result.n_p = r->n_p;
        r->result.n_q = r->n_q;
        r->result.S = r->sig_model >= 0 ? s.S_h[i] : -1.0;
        r->status = DDKS_OK;
        r->done = true;
        r->t_done = now;
        arena.release((size_t)r->off, r->bytes);
        r->off = -1;
        std::vector<float>().swap(r->data);
        completed += 1;
        lat_us.push_back(std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count());
    }
    s.reqs.clear();
    s.busy = false;
}

void Serve::loop()
{
    (void)hipSetDevice(c->device);
    // cap on work items per launch, so that a flood of requests still yields
    // several launches that overlap instead of one long one
    const size_t max_items = 1u << 16;
    // test override: the first launch waits until this many requests are held
    // (or the context closes), so that a burst lands in one batch
    int64_t hold = c->serve_hold;
    std::unique_lock<std::mutex> lk(m);
    while (true) {
        bool progress = false;
        for (Slot &s : slots) {
            if (!s.busy) continue;
            hipError_t q = hipEventQuery(s.done);
            if (q == hipSuccess && fault_injected(c, FAULT_SERVE_EVENT))
                q = hipErrorLaunchFailure;  // after the real completion: nothing is left running
            if (q == hipSuccess) {
                retire(s);
                progress = true;
            } else if (q != hipErrorNotReady) {
                failed = true;
                error = std::string("device error in serving: ") + hipGetErrorString(q);
                (void)hipGetLastError();
                (void)hipStreamSynchronize(s.stream);  // whatever can still finish, before its memory is returned
                (void)hipGetLastError();
                for (Req *r : s.reqs) fail_req(r);
                s.reqs.clear();
                s.busy = false;
                progress = true;
            }
        }
        if (progress) cv_done.notify_all();
        while (!pending.empty() && !failed) {
            Req *r = pending.front();
            int64_t off = arena.alloc(r->bytes);
            if (off < 0) break;
            r->off = off;
            ready.push_back(r);
            pending.pop_front();
        }
        if (hold > 0 && (stop || (int64_t)(ready.size() + pending.size()) >= hold)) hold = 0;
        if (!ready.empty() && !failed && hold <= 0) {
            Slot *free_slot = nullptr;
            for (Slot &s : slots)
                if (!s.busy) {
                    free_slot = &s;
                    break;
                }
            if (free_slot) {
                std::vector<Req *> batch;
                size_t items = 0;
                while (!ready.empty()) {
                    Req *r = ready.front();
                    size_t gi = (size_t)((r->N + 63) / 64);
                    if (!batch.empty() && items + gi > max_items) break;
                    batch.push_back(r);
                    items += gi;
                    ready.pop_front();
                }
                if (!launch_batch(*free_slot, batch)) {
                    // the requests taken for the batch are in no queue and on no
                    // slot: fail them here, once the slot's stream has drained
                    // any copies enqueued before the failure
                    failed = true;
                    (void)hipGetLastError();
                    (void)hipStreamSynchronize(free_slot->stream);
                    (void)hipGetLastError();
                    for (Req *r : batch) fail_req(r);
                }
                progress = true;
            }
        }
        if (failed) {
            // fail every request still queued and stop launching (requests on
            // slots still in flight are retired, or failed, with their slot)
            for (Req *r : pending) fail_req(r);
            for (Req *r : ready) fail_req(r);
            pending.clear();
            ready.clear();
            c->poisoned = true;
            cv_done.notify_all();
        }
        bool inflight = false;
        for (Slot &s : slots) inflight |= s.busy;
        if (stop && pending.empty() && ready.empty() && !inflight) break;
        if (failed && !inflight) {
            if (stop) break;
            cv_sched.wait(lk);
            continue;
        }
        if (progress) continue;
        if (inflight)
            cv_sched.wait_for(lk, std::chrono::microseconds(20));
        else
            cv_sched.wait(lk);
    }
}

int serve_start(ddks_ctx *c)
{
    if (c->serve) return DDKS_OK;
    Serve *sv = new (std::nothrow) Serve();
    if (!sv) return DDKS_E_NOMEM;
    sv->c = c;
    sv->slots.resize((size_t)std::max(1, c->serve_streams));
    // Per-slot rank scratch (charged to the budget) when the budget also
    // leaves a 64 MB arena; otherwise every test takes the fp32 path.  Then
    // the arena takes what the budget leaves, up to 8 GB.
    const size_t ctl_bytes = RANK_CTL_WORDS * sizeof(uint32_t);
    const size_t rank_bytes =
        std::max(rank16_scratch_bytes(65536, 8), rank16_scratch_bytes(SERVE_R16_MAX, 8)) + ctl_bytes;
    {
        const uint64_t used = c->used.load();
        const uint64_t need = (uint64_t)sv->slots.size() * rank_bytes + (64ull << 20);
        sv->use_r16 = c->budget > used && c->budget - used >= need;
    }
    for (Slot &s : sv->slots) {
        if (!sv->use_r16) break;
        if (hipMalloc(&s.rank_scratch, rank_bytes - ctl_bytes) != hipSuccess ||
            hipMalloc((void **)&s.rank_ctl, ctl_bytes) != hipSuccess ||
            hipMemset(s.rank_ctl, 0, ctl_bytes) != hipSuccess) {
            (void)hipGetLastError();
            c->serve = sv;
            serve_stop(c);
            return fail(c, DDKS_E_NOMEM, "serving scratch allocation failed");
        }
        c->used += rank_bytes;
        sv->slot_bytes += rank_bytes;
    }
    // Per-slot buffers of the solo sweeps, likewise only when the budget
    // still leaves a 64 MB arena.
    {
        const uint64_t used = c->used.load();
        const uint64_t per = SERVE_SOLO_PARTIAL + 256;
        const uint64_t need = (uint64_t)sv->slots.size() * per + (64ull << 20);
        sv->use_solo = c->budget > used && c->budget - used >= need;
    }
    for (Slot &s : sv->slots) {
        if (!sv->use_solo) break;
        if (hipMalloc((void **)&s.partial, SERVE_SOLO_PARTIAL) != hipSuccess ||
            hipMalloc((void **)&s.flags_d, 256) != hipSuccess || hipMemset(s.flags_d, 0, 256) != hipSuccess) {
            (void)hipGetLastError();
            c->serve = sv;
            serve_stop(c);
            return fail(c, DDKS_E_NOMEM, "serving scratch allocation failed");
        }
        c->used += SERVE_SOLO_PARTIAL + 256;
        sv->slot_bytes += SERVE_SOLO_PARTIAL + 256;
    }
    uint64_t left = c->budget > c->used.load() ? c->budget - c->used.load() : 0;
    uint64_t arena = std::min<uint64_t>(left, 8ull << 30);
    arena &= ~(uint64_t)255;
    if (arena < 4096) {
        c->serve = sv;
        serve_stop(c);
        return fail(c, DDKS_E_NOMEM, "no device memory budget left for serving");
    }
    if (hipMalloc(&sv->arena_base, arena + 256) != hipSuccess) {  // + slack for wide scalar loads
        (void)hipGetLastError();
        c->serve = sv;
        serve_stop(c);
        return fail(c, DDKS_E_NOMEM, "serving arena allocation failed");
    }
    c->used += arena;
    sv->arena.init(arena);
    for (Slot &s : sv->slots) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreate(&s.t0) != hipSuccess || hipEventCreate(&s.t1) != hipSuccess) {
            c->serve = sv;
            serve_stop(c);
            return hip_check(c, hipErrorOutOfMemory, "serving stream creation");
        }
    }
    if (hipEventCreate(&sv->tune_e0) != hipSuccess || hipEventCreate(&sv->tune_e1) != hipSuccess) {
        c->serve = sv;
        serve_stop(c);
        return hip_check(c, hipErrorOutOfMemory, "serving event creation");
    }
    if (hipEventCreate(&sv->ref) != hipSuccess || hipEventRecord(sv->ref, sv->slots[0].stream) != hipSuccess ||
        hipEventSynchronize(sv->ref) != hipSuccess) {
        c->serve = sv;
        serve_stop(c);
        return hip_check(c, hipErrorOutOfMemory, "serving event creation");
    }
    c->serve = sv;
    sv->th = std::thread([sv] { sv->loop(); });
    return DDKS_OK;
}

void serve_stop(ddks_ctx *c)
{
    Serve *sv = c->serve;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->m);
        sv->stop = true;
    }
    sv->cv_sched.notify_all();
    if (sv->th.joinable()) sv->th.join();
    for (Slot &s : sv->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.t0) (void)hipEventDestroy(s.t0);
        if (s.t1) (void)hipEventDestroy(s.t1);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.tests_h) (void)hipHostFree(s.tests_h);
        if (s.tests_d) (void)hipFree(s.tests_d);
        if (s.items_h) (void)hipHostFree(s.items_h);
        if (s.items_d) (void)hipFree(s.items_d);
        if (s.res_h) (void)hipHostFree(s.res_h);
        if (s.res_d) (void)hipFree(s.res_d);
        if (s.rank_scratch) (void)hipFree(s.rank_scratch);
        if (s.rank_ctl) (void)hipFree(s.rank_ctl);
        if (s.partial) (void)hipFree(s.partial);
        if (s.flags_d) (void)hipFree(s.flags_d);
    }
    c->used -= sv->slot_bytes;
    if (sv->arena_base) {
        (void)hipFree(sv->arena_base);
        c->used -= sv->arena.size;
    }
    if (sv->ref) (void)hipEventDestroy(sv->ref);
    if (sv->tune_e0) (void)hipEventDestroy(sv->tune_e0);
    if (sv->tune_e1) (void)hipEventDestroy(sv->tune_e1);
    for (auto &kv : sv->table) delete kv.second;
    delete sv;
    c->serve = nullptr;
}

}  // namespace ddks

using namespace ddks;

extern "C" {

int ddks_serve_submit(ddks_ctx *c, const ddks_request *req, uint64_t *ticket)
{
    if (!c) return DDKS_E_INVALID_ARG;
    if (!req || !ticket || !req->P || !req->Q) return fail(c, DDKS_E_INVALID_ARG, "null pointer argument");
    if (req->d < 1 || req->d > 8) return fail(c, DDKS_E_INVALID_ARG, "d must be in [1, 8]");
    if (req->n_p < 1 || req->n_q < 1) return fail(c, DDKS_E_INVALID_ARG, "each sample needs at least one point");
    if (req->flags & ~(uint32_t)(DDKS_WITH_SIGNIFICANCE | DDKS_SIG_POISSON))
        return fail(c, DDKS_E_INVALID_ARG, "request flags other than DDKS_WITH_SIGNIFICANCE and DDKS_SIG_POISSON");
    const int64_t N = req->n_p + req->n_q;
    // one block of PACKED_WAVES waves sweeps a whole test: its histograms must
    // hold either sample's share without overflow and fit in LDS
    const int hists = sweep_hists(req->d, PACKED_WAVES, N, req->n_p, req->n_q);
    if (hists == 0)
        return fail(c, DDKS_E_NOT_SUPPORTED,
                    "a sample is too large for serving (about 8 * 65535 points per sample, 4 * 65535 at d = 7, 2 * 65535 at d = 8); use ddks_distance");
    if (c->poisoned) return fail(c, DDKS_E_DEVICE, "context poisoned by an earlier device error");
    {
        std::lock_guard<std::mutex> lk(c->serve_mu);
        if (!c->serve) {
            std::lock_guard<std::mutex> lk2(c->mu);
            if (hipSetDevice(c->device) != hipSuccess) return hip_check(c, hipGetLastError(), "hipSetDevice");
            int st = serve_start(c);
            if (st) return st;
        }
    }
    Serve *sv = c->serve;
    Req *r = new (std::nothrow) Req();
    if (!r) return DDKS_E_NOMEM;
    r->d = req->d;
    r->n_p = req->n_p;
    r->n_q = req->n_q;
    r->N = N;
    r->hists = hists;
    const size_t np_el = (size_t)req->n_p * req->d, nq_el = (size_t)req->n_q * req->d;
    try {
        r->data.resize(np_el + nq_el);
    } catch (...) {
        delete r;
        return DDKS_E_NOMEM;
    }
    bool finite = true;
    for (size_t i = 0; i < np_el; ++i) {
        float v = req->P[i];
        finite &= std::isfinite(v);
        r->data[i] = v + 0.0f;  // -0 -> +0
    }
    for (size_t i = 0; i < nq_el; ++i) {
        float v = req->Q[i];
        finite &= std::isfinite(v);
        r->data[np_el + i] = v + 0.0f;
    }
    if (!finite) {
        delete r;
        return fail(c, DDKS_E_NONFINITE, "input contains NaN or infinity");
    }
    r->path = (sv->use_r16 && N >= SERVE_R16_MIN && N <= 65536) ? PATH_R16 : PATH_F32;
    // the launch heuristics of a plain call (not the tuner's entries, which
    // the calling threads may be updating), with no more chunks than the
    // slot's partial-count buffer holds.  Shifted codes need two chunks at
    // least (their corrections go into the partial counts).
    auto solo_plan = [&](int path, bool shifted, SweepPlan *out) {
        SweepPlan p = plan_for(nullptr, path, req->d, N, req->n_p);
        const size_t per_chunk = (size_t)p.groups * ((size_t)1 << p.d) * 64 * sizeof(uint2);
        if (shifted && p.chunks < 2) p.chunks = 2;
        if (p.chunks > 1 && (size_t)p.chunks * per_chunk > SERVE_SOLO_PARTIAL) {
            p.chunks = std::max<int64_t>(1, (int64_t)(SERVE_SOLO_PARTIAL / per_chunk));
        }
        if (shifted && p.chunks < 2) return false;
        if (!plan_complete(p, N, req->n_p)) return false;
        if (p.chunks > 1 && partial_bytes(p) > SERVE_SOLO_PARTIAL) return false;
        *out = p;
        return true;
    };
    // The analytic significance needs the counts, which only a solo sweep
    // writes, so such a test is swept on its own whatever its size.
    const bool want_S = (req->flags & DDKS_WITH_SIGNIFICANCE) != 0;
    if (sv->use_solo && (N >= SERVE_SOLO_MIN || want_S)) {
        SweepPlan p;
        if (sv->use_r16 && N > 65536 && N <= SERVE_R16_MAX && solo_plan(PATH_R16, true, &p)) {
            r->path = PATH_R16;
            r->shifts = shifts_all(rank_position_shift(N), req->d);
            r->solo = true;
            r->plan = p;
        } else if (solo_plan(r->path, false, &p)) {
            r->solo = true;
            r->plan = p;
        }
    }
    r->pts_bytes = align256((np_el + nq_el) * sizeof(float));
    r->r16_bytes = r->path == PATH_R16
                       ? align256((size_t)N * point_words(PATH_R16, req->d) * sizeof(uint32_t))
                       : 0;
    r->bb_bytes = align256((size_t)((N + 63) / 64) * sizeof(BlockBest));
    if (want_S) {
        if (!r->solo) {
            delete r;
            return fail(c, DDKS_E_NOT_SUPPORTED,
                        "the significance of a served test needs a solo sweep, which this memory budget leaves out");
        }
        r->sig_model = (req->flags & DDKS_SIG_POISSON) ? SIG_MODEL_POISSON : SIG_MODEL_BINOMIAL;
        r->sig_rows = significance_rows(req->n_q, r->sig_model);
        r->counts_bytes = align256((size_t)N * ((size_t)2 << req->d) * sizeof(uint32_t));
        r->sig_bytes = align256(significance_scratch_bytes(req->n_p, req->n_q, r->sig_rows, r->sig_model) + 64);
    }
    r->bytes = r->pts_bytes + r->r16_bytes + r->bb_bytes + r->counts_bytes + r->sig_bytes;
    std::lock_guard<std::mutex> lk(sv->m);
    if (sv->failed) {
        delete r;
        return fail(c, DDKS_E_DEVICE, sv->error);
    }
    if (r->bytes > sv->arena.size) {
        sv->rej_nomem += 1;
        delete r;
        return fail(c, DDKS_E_NOMEM, "request can never fit the serving memory budget");
    }
    if (sv->held >= (size_t)c->serve_queue_depth) {
        sv->rej_again += 1;
        delete r;
        return DDKS_E_AGAIN;
    }
    r->ticket = sv->next_ticket++;
    r->t_submit = Clock::now();
    sv->table[r->ticket] = r;
    sv->pending.push_back(r);
    sv->held += 1;
    sv->submitted += 1;
    *ticket = r->ticket;
    sv->cv_sched.notify_one();
    return DDKS_OK;
}

int ddks_serve_poll(ddks_ctx *c, uint64_t ticket, int32_t timeout_us, ddks_result *out)
{
    if (!c || !out) return DDKS_E_INVALID_ARG;
    Serve *sv = c->serve;
    if (!sv) return DDKS_E_UNKNOWN_TICKET;
    std::unique_lock<std::mutex> lk(sv->m);
    auto itr = sv->table.find(ticket);
    if (itr == sv->table.end()) return DDKS_E_UNKNOWN_TICKET;
    Req *r = itr->second;
    if (!r->done) {
        if (timeout_us < 0)
            sv->cv_done.wait(lk, [&] { return r->done; });
        else if (timeout_us > 0)
            sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->done; });
    }
    if (!r->done) return DDKS_E_PENDING;
    const int st = r->status;
    if (st == DDKS_OK) *out = r->result;
    sv->table.erase(itr);
    sv->held -= 1;
    delete r;
    return st;
}

int ddks_serve_stats_get(ddks_ctx *c, ddks_serve_stats *out, int32_t reset)
{
    if (!c || !out) return DDKS_E_INVALID_ARG;
    memset(out, 0, sizeof(*out));
    Serve *sv = c->serve;
    if (!sv) return DDKS_OK;
    std::lock_guard<std::mutex> lk(sv->m);
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->rejected_again = sv->rej_again;
    out->rejected_nomem = sv->rej_nomem;
    out->launches = sv->launches;
    out->shifted_tests = sv->shifted_tests;
    out->mean_batch = sv->launches ? (double)sv->launched_tests / (double)sv->launches : 0.0;
    out->resident_bytes = sv->arena.size;
    for (auto &kv : sv->arena.free_) out->resident_bytes -= kv.second;
    if (!sv->lat_us.empty()) {
        std::vector<double> v = sv->lat_us;
        std::sort(v.begin(), v.end());
        auto pct = [&](double q) {
            size_t i = (size_t)std::min<double>((double)v.size() - 1, q * (double)(v.size() - 1) + 0.5);
            return v[i];
        };
        out->p50_latency_us = pct(0.50);
        out->p99_latency_us = pct(0.99);
    }
    // union of the launches' device intervals (launches on several streams overlap)
    std::vector<std::pair<float, float>> sp = sv->spans;
    std::sort(sp.begin(), sp.end());
    double busy = 0.0, cur_a = 0.0, cur_b = -1.0;
    for (const auto &x : sp) {
        if (x.first > cur_b) {
            if (cur_b > cur_a) busy += cur_b - cur_a;
            cur_a = x.first;
            cur_b = x.second;
        } else if (x.second > cur_b) {
            cur_b = x.second;
        }
    }
    if (cur_b > cur_a) busy += cur_b - cur_a;
    out->busy_us = busy * 1e3;
    if (reset) {
        sv->submitted = sv->completed = sv->rej_again = sv->rej_nomem = 0;
        sv->launches = sv->launched_tests = sv->shifted_tests = 0;
        sv->lat_us.clear();
        sv->spans.clear();
    }
    return DDKS_OK;
}

}  // extern "C"
