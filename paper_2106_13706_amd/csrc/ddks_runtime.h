// Host-side context of libddks: device buffers under a memory budget, the
// context stream, launch planning, and the helpers shared by the single-test,
// permutation and serving paths.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ddks.h"
#include "ddks_internal.h"

namespace ddks {

struct Serve;  // serving loop (ddks_serve.cpp)

// A device allocation that grows on demand and is charged to its context's budget.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Tuner;  // launch-shape autotuner (ddks_tune.cpp)

}  // namespace ddks

struct ddks_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    uint32_t opt_flags = 0;
    int serve_streams = 4;
    int serve_queue_depth = 65536;
    std::string tune_cache;
    int force_waves = 0;   // test override (DDKS_FORCE_WAVES)
    int64_t force_chunks = 0;  // test override (DDKS_FORCE_CHUNKS)
    int force_perm_waves = 0, force_perm_pb = 0;  // test override (DDKS_FORCE_PERM="waves:pb")
    int force_packed_waves = 0;  // test override (DDKS_FORCE_PACKED_WAVES)
    int64_t serve_hold = 0;      // test override (DDKS_SERVE_HOLD): first launch waits for this many requests
    ddks::VSweepPlan force_vsweep{0, 1, 1};  // test override (DDKS_FORCE_VSWEEP="waves:chunks[:groups]")
    int fault_site = 0;        // test override (DDKS_FAULT_INJECT), see fault_injected
    std::atomic<int64_t> fault_countdown{0};
    std::atomic<bool> poisoned{false};
    std::string last_error;
    std::mutex mu;  // serialises the synchronous calls on `stream`

    // buffers of the synchronous path
    ddks::DevBuf z, zr, partial, block_best, counts, rank_scratch, labels, nums, sig, inc, obs, vox;
    uint64_t buf_gen = 0;  // bumped whenever a buffer is reallocated

    // captured permutation-batch graph, replayed while its key matches
    hipGraphExec_t batch_exec = nullptr;
    std::vector<uint64_t> batch_key;
    // captured single-test graph (device-resident inputs), same scheme
    hipGraphExec_t dist_exec = nullptr;
    std::vector<uint64_t> dist_key;
    bool dist_graphs = true;  // cleared for good if a capture ever fails
    // vdKS with device-resident inputs: the launches before the host read of
    // the filled-voxel count, and those after it, each captured and replayed
    // while their key matches (the second key includes the count and shape)
    hipGraphExec_t vdks_front_exec = nullptr, vdks_back_exec = nullptr;
    std::vector<uint64_t> vdks_front_key, vdks_back_key;
    bool vdks_graphs = true;  // cleared for good if a capture ever fails
    // rdKS with device-resident inputs: the whole call, same scheme
    hipGraphExec_t rdks_exec = nullptr;
    std::vector<uint64_t> rdks_key;
    bool rdks_graphs = true;
    ddks::ResultDev *result_dev = nullptr;  // device
    ddks::ResultDev *result_host = nullptr; // pinned
    uint32_t *flags_dev = nullptr;          // device, cleared by the reduction
    uint32_t *done_host = nullptr;          // pinned, coherent: 1 once a call's result is in result_host
    uint32_t *rank_distinct_host = nullptr; // pinned
    uint32_t *count_host = nullptr;         // pinned, coherent: vdKS's filled-voxel count, polled by the host
    double *sig_host = nullptr;             // pinned, 2 doubles
    uint32_t *rank_ctl_dev = nullptr;

    // kernel timing (DDKS_PROFILE_KERNELS)
    bool profile = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ev_pending = false;
    bool ev_score = false;
    bool batch_capturing = false;  // no event records while a graph is being captured
    bool graph_pending = false;
    int64_t ev_compares = 0;
    ddks_profile prof{};

    ddks::Tuner *tuner = nullptr;
    ddks::Serve *serve = nullptr;
    std::mutex serve_mu;
};

namespace ddks {

// Test-only fault injection, for the error paths that a real device fault
// would take: with DDKS_FAULT_INJECT="<site>:<k>" in the environment at
// context creation (site: call, serve_launch or serve_event), the k-th time
// the context reaches that site (k >= 1) the library acts as if the HIP
// runtime had reported a launch failure there.  Nothing is launched at a
// failing call or serving launch; a failing serving event is reported only
// after the launch it marks has really completed.
enum FaultSite : int { FAULT_NONE = 0, FAULT_CALL = 1, FAULT_SERVE_LAUNCH = 2, FAULT_SERVE_EVENT = 3 };
bool fault_injected(ddks_ctx *c, int site);

// Records an error on the context and returns status.
int fail(ddks_ctx *c, int status, const std::string &msg);
// Checks a HIP return code; on failure poisons the context.
int hip_check(ddks_ctx *c, hipError_t e, const char *what);

// Grows b to at least bytes (contents not preserved), charging the budget.
int ensure(ddks_ctx *c, DevBuf &b, size_t bytes, const char *what);
void release(ddks_ctx *c, DevBuf &b);

// Launch shape for one test of N points in dimension d on the given path.
// Fills groups, chunk_len and hists of a plan whose path, d, waves and chunks
// are set; false if no admissible histogram count exists for that shape.
bool plan_complete(SweepPlan &p, int64_t N, int64_t n_p);
// Launch shape for a sweep of N points (n_p of the first sample): the tuned
// shape if there is one, else a heuristic.
SweepPlan plan_for(ddks_ctx *c, int path, int d, int64_t N, int64_t n_p);

// Runs the sweep + score + reduce of one test whose points are already in a
// device buffer (fp32 N x d at zf, and when path == PATH_R16 the rank
// encoding at zr).  Leaves the result in c->result_dev; does not synchronise.
// shifts != 0: zdata is the shifted rank encoding of c->rank_scratch's
// tables (4-bit shift per dimension, plan.chunks >= 2); the rank-group
// corrections run between sweep and score.
int run_sweep(ddks_ctx *c, const SweepPlan &plan, const void *zdata, int64_t N, int64_t n_p,
              int64_t n_q, uint32_t *counts_dev, ddks::ResultDev *res, hipStream_t s, uint32_t shifts = 0);

// run_sweep on buffers the caller provides (block_best: plan.groups entries;
// partial: partial_bytes(plan) when plan.chunks > 1; rank_scratch: the
// encoding's tables when shifts != 0); allocates nothing.  prof: record the
// timing events of DDKS_PROFILE_KERNELS.
int sweep_into(ddks_ctx *c, const SweepPlan &plan, const void *zdata, int64_t N, int64_t n_p, int64_t n_q,
               uint32_t *counts_dev, ddks::ResultDev *res, hipStream_t s, uint32_t shifts, ddks::BlockBest *bb,
               void *partial, void *rank_scratch, bool prof);

// Folds the events recorded by the last run_sweep into c->prof (after the
// stream has been synchronised).
void profile_collect(ddks_ctx *c);

// Chooses the path for a test (fp32 or rank-16) given the caller's flags.
int choose_path(ddks_ctx *c, int d, int64_t N, uint32_t flags);

// Encodes the fp32 points in c->z (N x d) as int16 ranks into c->zr.  A
// dimension with more than 65536 distinct values is coded by shifted first
// sorted positions (F >> shift_m, the smallest shift_m with N <= 65536 <<
// shift_m, packed 4 bits per dimension into *shifts) and the sweep needs the
// corrections of launch_rank_fixups (run_sweep with shifts); past
// N = 65536 << RANK_MAX_SHIFT, *ok = false and the caller falls back to the
// fp32 path.
constexpr int RANK_MAX_SHIFT = 6;
// The shift that codes N sorted positions in 16 bits: 0 for N <= 65536, -1
// past 65536 << RANK_MAX_SHIFT.
int rank_position_shift(int64_t N);
// `shift` in the 4-bit fields of all d dimensions: the coding of calls that
// cannot wait for the distinct counts (captured graphs, serving).
uint32_t shifts_all(int shift, int d);
int encode_rank16(ddks_ctx *c, int64_t N, int d, bool *ok, uint32_t *shifts);

// Serving lifecycle (ddks_serve.cpp).
int serve_start(ddks_ctx *c);
void serve_stop(ddks_ctx *c);

// Autotuner (ddks_tune.cpp).
Tuner *tuner_create(const char *cache_path);
void tuner_destroy(Tuner *t);
// Returns true and fills plan (waves, chunks) if a tuned shape exists for (path, d, N bucket).
bool tuner_lookup(Tuner *t, int path, int d, int64_t N, SweepPlan *plan);
// Times the admissible launch shapes of a sweep on the given (already
// ingested) input once per (path, d, N bucket) and records the fastest.
int tune_sweep(ddks_ctx *c, int path, int d, int64_t N, int64_t n_p, int64_t n_q, const void *zdata);
// True if tune_sweep would time candidate shapes for this key.
bool tune_pending(ddks_ctx *c, int path, int d, int64_t N);
// The permutation kernel's tuned (waves, relabellings per block) for (path, d,
// log2 n), and recording one.
bool tuner_lookup_perm(Tuner *t, int path, int d, int64_t n, int *waves, int *pb);
void tuner_store_perm(Tuner *t, int path, int d, int64_t n, int waves, int pb);
// The packed (serving) sweep's tuned waves per block for (path, d, log2 of
// the launch's largest test), and recording one.
bool tuner_lookup_packed(Tuner *t, int path, int d, int64_t n, int *waves);
void tuner_store_packed(Tuner *t, int path, int d, int64_t n, int waves);
// vdKS's weighted sweep: the tuned (waves, chunks) for (d, log2 of the filled voxels).
bool tuner_lookup_vsweep(Tuner *t, int d, int64_t M, bool bytes, VSweepPlan *plan);
void tuner_store_vsweep(Tuner *t, int d, int64_t M, bool bytes, const VSweepPlan &plan);

// Launches enqueue()'s work on s: by replaying the graph in *exec when
// *key_have equals key, else by capturing enqueue() into a new graph first.
// A failed capture falls back to an eager run, and to eager runs for good
// (*enabled cleared; launches refused inside a failed capture are not device
// errors, so they do not poison the context: a real fault shows again on the
// eager path).
template <typename F>
int replay_or_capture(ddks_ctx *c, bool *enabled, hipGraphExec_t *exec, std::vector<uint64_t> *key_have,
                      const std::vector<uint64_t> &key, hipStream_t s, F enqueue)
{
    if (!*enabled) return enqueue();
    if (*exec && *key_have != key) {
        (void)hipGraphExecDestroy(*exec);
        *exec = nullptr;
    }
    if (!*exec) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ex = nullptr;
        bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
        int st = DDKS_OK;
        if (ok) {
            st = enqueue();
            ok = hipStreamEndCapture(s, &g) == hipSuccess && st == DDKS_OK;
        }
        ok = ok && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (!ok) {
            (void)hipGetLastError();
            if (ex) (void)hipGraphExecDestroy(ex);
            *enabled = false;
            c->poisoned = false;
            return enqueue();
        }
        *exec = ex;
        *key_have = key;
    }
    return hip_check(c, hipGraphLaunch(*exec, s), "graph launch");
}

}  // namespace ddks
