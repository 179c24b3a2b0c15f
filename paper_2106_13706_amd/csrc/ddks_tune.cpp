// Launch-shape autotuner for the orthant-counting sweep (and the shapes of
// the permutation kernel and of the packed serving sweep).
//
// The sweep's speed depends on how many waves share a block's origins (and
// how many LDS histograms they need, hence occupancy) and on how many point
// chunks the origin groups are split into (grid size vs. the cost of partial
// counts).
// On the first sizeable call for a (path, d, log2 N) key the tuner times
// every admissible shape on the real input with HIP events, keeps the
// fastest, and (optionally) appends it to a text cache file of lines
// "path d log2N waves chunks".
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <map>
#include <tuple>

#include "ddks_runtime.h"

namespace ddks {

struct Tuner {
    std::mutex m;
    std::map<std::tuple<int, int, int>, std::pair<int, int64_t>> best;
    std::string path;
};

static int bucket(int64_t N) { return (int)lround(log2((double)std::max<int64_t>(N, 1))); }

Tuner *tuner_create(const char *cache_path)
{
    Tuner *t = new (std::nothrow) Tuner();
    if (!t) return nullptr;
    if (cache_path) {
        t->path = cache_path;
        if (FILE *f = fopen(cache_path, "r")) {
            int p, d, b, w;
            long long ch;
            while (fscanf(f, "%d %d %d %d %lld", &p, &d, &b, &w, &ch) == 5)
                t->best[{p, d, b}] = {w, (int64_t)ch};
            fclose(f);
        }
    }
    return t;
}

void tuner_destroy(Tuner *t) { delete t; }

bool tuner_lookup(Tuner *t, int path, int d, int64_t N, SweepPlan *plan)
{
    if (!t) return false;
    std::lock_guard<std::mutex> lk(t->m);
    auto it = t->best.find({path, d, bucket(N)});
    if (it == t->best.end()) return false;
    plan->waves = it->second.first;
    plan->chunks = std::min<int64_t>(it->second.second, N);
    return true;
}

static void tuner_store(Tuner *t, int path, int d, int64_t N, int waves, int64_t chunks)
{
    std::lock_guard<std::mutex> lk(t->m);
    t->best[{path, d, bucket(N)}] = {waves, chunks};
    if (!t->path.empty())
        if (FILE *f = fopen(t->path.c_str(), "a")) {
            fprintf(f, "%d %d %d %d %lld\n", path, d, bucket(N), waves, (long long)chunks);
            fclose(f);
        }
}

// Entries of the other kernels share the map and the cache file, under
// their own kinds in the first field: the permutation kernel as PERM_KIND +
// path with (waves, relabellings per block), the packed sweep as
// PACKED_KIND + path with (waves, 0), vdKS's weighted sweep as VSWEEP_KIND
// (+ 1 for its byte encoding of the voxel coordinates) with (waves, chunks +
// 256 (origin groups per block - 1)).
static constexpr int PERM_KIND = 10, PACKED_KIND = 20;

bool tuner_lookup_perm(Tuner *t, int path, int d, int64_t n, int *waves, int *pb)
{
    if (!t) return false;
    std::lock_guard<std::mutex> lk(t->m);
    auto it = t->best.find({PERM_KIND + path, d, bucket(n)});
    if (it == t->best.end() || !perm_shape_ok(d, (int)it->second.second, it->second.first)) return false;
    *waves = it->second.first;
    *pb = (int)it->second.second;
    return true;
}

void tuner_store_perm(Tuner *t, int path, int d, int64_t n, int waves, int pb)
{
    if (t) tuner_store(t, PERM_KIND + path, d, n, waves, pb);
}

bool tuner_lookup_packed(Tuner *t, int path, int d, int64_t n, int *waves)
{
    if (!t) return false;
    std::lock_guard<std::mutex> lk(t->m);
    auto it = t->best.find({PACKED_KIND + path, d, bucket(n)});
    if (it == t->best.end()) return false;
    *waves = it->second.first;
    return true;
}

void tuner_store_packed(Tuner *t, int path, int d, int64_t n, int waves)
{
    if (t) tuner_store(t, PACKED_KIND + path, d, n, waves, 0);
}

static constexpr int VSWEEP_KIND = 30;

bool tuner_lookup_vsweep(Tuner *t, int d, int64_t M, bool bytes, VSweepPlan *plan)
{
    if (!t) return false;
    std::lock_guard<std::mutex> lk(t->m);
    auto it = t->best.find({VSWEEP_KIND + (bytes ? 1 : 0), d, bucket(M)});
    if (it == t->best.end()) return false;
    plan->waves = it->second.first;
    plan->chunks = (int)(it->second.second & 0xff);
    plan->per_block = (int)(it->second.second >> 8) + 1;
    return true;
}

// stored as (waves, chunks + 256 (origin groups per block - 1))
void tuner_store_vsweep(Tuner *t, int d, int64_t M, bool bytes, const VSweepPlan &plan)
{
    if (t) tuner_store(t, VSWEEP_KIND + (bytes ? 1 : 0), d, M, plan.waves, plan.chunks + 256 * (plan.per_block - 1));
}

bool tune_pending(ddks_ctx *c, int path, int d, int64_t N)
{
    if (!c->tuner || (c->opt_flags & DDKS_NO_AUTOTUNE) || c->force_waves || c->force_chunks)
        return false;
    if (N < 16384) return false;  // launch-bound sizes: the heuristic is as good
    SweepPlan probe;
    return !tuner_lookup(c->tuner, path, d, N, &probe);
}

int tune_sweep(ddks_ctx *c, int path, int d, int64_t N, int64_t n_p, int64_t n_q, const void *zdata)
{
    if (!tune_pending(c, path, d, N)) return DDKS_OK;
    const int64_t groups = (N + 63) / 64;
    std::vector<SweepPlan> cand;
    for (int w : {1, 2, 4, 8, 12, 16}) {
        // 12-wave blocks: two per CU beside the d = 4 pair table
        if (w == 12 && d != 4) continue;
        for (int64_t ch : {1, 2, 3, 4, 6, 8, 12, 16}) {
            SweepPlan p;
            p.path = path;
            p.d = d;
            p.waves = w;
            p.chunks = ch;
            if (!plan_complete(p, N, n_p) || p.chunks != ch) continue;
            if (p.chunk_len < (int64_t)w * 256) continue;
            if (groups * ch * w > 65536 * 4) continue;
            cand.push_back(p);
        }
    }
    if (cand.size() < 2) return DDKS_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = hip_check(c, hipEventCreate(&e0), "hipEventCreate");
    if (!st) st = hip_check(c, hipEventCreate(&e1), "hipEventCreate");
    float best_ms = 1e30f;
    SweepPlan best = cand[0];
    const bool prof = c->profile;
    c->profile = false;  // tuning runs are not part of the profile
    for (const SweepPlan &p : cand) {
        if (st) break;
        float ms_min = 1e30f;
        for (int rep = 0; rep < 2 && !st; ++rep) {
            st = hip_check(c, hipEventRecord(e0, c->stream), "hipEventRecord");
            if (!st) st = run_sweep(c, p, zdata, N, n_p, n_q, nullptr, c->result_dev, c->stream);
            if (!st) st = hip_check(c, hipEventRecord(e1, c->stream), "hipEventRecord");
            if (!st) st = hip_check(c, hipEventSynchronize(e1), "hipEventSynchronize");
            float ms = 0.f;
            if (!st) {
                if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) ms_min = std::min(ms_min, ms);
                else (void)hipGetLastError();
            }
        }
        if (ms_min < best_ms) {
            best_ms = ms_min;
            best = p;
        }
    }
    c->profile = prof;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) return st;
    tuner_store(c->tuner, path, d, N, best.waves, best.chunks);
    return DDKS_OK;
}

}  // namespace ddks
