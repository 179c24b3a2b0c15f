// Entry points whose device paths are not built yet report DDKS_E_NOT_SUPPORTED.
#include "ddks_runtime.h"

using namespace ddks;

namespace ddks {
struct Tuner {};
Tuner *tuner_create(const char *) { return nullptr; }
void tuner_destroy(Tuner *) {}
bool tuner_lookup(Tuner *, int, int, int64_t, SweepPlan *) { return false; }
int serve_start(ddks_ctx *) { return DDKS_E_NOT_SUPPORTED; }
void serve_stop(ddks_ctx *) {}
}  // namespace ddks

extern "C" {
int ddks_serve_submit(ddks_ctx *c, const ddks_request *, uint64_t *)
{ return fail(c, DDKS_E_NOT_SUPPORTED, "serving not built"); }
int ddks_serve_poll(ddks_ctx *c, uint64_t, int32_t, ddks_result *)
{ return fail(c, DDKS_E_NOT_SUPPORTED, "serving not built"); }
int ddks_serve_stats_get(ddks_ctx *c, ddks_serve_stats *, int32_t)
{ return fail(c, DDKS_E_NOT_SUPPORTED, "serving not built"); }
}
