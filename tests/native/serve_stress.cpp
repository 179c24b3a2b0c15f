// Concurrent clients of the serving loop (ddks_serve_submit / ddks_serve_poll)
// against plain ddks_distance calls, for a build of the library whose host
// code carries AddressSanitizer and UndefinedBehaviorSanitizer (the device
// code is built as usual).  T threads each submit R tests of random shape
// (d in 1..6, 16..6000 points per sample, some with the analytic
// significance) and poll their tickets, some submitted in bursts before any
// poll; the main thread then checks every result against a plain call on the
// same inputs, and finally destroys a context with requests still in flight
// (they must be failed and drained, not leaked or touched after free).
// Usage: serve_stress [threads] [requests per thread]; exit status 0 when
// every served result equals the plain call's; a sanitizer report aborts
// with its own status.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <unistd.h>
#include <vector>

#include "ddks.h"

namespace {

struct Test {
    std::vector<float> P, Q;
    int d = 1;
    uint32_t flags = 0;
    uint64_t ticket = 0;
    ddks_result served{};
    int status = -1;
};

// splitmix64: reproducible inputs from (thread, index)
uint64_t mix(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

void make_test(Test &t, uint64_t seed)
{
    uint64_t s = mix(seed);
    t.d = 1 + (int)(s % 6);
    s = mix(s);
    const int64_t n_p = 16 + (int64_t)(s % 6000);
    s = mix(s);
    const int64_t n_q = 16 + (int64_t)(s % 6000);
    s = mix(s);
    t.flags = (s % 7 == 0) ? DDKS_WITH_SIGNIFICANCE : 0u;
    t.P.resize((size_t)n_p * t.d);
    t.Q.resize((size_t)n_q * t.d);
    for (float &x : t.P) {
        s = mix(s);
        x = (float)((int64_t)(s % 2001) - 1000) / 250.0f;  // ties likely
    }
    for (float &x : t.Q) {
        s = mix(s);
        x = (float)((int64_t)(s % 2001) - 1000) / 230.0f + 0.1f;
    }
}

int submit(ddks_ctx *c, Test &t)
{
    ddks_request r;
    r.P = t.P.data();
    r.n_p = (int64_t)t.P.size() / t.d;
    r.Q = t.Q.data();
    r.n_q = (int64_t)t.Q.size() / t.d;
    r.d = t.d;
    r.flags = t.flags;
    for (;;) {
        const int st = ddks_serve_submit(c, &r, &t.ticket);
        if (st != DDKS_E_AGAIN) return st;
        std::this_thread::yield();
    }
}

}  // namespace

int main(int argc, char **argv)
{
    const int T = argc > 1 ? atoi(argv[1]) : 4;
    const int R = argc > 2 ? atoi(argv[2]) : 60;
    if (T < 1 || T > 16 || R < 1 || R > 1000) {
        fprintf(stderr, "threads in [1, 16], requests in [1, 1000]\n");
        return 2;
    }
    ddks_ctx *c = nullptr;
    if (ddks_create(nullptr, &c) != DDKS_OK) {
        fprintf(stderr, "ddks_create failed\n");
        return 1;
    }
    std::vector<std::vector<Test>> tests(T, std::vector<Test>(R));
    std::atomic<int> bad{0};
    std::vector<std::thread> th;
    for (int k = 0; k < T; ++k)
        th.emplace_back([&, k] {
            std::vector<Test> &v = tests[k];
            for (int i = 0; i < R; ++i) make_test(v[i], (uint64_t)k * 100003u + (uint64_t)i);
            // bursts of 8 submissions, then their polls
            for (int i0 = 0; i0 < R; i0 += 8) {
                const int i1 = i0 + 8 < R ? i0 + 8 : R;
                for (int i = i0; i < i1; ++i)
                    if (submit(c, v[i]) != DDKS_OK) ++bad;
                for (int i = i0; i < i1; ++i) v[i].status = ddks_serve_poll(c, v[i].ticket, -1, &v[i].served);
            }
        });
    for (std::thread &t : th) t.join();
    int checked = 0;
    for (int k = 0; k < T; ++k)
        for (Test &t : tests[k]) {
            ddks_result plain{};
            const int64_t n_p = (int64_t)t.P.size() / t.d, n_q = (int64_t)t.Q.size() / t.d;
            const int st = ddks_distance(c, t.P.data(), n_p, t.Q.data(), n_q, t.d, t.flags, &plain, nullptr);
            const bool same = st == DDKS_OK && t.status == DDKS_OK && plain.num == t.served.num &&
                              plain.den == t.served.den && plain.argmax_origin == t.served.argmax_origin &&
                              plain.argmax_orthant == t.served.argmax_orthant &&
                              (t.flags == 0u || plain.S == t.served.S);
            if (!same) {
                ++bad;
                fprintf(stderr, "mismatch: d=%d n=(%lld,%lld) status %d/%d num %llu/%llu\n", t.d,
                        (long long)n_p, (long long)n_q, t.status, st, (unsigned long long)t.served.num,
                        (unsigned long long)plain.num);
            }
            ++checked;
        }
    // a context destroyed with requests still queued or in flight
    std::vector<Test> last(32);
    for (int i = 0; i < 32; ++i) {
        make_test(last[i], 777000u + (uint64_t)i);
        if (submit(c, last[i]) != DDKS_OK) ++bad;
    }
    if (ddks_destroy(c) != DDKS_OK) ++bad;
    printf("serve_stress: %d threads x %d requests, %d checked against plain calls, %d bad\n", T, R, checked,
           bad.load());
    fflush(stdout);
    // skip the exit handlers: a host-sanitized runtime's allocator checks can
    // trip over the HIP runtime's own teardown after every check above is done
    _exit(bad.load() == 0 ? 0 : 1);
}
