// How many waves of a kernel stay resident per SIMD on this GPU, as a
// function of the kernel's scalar and vector register counts and its block
// size.  Each wave spins for a fixed real time (20 us of the 100 MHz
// constant clock), then records when it started and ended and where it ran
// (hardware wave id and XCC id); the host counts the most waves alive at once
// on the whole GPU and on each CU.  Register counts are set by clobbering one
// high register in an empty asm statement, so every variant runs the same
// instructions.  A grid holding more waves than fit at once runs in several
// rounds, which the kernel time (a multiple of 20 us) shows as well.  Usage:
// occupancy; prints one line per case.  Exit status 1 on a HIP error.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <utility>
#include <vector>

namespace {

constexpr long long SPIN_TICKS = 2000;  // 20 us at 100 MHz

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

// VG / SG: the highest vector / scalar register the kernel claims (0: none).
template <int NT, int VG, int SG>
__global__ __launch_bounds__(NT) void k_occ(unsigned long long *out, long long spin, int nwaves)
{
    extern __shared__ unsigned lds[];
    lds[threadIdx.x] = threadIdx.x;  // the launch passes at least NT words
    if constexpr (VG == 56) asm volatile("" ::: "v56");
    if constexpr (VG == 63) asm volatile("" ::: "v63");
    if constexpr (VG == 64) asm volatile("" ::: "v64");
    if constexpr (SG == 70) asm volatile("" ::: "s70");
    if constexpr (SG == 78) asm volatile("" ::: "s78");
    if constexpr (SG == 86) asm volatile("" ::: "s86");
    if constexpr (SG == 94) asm volatile("" ::: "s94");
    if constexpr (SG == 100) asm volatile("" ::: "s100");
    __syncthreads();
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    const unsigned hw = __builtin_amdgcn_s_getreg(4 | (31 << 11));    // HW_ID
    const unsigned xcc = __builtin_amdgcn_s_getreg(20 | (31 << 11));  // XCC_ID
    unsigned long long t1 = t0;
    while ((long long)(t1 - t0) < spin) t1 = __builtin_amdgcn_s_memrealtime();
    __syncthreads();
    const unsigned long long t2 = __builtin_amdgcn_s_memrealtime();
    const int wave = (int)((blockIdx.x * NT + threadIdx.x) / 64);
    if ((threadIdx.x & 63) == 0 && wave < nwaves) {
        out[wave * 4 + 0] = t0;
        out[wave * 4 + 1] = t2;
        out[wave * 4 + 2] = hw;
        out[wave * 4 + 3] = (xcc & 0xfu) + 0ull * lds[(threadIdx.x + 1) % NT];
    }
}

int peak(std::vector<std::pair<unsigned long long, int>> ev)
{
    std::sort(ev.begin(), ev.end());
    int cur = 0, best = 0;
    for (const auto &e : ev) {
        cur += e.second;
        best = std::max(best, cur);
    }
    return best;
}

template <int NT, int VG, int SG>
void run(const char *name, int blocks)
{
    const int waves = blocks * NT / 64;
    const size_t lds = (size_t)NT * sizeof(unsigned);
    unsigned long long *d = nullptr;
    CHECK(hipMalloc(&d, (size_t)waves * 4 * sizeof(unsigned long long)));
    CHECK(hipMemset(d, 0, (size_t)waves * 4 * sizeof(unsigned long long)));
    hipFuncAttributes attr;
    CHECK(hipFuncGetAttributes(&attr, (const void *)k_occ<NT, VG, SG>));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL((k_occ<NT, VG, SG>), dim3(blocks), dim3(NT), lds, 0, d, SPIN_TICKS, waves);  // warm-up
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL((k_occ<NT, VG, SG>), dim3(blocks), dim3(NT), lds, 0, d, SPIN_TICKS, waves);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    std::vector<unsigned long long> h((size_t)waves * 4);
    CHECK(hipMemcpy(h.data(), d, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    std::vector<std::pair<unsigned long long, int>> all;
    std::map<unsigned long long, std::vector<std::pair<unsigned long long, int>>> per_cu;
    for (int w = 0; w < waves; ++w) {
        const unsigned long long t0 = h[w * 4], t1 = h[w * 4 + 1];
        const unsigned hw = (unsigned)h[w * 4 + 2];
        // CU = (XCC, SE, SH, CU) from HW_ID's cu_id (bits 8-11), sh_id (12), se_id (13-15)
        const unsigned long long cu = (h[w * 4 + 3] << 16) | ((hw >> 8) & 0xffu);
        all.push_back({t0, +1});
        all.push_back({t1, -1});
        per_cu[cu].push_back({t0, +1});
        per_cu[cu].push_back({t1, -1});
    }
    int cu_min = 1 << 30, cu_max = 0;
    for (auto &kv : per_cu) {
        const int p = peak(kv.second);
        cu_min = std::min(cu_min, p);
        cu_max = std::max(cu_max, p);
    }
    std::printf("%-16s %3d VGPRs | %5d blocks x %4d threads: kernel %6.1f us, peak %5d of %5d waves "
                "at once, %zu CUs, per-CU peak %d..%d waves\n",
                name, attr.numRegs, blocks, NT, ms * 1000.0, peak(all), waves, per_cu.size(), cu_min, cu_max);
    std::fflush(stdout);
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    CHECK(hipFree(d));
}

}  // namespace

int main()
{
    // 4-wave blocks, 2048 of them: 32 waves per CU if 8 per SIMD stay resident
    run<256, 0, 0>("few registers", 2048);
    run<256, 63, 0>("64 VGPRs", 2048);
    run<256, 64, 0>("65 VGPRs", 2048);
    run<256, 0, 70>("s70 clobbered", 2048);
    run<256, 0, 78>("s78 clobbered", 2048);
    run<256, 0, 86>("s86 clobbered", 2048);
    run<256, 0, 94>("s94 clobbered", 2048);
    run<256, 0, 100>("s100 clobbered", 2048);
    // 16-wave blocks: two per CU need 8 waves per SIMD
    run<1024, 0, 70>("16-wave, s70", 512);
    run<1024, 0, 86>("16-wave, s86", 512);
    return 0;
}
