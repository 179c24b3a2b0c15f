// Throughput of the LDS atomics the kernels are built on, in CU clocks per
// wave64 instruction (at the nominal 2.4 GHz), for the rooflines that are
// bound by them:
//   ds_add_u32, lane-minor bins (bin * 64 + lane, one histogram shared by the
//     block's waves): one 32-bit bin per point of the sweeps; the 64 lanes of
//     an instruction always fall in 64 different banks;
//   ds_add_u64, lane-minor bins: the permutation kernel's four 16-bit counters
//     per 64-bit word;
//   ds_add_u32, lane-major bins (lane * (B + 1) + bin): the layout the sweeps
//     do not use (bank conflicts whenever two lanes' bins collide).
// Each wave issues NI independent atomics per iteration to bins drawn once per
// lane from a fixed pseudo-random sequence, so the loop is bound by the LDS
// pipe, not by the few vector instructions around it.  Usage: lds_atomic_rate
// [iterations]; prints one line per case.  Exit status 1 on a HIP error.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int THREADS = 256;  // 4 waves per block
constexpr int NI = 8;         // atomics in flight per lane and iteration
constexpr int BINS = 64;      // bins per lane (a d = 6 histogram)

enum Layout { LANE_MINOR = 0, LANE_MAJOR = 1 };

template <typename T, int LAYOUT>
__global__ __launch_bounds__(THREADS) void k_lds_rate(int iters, unsigned long long *sink)
{
    // lane-minor: BINS x 64 entries; lane-major: 64 x (BINS + 1) entries
    __shared__ T h[LAYOUT == LANE_MINOR ? BINS * 64 : 64 * (BINS + 1)];
    for (int i = threadIdx.x; i < (int)(sizeof(h) / sizeof(T)); i += THREADS) h[i] = 0;
    __syncthreads();
    const int t = threadIdx.x, lane = t & 63;
    unsigned x = 2463534242u ^ (t * 2654435761u) ^ (blockIdx.x * 40503u);
    int idx[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        const int bin = (int)(x % BINS);
        idx[k] = LAYOUT == LANE_MINOR ? bin * 64 + lane : lane * (BINS + 1) + bin;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < NI; ++k) atomicAdd(&h[idx[k]], (T)1);
    }
    __syncthreads();
    T s = 0;
    for (int i = threadIdx.x; i < (int)(sizeof(h) / sizeof(T)); i += THREADS) s += h[i];
    if (s == (T)0x7fffffff) sink[0] = (unsigned long long)s;  // keeps the work observable
}

template <typename T, int LAYOUT>
int run(const char *name, int iters, int blocks, unsigned long long *sink)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
    hipLaunchKernelGGL((k_lds_rate<T, LAYOUT>), dim3(blocks), dim3(THREADS), 0, 0, 16, sink);  // warm-up
    if (hipEventRecord(e0, 0) != hipSuccess) return 1;
    hipLaunchKernelGGL((k_lds_rate<T, LAYOUT>), dim3(blocks), dim3(THREADS), 0, 0, iters, sink);
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, 0) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess)
        return 1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess) return 1;
    const double wave_insts = (double)blocks * (THREADS / 64) * (double)iters * NI;
    const double cu_clocks = ms * 1e-3 * 2.4e9 * prop.multiProcessorCount;
    printf("%-44s %8.3f ms  %6.2f CU clocks per wave instruction (%d CUs, %d blocks x %d waves, %d x %d atomics)\n",
           name, ms, cu_clocks / wave_insts, prop.multiProcessorCount, blocks, THREADS / 64, iters, NI);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return 0;
}

}  // namespace

int main(int argc, char **argv)
{
    const int iters = argc > 1 ? atoi(argv[1]) : 4096;
    if (iters < 1 || iters > (1 << 20)) {
        fprintf(stderr, "iterations must be in [1, 2^20]\n");
        return 2;
    }
    unsigned long long *sink = nullptr;
    if (hipMalloc(&sink, sizeof(*sink)) != hipSuccess) return 1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, 0) != hipSuccess) return 1;
    const int blocks = prop.multiProcessorCount * 8;
    int st = 0;
    st |= run<unsigned, LANE_MINOR>("ds_add_u32, lane-minor bins", iters, blocks, sink);
    st |= run<unsigned long long, LANE_MINOR>("ds_add_u64, lane-minor bins", iters, blocks, sink);
    st |= run<unsigned, LANE_MAJOR>("ds_add_u32, lane-major bins (lane*(B+1)+bin)", iters, blocks, sink);
    (void)hipFree(sink);
    if (st) fprintf(stderr, "HIP error\n");
    return st ? 1 : 0;
}
