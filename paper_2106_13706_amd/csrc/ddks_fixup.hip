// Corrections that make a sweep on shifted 16-bit codes exact
// (arXiv:2106.13706, Sec. 2.1 Eq. membership: the orthant code compares full
// coordinates, which a 16-bit code only approximates once a dimension has
// more than 65536 distinct values).
//
// Such a dimension codes a point by F >> shift, F the first sorted position
// of its value.  A compare of point x against origin o there is exact except
// when the two share a code and x's value is the smaller: the sweep then
// counted x as x_m >= o_m.  Those points lie in sorted positions
// [(F_o >> shift) << shift, F_o), fewer than 2^shift of them whatever the
// ties, and this pass moves each from the orthant the sweep used to the exact
// one, in the partial counts of the chunk that holds the point, before
// scoring.  That chunk counted the point in the orthant it is taken from, and
// a move keeps the chunk's counts a partition of its own points, so no count
// goes below zero or past the chunk's size (packed 16-bit halves stay valid).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "ddks_device.h"

namespace ddks {

// One thread per origin o, which alone owns its partial counts (lane o mod
// 64 of group o / 64, in every chunk), so plain read-modify-writes suffice.
// F holds, for shifted dimensions, the first sorted position of each point's
// value (dense ranks elsewhere, where nothing is corrected).  A point to
// correct in several dimensions is moved once, in the lowest of them.
template <int D>
__global__ __launch_bounds__(256) void k_rank_fixups(const uint32_t *__restrict__ F,
                                                     const uint64_t *__restrict__ S, int64_t N,
                                                     int64_t n_p, uint32_t shifts, int64_t chunk_len,
                                                     int64_t groups, int packed,
                                                     void *__restrict__ partial)
{
    constexpr int BINS = Geo<D>::BINS;
    uint32_t sh[D];
#pragma unroll
    for (int m = 0; m < D; ++m) sh[m] = (shifts >> (4 * m)) & 15u;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < N;
         o += (int64_t)gridDim.x * blockDim.x) {
        uint32_t fo[D];
#pragma unroll
        for (int m = 0; m < D; ++m) fo[m] = F[o * D + m];
        // entry of bin 0 of this origin in chunk 0; chunk c is c * groups * BINS * 64 entries on
        const size_t o0 = (size_t)(o >> 6) * BINS * 64 + (o & 63);
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const uint32_t code = fo[m] >> sh[m];
            // the sorted positions of o's code below o's own value
            for (uint32_t p = code << sh[m]; p < fo[m]; ++p) {
                const int64_t x = (int64_t)(uint32_t)S[(size_t)m * N + p];
                uint32_t fx[D];
#pragma unroll
                for (int k = 0; k < D; ++k) fx[k] = F[x * D + k];
                if ((fx[m] >> sh[m]) != code) continue;  // a value that starts in the code below
                bool done_before = false;
#pragma unroll
                for (int k = 0; k < m; ++k)
                    done_before |= ((fx[k] >> sh[k]) == (fo[k] >> sh[k])) && (fx[k] < fo[k]);
                if (done_before) continue;
                uint32_t ca = 0, ce = 0;  // codes of the sweep's compares and of the exact ones
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    ca |= ((fx[k] >> sh[k]) >= (fo[k] >> sh[k]) ? 1u : 0u) << k;
                    ce |= (fx[k] >= fo[k] ? 1u : 0u) << k;
                }
                const size_t at = o0 + (size_t)(x / chunk_len) * groups * BINS * 64;
                const size_t ia = at + (size_t)(ca ^ Geo<D>::FLIP) * 64;
                const size_t ie = at + (size_t)(ce ^ Geo<D>::FLIP) * 64;
                if (packed) {
                    uint32_t *p32 = static_cast<uint32_t *>(partial);
                    const uint32_t one = x < n_p ? 1u : 0x10000u;
                    p32[ia] -= one;
                    p32[ie] += one;
                } else {
                    uint2 *p64 = static_cast<uint2 *>(partial);
                    if (x < n_p) {
                        p64[ia].x -= 1u;
                        p64[ie].x += 1u;
                    } else {
                        p64[ia].y -= 1u;
                        p64[ie].y += 1u;
                    }
                }
            }
        }
    }
}

hipError_t launch_rank_fixups(const SweepPlan &plan, const RankTables &t, int64_t N, int64_t n_p,
                              uint32_t shifts, void *partial, hipStream_t s)
{
    if (shifts == 0 || N < 1 || plan.chunks < 2 || plan.chunk_len < 1 || !partial) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)std::min<int64_t>((N + 255) / 256, 4096);
    const int packed = partial_packed(plan) ? 1 : 0;
    switch (plan.d) {
#define DDKS_FIX(DD)                                                                                     \
    case DD:                                                                                             \
        hipLaunchKernelGGL(k_rank_fixups<DD>, dim3(blocks), dim3(256), 0, s, t.R32, t.S, N, n_p, shifts, \
                           plan.chunk_len, plan.groups, packed, partial);                                \
        return hipGetLastError();
        DDKS_FIX(1) DDKS_FIX(2) DDKS_FIX(3) DDKS_FIX(4) DDKS_FIX(5) DDKS_FIX(6) DDKS_FIX(7) DDKS_FIX(8)
#undef DDKS_FIX
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ddks
