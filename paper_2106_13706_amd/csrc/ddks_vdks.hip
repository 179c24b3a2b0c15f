// vdKS, the voxel approximation of the statistic (arXiv:2106.13706,
// Sec. 2.2.2, Alg. 1), on gfx950.
//
// Readings: the pooled points are normalised per dimension onto [0, 1]
// (u = (x - lo)/(hi - lo), u = 0 where hi == lo) and binned on a V^d grid,
// voxel coordinate v_m = min(V - 1, floor(u_m V)) in fp64; around every filled
// voxel the voxels split into orthants as points do around an origin in
// Eq. g (bit m = [w_m >= u_m]); the statistic is the largest absolute
// difference of the two samples' proportions in an orthant (Eq. d1).
//
// That is the exact statistic of the voxel coordinates with every filled
// voxel as an origin, so the device work is:
//   1. per-dimension minimum and maximum (ordered-key atomics);
//   2. each point's voxel key sum_m v_m V^m, merged into an open-addressing
//      hash table (64-bit CAS) that counts each sample's points per voxel;
//   3. the filled voxels compacted into a list, their coordinates written as
//      biased int16 ranks (a voxel coordinate is its own rank) and their
//      counts as one 64-bit increment (P in the low, Q in the high word);
//   4. the weighted sweep: every filled voxel against every filled voxel,
//      the orthant code exactly as in the exact sweep, 64-bit LDS bins so
//      that any sample size fits, then the scores |c_P n_Q - c_Q n_P| and the
//      maximum with ties to the lowest voxel key, then the lowest code.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "ddks_device.h"

namespace ddks {

typedef __attribute__((address_space(3))) uint64_t lds_u64v;

static constexpr uint64_t VOX_EMPTY = ~0ull;

// Order-preserving image of a finite fp32 value, and its inverse.
__device__ __forceinline__ uint32_t vox_order_key(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float vox_from_key(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void k_vox_init(uint32_t *__restrict__ mm, int d, uint64_t *__restrict__ tab_key,
                           uint32_t *__restrict__ tab_cnt, int64_t slots, uint32_t *__restrict__ counter)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < slots;
         i += (int64_t)gridDim.x * blockDim.x) {
        tab_key[i] = VOX_EMPTY;
        tab_cnt[2 * i] = 0u;
        tab_cnt[2 * i + 1] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)d) {
        mm[2 * threadIdx.x] = 0xffffffffu;  // running minimum key
        mm[2 * threadIdx.x + 1] = 0u;       // running maximum key
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
}

// Per-dimension extents in two steps, with no atomics (thousands of waves
// updating the same few words serialise): every block writes the minimum and
// maximum order keys of its share of the points to part[block][2 D], then one
// block combines the rows into mm.
template <int D>
__global__ __launch_bounds__(256) void k_vox_minmax(const float *__restrict__ Z, int64_t N,
                                                    uint32_t *__restrict__ part)
{
    __shared__ uint32_t red[4][2 * D];
    uint32_t lo[D], hi[D];
#pragma unroll
    for (int m = 0; m < D; ++m) {
        lo[m] = 0xffffffffu;
        hi[m] = 0u;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const uint32_t k = vox_order_key(Z[i * D + m]);
            lo[m] = min(lo[m], k);
            hi[m] = max(hi[m], k);
        }
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < D; ++m) {
        for (int off = 32; off >= 1; off >>= 1) {
            lo[m] = min(lo[m], (uint32_t)__shfl_xor((int)lo[m], off, 64));
            hi[m] = max(hi[m], (uint32_t)__shfl_xor((int)hi[m], off, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            red[w][2 * m] = lo[m];
            red[w][2 * m + 1] = hi[m];
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * D) {
        const int j = threadIdx.x;
        uint32_t v = red[0][j];
        for (int x = 1; x < 4; ++x) v = (j & 1) ? max(v, red[x][j]) : min(v, red[x][j]);
        part[(size_t)blockIdx.x * (2 * D) + j] = v;
    }
}

// mm[2 m] / mm[2 m + 1] = smallest / largest order key of dimension m over
// the rows part[0 .. rows) (one block of 256 threads, rows <= 256).
template <int D>
__global__ __launch_bounds__(256) void k_vox_minmax_final(const uint32_t *__restrict__ part, int rows,
                                                          uint32_t *__restrict__ mm)
{
    __shared__ uint32_t red[4][2 * D];
    const int r = threadIdx.x, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) {
        uint32_t v = r < rows ? part[(size_t)r * (2 * D) + j] : ((j & 1) ? 0u : 0xffffffffu);
        for (int off = 32; off >= 1; off >>= 1) {
            const uint32_t o = (uint32_t)__shfl_xor((int)v, off, 64);
            v = (j & 1) ? max(v, o) : min(v, o);
        }
        if ((threadIdx.x & 63) == 0) red[w][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < 2 * D) {
        const int j = threadIdx.x;
        uint32_t v = red[0][j];
        for (int x = 1; x < 4; ++x) v = (j & 1) ? max(v, red[x][j]) : min(v, red[x][j]);
        mm[j] = v;
    }
}

__device__ __forceinline__ uint64_t vox_hash(uint64_t key, uint64_t mask)
{
    return (key * 0x9e3779b97f4a7c15ull >> 17) & mask;
}

// Voxel key of every point, merged into the table (linear probing; the table
// has at least twice as many slots as points, so every probe ends).
template <int D>
__global__ __launch_bounds__(256) void k_vox_insert(const float *__restrict__ Z, int64_t N, int64_t n_p,
                                                    int V, const uint32_t *__restrict__ mm,
                                                    uint64_t *__restrict__ tab_key,
                                                    uint32_t *__restrict__ tab_cnt, uint64_t mask)
{
    double lo[D], span[D];
#pragma unroll
    for (int m = 0; m < D; ++m) {
        lo[m] = (double)vox_from_key(mm[2 * m]);
        span[m] = (double)vox_from_key(mm[2 * m + 1]) - lo[m];
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t key = 0, scale = 1;
#pragma unroll
        for (int m = 0; m < D; ++m) {
            int64_t v = 0;
            if (span[m] > 0.0) {
                const double u = ((double)Z[i * D + m] - lo[m]) / span[m];
                v = (int64_t)floor(u * (double)V);
                v = v > V - 1 ? V - 1 : (v < 0 ? 0 : v);
            }
            key += (uint64_t)v * scale;
            scale *= (uint64_t)V;
        }
        uint64_t h = vox_hash(key, mask);
        while (true) {
            const unsigned long long old = atomicCAS((unsigned long long *)&tab_key[h], VOX_EMPTY, key);
            if (old == VOX_EMPTY || old == key) break;
            h = (h + 1) & mask;
        }
        atomicAdd(&tab_cnt[2 * h + (i < n_p ? 0 : 1)], 1u);
    }
}

// Filled slots to a list: key, and the 64-bit increment c_P | c_Q << 32.
// One counter update per block of 1024 slots (a single word updated by
// every wave or slot serialises across the chip): the filled slots of a
// block take consecutive places, in slot order within the block.
static constexpr int COMPACT_THREADS = 1024;
__global__ __launch_bounds__(COMPACT_THREADS) void k_vox_compact(const uint64_t *__restrict__ tab_key,
                                                                 const uint32_t *__restrict__ tab_cnt,
                                                                 int64_t slots, uint32_t *__restrict__ counter,
                                                                 uint64_t *__restrict__ keys,
                                                                 uint64_t *__restrict__ inc)
{
    __shared__ uint32_t wbase[COMPACT_THREADS / 64];
    __shared__ uint32_t bbase;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t stride = (int64_t)gridDim.x * COMPACT_THREADS;
    for (int64_t h0 = (int64_t)blockIdx.x * COMPACT_THREADS; h0 < slots; h0 += stride) {
        const int64_t h = h0 + threadIdx.x;
        const uint64_t k = h < slots ? tab_key[h] : VOX_EMPTY;
        const bool filled = k != VOX_EMPTY;
        const uint64_t mask = __ballot(filled);
        if (lane == 0) wbase[w] = (uint32_t)__popcll(mask);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (int v = 0; v < COMPACT_THREADS / 64; ++v) {
                const uint32_t c = wbase[v];
                wbase[v] = tot;
                tot += c;
            }
            bbase = tot ? atomicAdd(counter, tot) : 0u;
        }
        __syncthreads();
        if (filled) {
            const uint32_t at = bbase + wbase[w] + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
            keys[at] = k;
            inc[at] = (uint64_t)tab_cnt[2 * h] | ((uint64_t)tab_cnt[2 * h + 1] << 32);
        }
        __syncthreads();  // wbase and bbase are rewritten for the next slots
    }
}

// Voxel coordinates as biased int16 ranks in the rank-16 point layout.
template <int D>
__global__ void k_vox_encode(const uint64_t *__restrict__ keys, int64_t M, int V,
                             uint32_t *__restrict__ R)
{
    constexpr int PW = Layout<PATH_R16, D>::PW;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[i];
        uint32_t w[PW];
#pragma unroll
        for (int p = 0; p < PW; ++p) w[p] = 0u;
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const uint32_t v = (uint32_t)(k % (uint64_t)V);
            k /= (uint64_t)V;
            const uint32_t r = (v - 32768u) & 0xffffu;
            w[m >> 1] |= r << (16 * (m & 1));
        }
#pragma unroll
        for (int p = 0; p < PW; ++p) R[i * PW + p] = w[p];
    }
}

struct VBest {
    uint64_t num;
    uint64_t key;
    int32_t code;
    int32_t pad;
};

__device__ __forceinline__ bool vbetter(uint64_t an, uint64_t ak, int32_t ac, uint64_t bn, uint64_t bk,
                                        int32_t bc)
{
    if (an != bn) return an > bn;
    if (ak != bk) return ak < bk;
    return ac < bc;
}

// Scores the 64 origins of a group from their lane-minor counts: get(j)
// returns the (c_P, c_Q) of bin j of this lane's origin; writes the group's
// best (largest numerator, then lowest voxel key, then lowest code) to
// bb[group].  red: LDS of W * 64 * 12 bytes, which may alias the counts (it
// is written only after every wave has read its bins).
template <int D, int W, typename Get>
__device__ __forceinline__ void vfinish(Get get, uint64_t *red, const uint64_t *__restrict__ keys, int64_t M,
                                        int64_t n_p, int64_t n_q, int64_t group, VBest *__restrict__ bb)
{
    constexpr int BINS = Geo<D>::BINS;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t k = group * 64 + lane;
    const bool valid = k < M;
    uint64_t best = 0;
    int32_t bcode = 0x7fffffff;
    if (valid) {
        for (int j = w; j < BINS; j += W) {  // this wave's share of the bins
            uint64_t cp, cq;
            get(j, cp, cq);
            const int64_t sd = (int64_t)cp * n_q - (int64_t)cq * n_p;
            const uint64_t s = (uint64_t)(sd < 0 ? -sd : sd);
            const int32_t code = j ^ Geo<D>::FLIP;
            if (s > best || (s == best && code < bcode)) {
                best = s;
                bcode = code;
            }
        }
    }
    __syncthreads();
    uint64_t *sn = red;
    int32_t *sc = reinterpret_cast<int32_t *>(red + W * 64);
    sn[w * 64 + lane] = best;
    sc[w * 64 + lane] = bcode;
    __syncthreads();
    if (w == 0) {
        for (int v = 1; v < W; ++v) {
            const uint64_t n2 = sn[v * 64 + lane];
            const int32_t c2 = sc[v * 64 + lane];
            if (n2 > best || (n2 == best && c2 < bcode)) {
                best = n2;
                bcode = c2;
            }
        }
        uint64_t key = valid ? keys[k] : VOX_EMPTY;
        if (!valid) {
            best = 0;
            bcode = 0x7fffffff;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const uint64_t n2 = __shfl_xor(best, off, 64);
            const uint64_t k2 = __shfl_xor(key, off, 64);
            const int32_t c2 = __shfl_xor(bcode, off, 64);
            if (vbetter(n2, k2, c2, best, key, bcode)) {
                best = n2;
                key = k2;
                bcode = c2;
            }
        }
        if (lane == 0) {
            VBest r;
            r.num = best;
            r.key = key;
            r.code = bcode;
            r.pad = 0;
            bb[group] = r;
        }
    }
}

// Bins of the weighted sweep: 32-bit words holding c_P | c_Q << 16 when no
// bin can reach 65536 points of either sample (ds_add_u32, the faster LDS
// atomic), else 64-bit words c_P | c_Q << 32 (ds_add_u64).
template <bool WIDE>
struct VBin {
    typedef typename std::conditional<WIDE, uint64_t, uint32_t>::type T;
    typedef __attribute__((address_space(3))) T lds_t;
    static constexpr int SH = WIDE ? 9 : 8;  // log2 of the bytes of one bin row (64 lanes)
    // a voxel's increment (c_P in the low, c_Q in the high word) in this format
    __device__ static __forceinline__ T of(uint64_t v)
    {
        if constexpr (WIDE) return v;
        else return (uint32_t)v | ((uint32_t)(v >> 32) << 16);
    }
    __device__ static __forceinline__ void split(T v, uint64_t &cp, uint64_t &cq)
    {
        if constexpr (WIDE) {
            cp = (uint32_t)v;
            cq = v >> 32;
        } else {
            cp = v & 0xffffu;
            cq = v >> 16;
        }
    }
};

// The weighted sweep of one block's 64 origins over the voxels [c0, c1),
// split over the W waves, into the block's shared histogram h (lane-minor:
// bin*64 + lane, zeroed beforehand).
template <int D, int W, bool WIDE>
__device__ __forceinline__ void vsweep_range(const uint32_t *__restrict__ R, const uint64_t *__restrict__ inc,
                                             const Origin<PATH_R16, D> &org, int64_t c0, int64_t c1,
                                             typename VBin<WIDE>::T *h)
{
    typedef VBin<WIDE> B;
    typedef typename B::T T;
    typedef typename B::lds_t lds_t;
    constexpr int PW = Layout<PATH_R16, D>::PW;
    constexpr int NP = Geo<D>::NPERM;
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t per = (c1 - c0 + W - 1) / W;
    int64_t a = c0 + (int64_t)w * per, b = a + per;
    a = a < c1 ? a : c1;
    b = b < c1 ? b : c1;
    a = __builtin_amdgcn_readfirstlane((int)a);
    b = __builtin_amdgcn_readfirstlane((int)b);

    const uint32_t base = (uint32_t)(uintptr_t)(lds_t *)(h + Geo<D>::KOFF * 64 + lane);
    const uint32_t w0 = dot_wts(D, 0), w1 = dot_wts(D, 1);
    // bin addresses of a block of U voxels, and their weighted increments
    auto addrs = [&](const uint32_t (&buf)[U * PW], uint32_t (&ad)[U]) {
        uint32_t Rg[2][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint32_t r[Geo<D>::NREG];
            signs<PATH_R16, D>(buf + u * PW, org, r);
            Rg[0][u] = group_bytes<D>(r, 0);
            Rg[1][u] = NP > 1 ? group_bytes<D>(r, 1) : 0u;
        }
        addr4<NP, B::SH>(Rg, base, ad, w0, w1);
    };
    auto adds = [&](const uint32_t (&ad)[U], const uint64_t (&iv)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            __hip_atomic_fetch_add((lds_t *)(uintptr_t)ad[u], B::of(iv[u]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto load = [&](int64_t at, uint32_t (&buf)[U * PW], uint64_t (&iv)[U]) {
#pragma unroll
        for (int e = 0; e < U * PW; ++e) buf[e] = R[at * PW + e];
#pragma unroll
        for (int u = 0; u < U; ++u) iv[u] = inc[at + u];
    };
    int64_t i = a;
    int64_t nblk = b > a ? (b - a) / U : 0;
    if (nblk & 1) {  // an odd block first, so the pipelined loop runs in pairs
        uint32_t buf[U * PW], ad[U];
        uint64_t iv[U];
        load(i, buf, iv);
        addrs(buf, ad);
        adds(ad, iv);
        i += U;
        --nblk;
    }
    if (nblk > 0) {
        // The same software pipeline as the exact sweep: the scalar loads of
        // the next block go out before this block's addresses are computed,
        // and one wait per block (scalar loads and LDS atomics share its
        // counter) covers loads issued a whole block earlier.  The last
        // trip's prefetch is clamped to the last full block (in bounds).
        const int64_t last = b - U;
        uint32_t bufA[U * PW], bufB[U * PW], ad[U];
        uint64_t ivA[U], ivB[U];
        load(i, bufA, ivA);
        __builtin_amdgcn_s_waitcnt(0);
        for (int64_t t = 0; t < nblk; t += 2) {
            load(i + U, bufB, ivB);
            addrs(bufA, ad);
            wait_lgkm();
            adds(ad, ivA);
            load((i + 2 * U < last) ? i + 2 * U : last, bufA, ivA);
            addrs(bufB, ad);
            wait_lgkm();
            adds(ad, ivB);
            i += 2 * U;
        }
    }
    for (; i < b; ++i) {
        uint32_t buf[PW];
#pragma unroll
        for (int e = 0; e < PW; ++e) buf[e] = R[i * PW + e];
        uint32_t r[Geo<D>::NREG];
        signs<PATH_R16, D>(buf, org, r);
        const uint32_t R0 = group_bytes<D>(r, 0);
        const uint32_t R1 = NP > 1 ? group_bytes<D>(r, 1) : 0u;
        __hip_atomic_fetch_add((lds_t *)(uintptr_t)addr1<NP, B::SH>(R0, R1, base, w0, w1), B::of(inc[i]),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// Block (group, chunk): the 64 filled voxels group*64 + lane as origins, the
// filled voxels of chunk blockIdx.y (of gridDim.y) as weighted points, split
// over the W waves, one shared histogram (lane-minor: bin*64 + lane).  The
// block first sums its chunk's increments: when neither sample has more than
// 65535 points in the chunk, no bin can overflow 16 bits and the histogram
// takes 32-bit bins.  With one chunk the block scores its origins itself;
// otherwise it writes its counts (every bin, c_P | c_Q << 32) to
// G[chunk][group][BINS][64] and k_vscore sums the chunks.
template <int D, int W>
__global__ __launch_bounds__(W * 64) void k_vsweep(const uint32_t *__restrict__ R,
                                                   const uint64_t *__restrict__ inc,
                                                   const uint64_t *__restrict__ keys, int64_t M,
                                                   int64_t n_p, int64_t n_q, unsigned long long *__restrict__ G,
                                                   VBest *__restrict__ bb)
{
    constexpr int BINS = Geo<D>::BINS;
    extern __shared__ uint64_t h64[];
    __shared__ uint64_t tot[2 * W];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t group = blockIdx.x;
    const int64_t c0 = M * (int64_t)blockIdx.y / gridDim.y, c1 = M * ((int64_t)blockIdx.y + 1) / gridDim.y;

    // the chunk's points per sample
    uint64_t sp = 0, sq = 0;
    for (int64_t e = c0 + threadIdx.x; e < c1; e += W * 64) {
        const uint64_t v = inc[e];
        sp += (uint32_t)v;
        sq += v >> 32;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sp += __shfl_xor(sp, off, 64);
        sq += __shfl_xor(sq, off, 64);
    }
    if (lane == 0) {
        tot[2 * w] = sp;
        tot[2 * w + 1] = sq;
    }
    for (int i = threadIdx.x; i < BINS * 64; i += W * 64) h64[i] = 0;
    const int64_t k = group * 64 + lane;
    Origin<PATH_R16, D> org;
    org.load(R, k < M ? k : M - 1);
    __syncthreads();
    sp = 0;
    sq = 0;
    for (int v = 0; v < W; ++v) {
        sp += tot[2 * v];
        sq += tot[2 * v + 1];
    }
    const bool wide = __builtin_amdgcn_readfirstlane((sp > 65535u || sq > 65535u) ? 1 : 0) != 0;
    if (wide)
        vsweep_range<D, W, true>(R, inc, org, c0, c1, h64);
    else
        vsweep_range<D, W, false>(R, inc, org, c0, c1, reinterpret_cast<uint32_t *>(h64));
    __syncthreads();
    if (gridDim.y > 1) {
        unsigned long long *g = G + ((size_t)blockIdx.y * gridDim.x + group) * BINS * 64;
        const uint32_t *h32 = reinterpret_cast<const uint32_t *>(h64);
        for (int e = threadIdx.x; e < BINS * 64; e += W * 64)
            g[e] = wide ? h64[e] : ((unsigned long long)(h32[e] & 0xffffu) | ((unsigned long long)(h32[e] >> 16) << 32));
        return;
    }
    if (wide) {
        vfinish<D, W>([&](int j, uint64_t &cp, uint64_t &cq) { VBin<true>::split(h64[j * 64 + lane], cp, cq); },
                      h64, keys, M, n_p, n_q, group, bb);
    } else {
        const uint32_t *h32 = reinterpret_cast<const uint32_t *>(h64);
        vfinish<D, W>([&](int j, uint64_t &cp, uint64_t &cq) { VBin<false>::split(h32[j * 64 + lane], cp, cq); },
                      h64, keys, M, n_p, n_q, group, bb);
    }
}

// Scores group blockIdx.x from the counts of the `chunks` chunks in G.
template <int D, int W>
__global__ __launch_bounds__(W * 64) void k_vscore(const unsigned long long *__restrict__ G, int chunks,
                                                   const uint64_t *__restrict__ keys, int64_t M,
                                                   int64_t n_p, int64_t n_q, VBest *__restrict__ bb)
{
    __shared__ uint64_t red[W * 64 * 12 / 8];
    constexpr int BINS = Geo<D>::BINS;
    const int64_t group = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const size_t stride = (size_t)gridDim.x * BINS * 64;
    const unsigned long long *g = G + (size_t)group * BINS * 64 + lane;
    vfinish<D, W>(
        [&](int j, uint64_t &cp, uint64_t &cq) {
            uint64_t v = 0;
            for (int c = 0; c < chunks; ++c) v += g[c * stride + (size_t)j * 64];
            cp = (uint32_t)v;
            cq = v >> 32;
        },
        red, keys, M, n_p, n_q, group, bb);
}

__global__ __launch_bounds__(1024) void k_vreduce(const VBest *__restrict__ bb, int64_t n,
                                                  uint32_t *__restrict__ flags,
                                                  ResultDev *__restrict__ out)
{
    __shared__ uint64_t sn[16], sk[16];
    __shared__ int32_t sc[16];
    uint64_t best = 0, key = VOX_EMPTY;
    int32_t code = 0x7fffffff;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const VBest b = bb[i];
        if (vbetter(b.num, b.key, b.code, best, key, code)) {
            best = b.num;
            key = b.key;
            code = b.code;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t n2 = __shfl_xor(best, off, 64);
        const uint64_t k2 = __shfl_xor(key, off, 64);
        const int32_t c2 = __shfl_xor(code, off, 64);
        if (vbetter(n2, k2, c2, best, key, code)) {
            best = n2;
            key = k2;
            code = c2;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sn[w] = best;
        sk[w] = key;
        sc[w] = code;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < (int)(blockDim.x >> 6); ++v)
            if (vbetter(sn[v], sk[v], sc[v], best, key, code)) {
                best = sn[v];
                key = sk[v];
                code = sc[v];
            }
        out->num = best;
        out->origin = (int64_t)key;
        out->code = code;
        out->flags = *flags;
        out->ge = 0;
        *flags = 0u;
    }
}

// ---------------------------------------------------------------- host side

static unsigned grid_for(int64_t n, int per_block = 256, int64_t cap = 4096)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + per_block - 1) / per_block, cap));
}

size_t vdks_table_slots(int64_t N)
{
    size_t s = 64;
    while (s < (size_t)(2 * N)) s <<= 1;
    return s;
}

template <int D>
static hipError_t launch_vox_front_d(const float *Z, int64_t N, int64_t n_p, int V, uint32_t *mm,
                                     uint32_t *part, uint64_t *tab_key, uint32_t *tab_cnt, int64_t slots,
                                     uint32_t *counter, uint64_t *keys, uint64_t *inc, hipStream_t s)
{
    hipLaunchKernelGGL(k_vox_init, dim3(grid_for(slots)), dim3(256), 0, s, mm, D, tab_key, tab_cnt,
                       slots, counter);
    const unsigned rows = grid_for(N, 256, VOX_EXTENT_ROWS);
    hipLaunchKernelGGL(k_vox_minmax<D>, dim3(rows), dim3(256), 0, s, Z, N, part);
    hipLaunchKernelGGL(k_vox_minmax_final<D>, dim3(1), dim3(256), 0, s, part, (int)rows, mm);
    hipLaunchKernelGGL(k_vox_insert<D>, dim3(grid_for(N)), dim3(256), 0, s, Z, N, n_p, V, mm, tab_key,
                       tab_cnt, (uint64_t)(slots - 1));
    hipLaunchKernelGGL(k_vox_compact, dim3(grid_for(slots, COMPACT_THREADS, 256)), dim3(COMPACT_THREADS), 0, s,
                       tab_key, tab_cnt, slots, counter, keys, inc);
    return hipGetLastError();
}

hipError_t launch_vox_front(const float *Z, int64_t N, int64_t n_p, int d, int V, uint32_t *mm,
                            uint32_t *part, uint64_t *tab_key, uint32_t *tab_cnt, int64_t slots, uint32_t *counter,
                            uint64_t *keys, uint64_t *inc, hipStream_t s)
{
    if (slots < 2 * N || (slots & (slots - 1))) return hipErrorInvalidValue;
    switch (d) {
#define DDKS_VF(DD) \
    case DD: return launch_vox_front_d<DD>(Z, N, n_p, V, mm, part, tab_key, tab_cnt, slots, counter, keys, inc, s);
        DDKS_VF(1) DDKS_VF(2) DDKS_VF(3) DDKS_VF(4) DDKS_VF(5) DDKS_VF(6) DDKS_VF(7) DDKS_VF(8)
#undef DDKS_VF
    default: return hipErrorInvalidValue;
    }
}

size_t vsweep_lds_bytes(int d, int waves)
{
    const size_t hist = ((size_t)1 << d) * 64 * 8;
    const size_t fin = (size_t)waves * 64 * 12;
    return std::max(hist, fin);
}

// Default shape of the weighted sweep: 8 waves per block, and point chunks
// enough for about four blocks per CU when the filled voxels are few, each
// chunk at least 512 points.
VSweepPlan vsweep_default_plan(int64_t M)
{
    VSweepPlan p;
    p.waves = 8;
    const int64_t groups = (M + 63) / 64;
    int64_t c = 1;
    if (groups < 1024) {
        c = (1024 + groups - 1) / groups;
        c = std::min<int64_t>(c, std::max<int64_t>(1, M / 512));
        c = std::max<int64_t>(1, std::min<int64_t>(c, 16));
    }
    p.chunks = (int)c;
    return p;
}

bool vsweep_plan_ok(const VSweepPlan &p, int64_t M)
{
    return (p.waves == 4 || p.waves == 8 || p.waves == 16) && p.chunks >= 1 && p.chunks <= 16 &&
           p.chunks <= M;
}

size_t vsweep_partial_bytes(int64_t M, int d, const VSweepPlan &p)
{
    if (p.chunks <= 1) return 0;
    return (size_t)p.chunks * ((M + 63) / 64) * ((size_t)1 << d) * 64 * sizeof(uint64_t);
}

template <int D, int W>
static hipError_t launch_vsweep_w(const uint64_t *keys, const uint64_t *inc, int64_t M, int chunks, int64_t n_p,
                                  int64_t n_q, const uint32_t *R, void *bb, void *partial, hipStream_t s)
{
    const size_t lds = vsweep_lds_bytes(D, W);
    static std::once_flag attr;
    if (lds > 64 * 1024)
        std::call_once(attr, [] {
            if (hipFuncSetAttribute((const void *)k_vsweep<D, W>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    MAX_LDS_BYTES) != hipSuccess)
                (void)hipGetLastError();
        });
    const int64_t groups = (M + 63) / 64;
    unsigned long long *G = (unsigned long long *)partial;
    if (chunks > 1 && !G) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_vsweep<D, W>), dim3((unsigned)groups, (unsigned)chunks), dim3(W * 64), lds, s, R,
                       inc, keys, M, n_p, n_q, G, (VBest *)bb);
    if (chunks > 1)
        hipLaunchKernelGGL((k_vscore<D, W>), dim3((unsigned)groups), dim3(W * 64), 0, s, G, chunks, keys, M, n_p,
                           n_q, (VBest *)bb);
    return hipGetLastError();
}

template <int D>
static hipError_t launch_vsweep_d(const uint64_t *keys, const uint64_t *inc, int64_t M, const VSweepPlan &p,
                                  int V, int64_t n_p, int64_t n_q, uint32_t *R, void *bb, void *partial,
                                  uint32_t *flags, ResultDev *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_vox_encode<D>, dim3(grid_for(M)), dim3(256), 0, s, keys, M, V, R);
    hipError_t e;
    switch (p.waves) {
    case 4: e = launch_vsweep_w<D, 4>(keys, inc, M, p.chunks, n_p, n_q, R, bb, partial, s); break;
    case 8: e = launch_vsweep_w<D, 8>(keys, inc, M, p.chunks, n_p, n_q, R, bb, partial, s); break;
    case 16: e = launch_vsweep_w<D, 16>(keys, inc, M, p.chunks, n_p, n_q, R, bb, partial, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    const int64_t groups = (M + 63) / 64;
    hipLaunchKernelGGL(k_vreduce, dim3(1), dim3(1024), 0, s, (const VBest *)bb, groups, flags, out);
    return hipGetLastError();
}

size_t vdks_best_bytes(int64_t M) { return (size_t)((M + 63) / 64) * sizeof(VBest); }

hipError_t launch_vsweep(const uint64_t *keys, const uint64_t *inc, int64_t M, int d, int V, int64_t n_p,
                         int64_t n_q, const VSweepPlan &plan, uint32_t *R, void *bb, void *partial, uint32_t *flags,
                         ResultDev *out, hipStream_t s)
{
    if (M < 1 || M > 0x7fffffff || !vsweep_plan_ok(plan, M)) return hipErrorInvalidValue;
    switch (d) {
#define DDKS_VS(DD) \
    case DD: return launch_vsweep_d<DD>(keys, inc, M, plan, V, n_p, n_q, R, bb, partial, flags, out, s);
        DDKS_VS(1) DDKS_VS(2) DDKS_VS(3) DDKS_VS(4) DDKS_VS(5) DDKS_VS(6) DDKS_VS(7) DDKS_VS(8)
#undef DDKS_VS
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ddks
