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
// has at least twice as many slots as points, so every probe ends).  dense:
// the grid has no more voxels than the table has slots, so slot = key and a
// point is one counter increment, with no key to claim first.
template <int D>
__global__ __launch_bounds__(256) void k_vox_insert(const float *__restrict__ Z, int64_t N, int64_t n_p,
                                                    int V, const uint32_t *__restrict__ mm,
                                                    uint64_t *__restrict__ tab_key,
                                                    uint32_t *__restrict__ tab_cnt, uint64_t mask, int dense)
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
        if (dense) {
            atomicAdd(&tab_cnt[2 * key + (i < n_p ? 0 : 1)], 1u);
            continue;
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
// block take consecutive places, in slot order within the block.  dense: a
// slot is filled when either count is, and its key is its index.
static constexpr int COMPACT_THREADS = 1024;
__global__ __launch_bounds__(COMPACT_THREADS) void k_vox_compact(const uint64_t *__restrict__ tab_key,
                                                                 const uint32_t *__restrict__ tab_cnt,
                                                                 int64_t slots, int dense,
                                                                 uint32_t *__restrict__ counter,
                                                                 uint64_t *__restrict__ keys,
                                                                 uint64_t *__restrict__ inc)
{
    __shared__ uint32_t wbase[COMPACT_THREADS / 64];
    __shared__ uint32_t bbase;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t stride = (int64_t)gridDim.x * COMPACT_THREADS;
    for (int64_t h0 = (int64_t)blockIdx.x * COMPACT_THREADS; h0 < slots; h0 += stride) {
        const int64_t h = h0 + threadIdx.x;
        uint64_t k = VOX_EMPTY;
        if (h < slots) {
            if (dense)
                k = (tab_cnt[2 * h] | tab_cnt[2 * h + 1]) != 0u ? (uint64_t)h : VOX_EMPTY;
            else
                k = tab_key[h];
        }
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
// The weighted sweep's encoding of a filled voxel: the sign words of the rank
// path (two dimensions each, biased int16), STRIDE words per voxel, and
// beside them one word of counts per voxel, c_P | c_Q << 16 (meaningful when
// both fit 16 bits), which the sweep reads into vector registers.
//
// With at most 128 voxels per dimension and d <= 7 (B8) the coordinates go
// one byte each instead, four dimensions per word, each byte 128 + v: then
// for an origin o (bytes v_o) the word x - o holds 128 + v_x - v_o in each
// byte, never below 1, so no byte borrows from the next, and its top bit is
// [v_x >= v_o]; masked to those bits, one v_dot4_u32_u8 against weights
// 2^(m+1) adds 256 * (sum of 2^m over those dimensions) to the lane's bin-0
// address: the bin of orthant code j, 32-bit bins of 64 lanes.  Three vector
// instructions per voxel at d <= 4 and six at d = 5..7, against five and
// seven and a half for the int16 signs, v_perm and the address shift.
template <int D, bool B8 = false>
struct VLayout {
    static constexpr int STRIDE = B8 ? (D + 3) / 4 : Geo<D>::NREG;
    // voxels per unrolled block: a multiple of four, about 32 scalar registers
    // (8 at most in the byte encoding: 16-voxel blocks took the kernel past 64
    // VGPRs at d = 4 and past 96 SGPRs at d = 6, below 8 waves per SIMD)
    static constexpr int U0 = ((32 / STRIDE) / 4) * 4 < 4 ? 4 : ((32 / STRIDE) / 4) * 4;
    static constexpr int U = B8 && U0 > 8 ? 8 : U0;
};

constexpr int VB8_MAX_V = 128;  // voxels per dimension of the byte encoding
__host__ __device__ constexpr bool vsweep_bytes(int d, int V) { return d <= 7 && V <= VB8_MAX_V; }

// Byte weights of word q of the byte encoding: 2^(m+1) for dimension m = 4q+i.
__host__ __device__ constexpr uint32_t dot_wts8(int D, int q)
{
    uint32_t w = 0;
    for (int i = 0; i < 4; ++i) {
        const int m = 4 * q + i;
        if (m < D) w |= (2u << m) << (8 * i);
    }
    return w;
}

int vox_words(int d) { return (d + 1) / 2 + 1; }

template <int D, bool B8>
__global__ void k_vox_encode(const uint64_t *__restrict__ keys, const uint64_t *__restrict__ inc, int64_t M,
                             int V, uint32_t *__restrict__ R, uint32_t *__restrict__ W32)
{
    constexpr int S = VLayout<D, B8>::STRIDE;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[i];
        uint32_t w[S];
#pragma unroll
        for (int p = 0; p < S; ++p) w[p] = 0u;
#pragma unroll
        for (int m = 0; m < D; ++m) {
            const uint32_t v = (uint32_t)(k % (uint64_t)V);
            k /= (uint64_t)V;
            if constexpr (B8) {
                w[m >> 2] |= (v + 128u) << (8 * (m & 3));
            } else {
                const uint32_t r = (v - 32768u) & 0xffffu;
                w[m >> 1] |= r << (16 * (m & 1));
            }
        }
#pragma unroll
        for (int p = 0; p < S; ++p) R[i * S + p] = w[p];
        const uint64_t c = inc[i];
        W32[i] = ((uint32_t)c & 0xffffu) | ((uint32_t)(c >> 32) << 16);
    }
}

// Bin width of the weighted sweep's chunks: all 32-bit, all 64-bit, or per
// chunk from k_vchunk_fit.
enum : int { VFIT_NARROW = 0, VFIT_WIDE = 1, VFIT_PER_CHUNK = 2 };

// fit[c] = 1 when chunk c of the M filled voxels (chunks even in voxel count)
// holds more than 65535 points of either sample, else 0.  Block c sums its
// chunk.
__global__ __launch_bounds__(256) void k_vchunk_fit(const uint64_t *__restrict__ inc, int64_t M, int chunks,
                                                    uint32_t *__restrict__ fit)
{
    __shared__ uint64_t sp[4], sq[4];
    const int c = blockIdx.x;
    const int64_t c0 = M * c / chunks, c1 = M * (c + 1) / chunks;
    uint64_t p = 0, q = 0;
    for (int64_t e = c0 + threadIdx.x; e < c1; e += blockDim.x) {
        const uint64_t v = inc[e];
        p += (uint32_t)v;
        q += v >> 32;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        p += __shfl_xor(p, off, 64);
        q += __shfl_xor(q, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sp[threadIdx.x >> 6] = p;
        sq[threadIdx.x >> 6] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        p = sp[0] + sp[1] + sp[2] + sp[3];
        q = sq[0] + sq[1] + sq[2] + sq[3];
        fit[c] = (p > 65535u || q > 65535u) ? 1u : 0u;
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

// The lane's origin in the byte encoding, its 128 offsets removed.
template <int D>
struct VOrigin8 {
    static constexpr int S = VLayout<D, true>::STRIDE;
    uint32_t o[S];
};
template <int D, bool B8>
struct VOrgSel {
    typedef Origin<PATH_R16, D> type;
};
template <int D>
struct VOrgSel<D, true> {
    typedef VOrigin8<D> type;
};

// Loads the lane's origin, voxel k of the encoding RV.
template <int D, bool B8>
__device__ __forceinline__ void vorigin_load(typename VOrgSel<D, B8>::type &org, const uint32_t *RV, int64_t k)
{
    constexpr int S = VLayout<D, B8>::STRIDE;
    if constexpr (B8) {
#pragma unroll
        for (int p = 0; p < S; ++p) org.o[p] = RV[k * S + p] & 0x7f7f7f7fu;
    } else {
#pragma unroll
        for (int p = 0; p < Layout<PATH_R16, D>::PW; ++p) org.o[p] = p < Geo<D>::NREG ? RV[k * S + p] : 0u;
    }
}

// Bin address of one voxel x (S words) against the lane's origin: from the
// bin-0 address base in the byte encoding, from the bin-KOFF one otherwise.
template <int D, bool B8>
__device__ __forceinline__ uint32_t vaddr1(const uint32_t *x, const typename VOrgSel<D, B8>::type &org, uint32_t base)
{
    if constexpr (B8) {
        uint32_t a = base;
#pragma unroll
        for (int q = 0; q < VLayout<D, true>::STRIDE; ++q)
            a = __builtin_amdgcn_udot4((x[q] - org.o[q]) & 0x80808080u, dot_wts8(D, q), a, false);
        return a;
    } else {
        constexpr int NP = Geo<D>::NPERM;
        uint32_t r[Geo<D>::NREG];
        signs<PATH_R16, D>(x, org, r);
        const uint32_t R0 = group_bytes<D>(r, 0);
        const uint32_t R1 = NP > 1 ? group_bytes<D>(r, 1) : 0u;
        return addr1<NP>(R0, R1, base, dot_wts(D, 0), dot_wts(D, 1));
    }
}

// Bin addresses (32-bit bins) of U consecutive voxels of the encoding held in
// buf (stride VLayout<D, B8>::STRIDE words), as block_addrs computes them for
// points of the rank path.
template <int D, int U, bool B8>
__device__ __forceinline__ void vblock_addrs(const uint32_t *buf, const typename VOrgSel<D, B8>::type &org,
                                             uint32_t base, uint32_t (&a)[U])
{
    constexpr int S = VLayout<D, B8>::STRIDE;
    if constexpr (B8) {
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = vaddr1<D, true>(buf + u * S, org, base);
    } else {
        constexpr int NP = Geo<D>::NPERM;
        const uint32_t w0 = dot_wts(D, 0), w1 = dot_wts(D, 1);
#pragma unroll
        for (int g = 0; g < U; g += 4) {
            uint32_t R[2][4];
            uint32_t q[4];
            if constexpr (D == 5 || D == 6) {
                // one v_perm serves the second groups of two voxels (dimensions 4, 5)
                constexpr uint32_t SEL = D == 6 ? 0x0b0a0908u : 0x0c0a0c08u;
#pragma unroll
                for (int u = 0; u < 4; u += 2) {
                    uint32_t r0[Geo<D>::NREG], r1[Geo<D>::NREG];
                    signs<PATH_R16, D>(buf + (g + u) * S, org, r0);
                    signs<PATH_R16, D>(buf + (g + u + 1) * S, org, r1);
                    R[0][u] = group_bytes<D>(r0, 0);
                    R[0][u + 1] = group_bytes<D>(r1, 0);
                    R[1][u] = R[1][u + 1] = __builtin_amdgcn_perm(r1[2], r0[2], SEL);
                }
                addr4_w2(R, base, q, w0, w1, w1 << 16);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    uint32_t r[Geo<D>::NREG];
                    signs<PATH_R16, D>(buf + (g + u) * S, org, r);
                    R[0][u] = group_bytes<D>(r, 0);
                    R[1][u] = NP > 1 ? group_bytes<D>(r, 1) : 0u;
                }
                addr4<NP>(R, base, q, w0, w1);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) a[g + u] = q[u];
        }
    }
}

// Voxels [lo, hi) of the encoding RV against the lane's G origins (one per
// origin group, histogram j at base[j]) into 32-bit bins (c_P | c_Q << 16,
// each voxel's counts word W32[i] as its increment): the exact sweep's
// software pipeline over blocks of VLayout<D, B8>::U voxels, each block's
// loads serving all G origin groups.  The coordinate words come through scalar loads;
// the counts words through vector loads from an address the compiler must
// treat as per-lane, so that they land in vector registers, where the LDS
// atomics take their data, without a move per voxel.
template <int D, int G, bool B8>
__device__ __forceinline__ void vsweep_narrow(const uint32_t *__restrict__ RV, const uint32_t *__restrict__ W32,
                                              int64_t lo, int64_t hi,
                                              const typename VOrgSel<D, B8>::type (&org)[G],
                                              const uint32_t (&base)[G])
{
    constexpr int S = VLayout<D, B8>::STRIDE;
    constexpr int U = VLayout<D, B8>::U;
    // the same address in every lane, held in vector registers (a global
    // pointer: global loads count only against the vector-memory counter, so
    // the waits for the scalar loads and LDS atomics do not include them)
    typedef const __attribute__((address_space(1))) uint32_t gu32;
    uint64_t wv = (uint64_t)(uintptr_t)W32;
    asm volatile("" : "+v"(wv));
    gu32 *Wv = (gu32 *)(uintptr_t)wv;
    auto block = [&](const uint32_t (&buf)[U * S], uint32_t (&a)[G][U]) {
#pragma unroll
        for (int j = 0; j < G; ++j) vblock_addrs<D, U, B8>(buf, org[j], base[j], a[j]);
    };
    auto adds = [&](const uint32_t (&wt)[U], const uint32_t (&a)[G][U]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < G; ++j) lds_add(a[j][u], wt[u]);
    };
    int64_t i = lo;
    int64_t nblk = hi > lo ? (hi - lo) / U : 0;
    if (nblk & 1) {  // an odd block first, so the pipelined loop runs in pairs
        uint32_t buf[U * S], wt[U], a[G][U];
#pragma unroll
        for (int e = 0; e < U * S; ++e) buf[e] = RV[i * S + e];
#pragma unroll
        for (int u = 0; u < U; ++u) wt[u] = Wv[i + u];
        block(buf, a);
        adds(wt, a);
        i += U;
        --nblk;
    }
    if (nblk > 0) {
        const int64_t last = hi - U;
        uint32_t bufA[U * S], bufB[U * S], wA[U], wB[U];
#pragma unroll
        for (int e = 0; e < U * S; ++e) bufA[e] = RV[i * S + e];
#pragma unroll
        for (int u = 0; u < U; ++u) wA[u] = Wv[i + u];
        __builtin_amdgcn_s_waitcnt(0);
        for (int64_t t = 0; t < nblk; t += 2) {
#pragma unroll
            for (int e = 0; e < U * S; ++e) bufB[e] = RV[(i + U) * S + e];
#pragma unroll
            for (int u = 0; u < U; ++u) wB[u] = Wv[i + U + u];
            uint32_t a[G][U];
            block(bufA, a);
            wait_lgkm();
            adds(wA, a);
            const int64_t na = (i + 2 * U < last) ? i + 2 * U : last;
#pragma unroll
            for (int e = 0; e < U * S; ++e) bufA[e] = RV[na * S + e];
#pragma unroll
            for (int u = 0; u < U; ++u) wA[u] = Wv[na + u];
            block(bufB, a);
            wait_lgkm();
            adds(wB, a);
            i += 2 * U;
        }
    }
    for (; i < hi; ++i) {
        uint32_t buf[S];
#pragma unroll
        for (int e = 0; e < S; ++e) buf[e] = RV[i * S + e];
        const uint32_t wt = Wv[i];
#pragma unroll
        for (int j = 0; j < G; ++j) lds_add(vaddr1<D, B8>(buf, org[j], base[j]), wt);
    }
}

// The same for a chunk with more than 65535 points of a sample, one sample at
// a time: 32-bit bins of that sample's counts alone (half = 0: c_P, the low
// word of each voxel's increment; 1: c_Q, the high word), one origin group.
template <int D, bool B8>
__device__ __forceinline__ void vsweep_one_sample(const uint32_t *__restrict__ RV, const uint64_t *__restrict__ inc,
                                                  int half, int64_t lo, int64_t hi,
                                                  const typename VOrgSel<D, B8>::type &org, uint32_t base)
{
    constexpr int S = VLayout<D, B8>::STRIDE;
    for (int64_t i = lo; i < hi; ++i) {
        uint32_t buf[S];
#pragma unroll
        for (int e = 0; e < S; ++e) buf[e] = RV[i * S + e];
        const uint32_t c = (uint32_t)(inc[i] >> (32 * half));
        if (c) lds_add(vaddr1<D, B8>(buf, org, base), c);
    }
}

// LDS bytes of the weighted sweep's block: H histograms of 2^d 32-bit bins x
// 64 lanes (H = G, or 2 for a single chunk too heavy for one-pass bins: one
// histogram per sample); the scoring's reduction space (W x 64 x 12 bytes)
// reuses them.
__host__ __device__ constexpr size_t vsweep_lds(int d, int waves, int H)
{
    return (size_t)H * ((size_t)1 << d) * 64 * 4 > (size_t)waves * 64 * 12 ? (size_t)H * ((size_t)1 << d) * 64 * 4
                                                                           : (size_t)waves * 64 * 12;
}

// Block (G origin groups, chunk): the filled voxels (blockIdx.x * G + j) *
// 64 + lane as origins, the filled voxels of chunk blockIdx.y (of gridDim.y)
// as weighted points, split over the W waves, one shared histogram of 32-bit
// bins per origin group (lane-minor: bin*64 + lane).  A chunk that holds at
// most 65535 points of each sample adds both samples' counts at once
// (c_P | c_Q << 16).  Heavier chunks add one sample at a time: with several
// chunks (mode VFIT_PER_CHUNK, where fit[chunk] is set) each sample's pass
// goes through the partial sums; a single chunk (mode VFIT_WIDE, G = 1) keeps
// one histogram per sample.  With part null the block scores its origins
// itself; otherwise it stores its counts as its chunk's rows of the partial
// counts (plain stores: every entry of every row is written) and k_vscore
// sums the chunks and scores them.  B8: the byte encoding (VLayout).
template <int D, int W, int G, bool B8>
__global__ __launch_bounds__(W * 64) void k_vsweep(const uint32_t *__restrict__ RV,
                                                   const uint32_t *__restrict__ W32,
                                                   const uint64_t *__restrict__ inc,
                                                   const uint64_t *__restrict__ keys, int64_t M,
                                                   int64_t n_p, int64_t n_q, int mode,
                                                   const uint32_t *__restrict__ fit,
                                                   uint32_t *__restrict__ part, VBest *__restrict__ bb)
{
    constexpr int HB = Geo<D>::BINS * 64;  // bins of one histogram
    extern __shared__ uint32_t h32[];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t groups = (M + 63) / 64;
    const bool wide =
        mode == VFIT_WIDE || (mode == VFIT_PER_CHUNK && __builtin_amdgcn_readfirstlane(fit[blockIdx.y]) != 0u);

    for (int i = threadIdx.x; i < (mode == VFIT_WIDE ? 2 : G) * HB; i += W * 64) h32[i] = 0;
    typename VOrgSel<D, B8>::type org[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const int64_t k = ((int64_t)blockIdx.x * G + j) * 64 + lane;
        vorigin_load<D, B8>(org[j], RV, k < M ? k : M - 1);
    }
    // the address a voxel's code is added to: bin 0 in the byte encoding,
    // bin KOFF for the int16 signs' negative dot sums
    constexpr int B0 = B8 ? 0 : Geo<D>::KOFF;
    uint32_t base[G];
#pragma unroll
    for (int j = 0; j < G; ++j) base[j] = (uint32_t)(uintptr_t)(lds_u32 *)(h32 + (size_t)j * HB + B0 * 64 + lane);
    __syncthreads();

    const int64_t c0 = M * (int64_t)blockIdx.y / gridDim.y, c1 = M * ((int64_t)blockIdx.y + 1) / gridDim.y;
    const int64_t per = (c1 - c0 + W - 1) / W;
    int64_t a = c0 + (int64_t)w * per, b = a + per;
    a = a < c1 ? a : c1;
    b = b < c1 ? b : c1;
    a = __builtin_amdgcn_readfirstlane((int)a);
    b = __builtin_amdgcn_readfirstlane((int)b);

    if (mode == VFIT_WIDE) {
        // one chunk (G = 1): c_P into the first histogram, c_Q into the second
        vsweep_one_sample<D, B8>(RV, inc, 0, a, b, org[0], base[0]);
        vsweep_one_sample<D, B8>(RV, inc, 1, a, b, org[0], base[0] + HB * 4);
        __syncthreads();
        if (blockIdx.x < groups)
            vfinish<D, W>(
                [&](int jb, uint64_t &cp, uint64_t &cq) {
                    cp = h32[jb * 64 + lane];
                    cq = h32[HB + jb * 64 + lane];
                },
                reinterpret_cast<uint64_t *>(h32), keys, M, n_p, n_q, blockIdx.x, bb);
        return;
    }
    // this chunk's rows of the partial counts: [chunk][group][bin][lane]
    // words, c_P | c_Q << 16 from a one-pass chunk, else c_P here and c_Q in
    // the second plane (gridDim.y chunks further on)
    const size_t plane = (size_t)gridDim.y * groups * HB;
    if (wide) {
        // one sample per pass, each pass's counts stored in its own plane
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            if (half) {
                __syncthreads();
                for (int i = threadIdx.x; i < G * HB; i += W * 64) h32[i] = 0;
                __syncthreads();
            }
#pragma unroll
            for (int j = 0; j < G; ++j) vsweep_one_sample<D, B8>(RV, inc, half, a, b, org[j], base[j]);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int64_t group = (int64_t)blockIdx.x * G + j;
                if (group >= groups) break;  // block-uniform
                uint32_t *g = part + half * plane + ((size_t)blockIdx.y * groups + group) * HB;
                for (int e = threadIdx.x; e < HB; e += W * 64) g[e] = h32[(size_t)j * HB + e];
            }
        }
        return;
    }
    vsweep_narrow<D, G, B8>(RV, W32, a, b, org, base);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < G; ++j) {
        const int64_t group = (int64_t)blockIdx.x * G + j;
        if (group >= groups) break;  // block-uniform
        if (part) {
            uint32_t *g = part + ((size_t)blockIdx.y * groups + group) * HB;
            for (int e = threadIdx.x; e < HB; e += W * 64) g[e] = h32[(size_t)j * HB + e];
        } else {
            // vfinish reads every bin of histogram j before it writes its
            // reduction space over the start of the histograms; the later
            // groups' histograms lie beyond that space (checked on the host)
            vfinish<D, W>(
                [&](int jb, uint64_t &cp, uint64_t &cq) {
                    const uint32_t v = h32[(size_t)j * HB + jb * 64 + lane];
                    cp = v & 0xffffu;
                    cq = v >> 16;
                },
                reinterpret_cast<uint64_t *>(h32), keys, M, n_p, n_q, group, bb);
        }
    }
}

// Scores group blockIdx.x from the chunks' rows of the partial counts
// (fit non-null: fit[chunk] set for a chunk stored in two planes, else every
// chunk one-pass).  Each bin's rows of all chunks are loaded together (MC >=
// chunks rows, clamped to the last chunk past `chunks`, whose repeats are
// dropped), so a bin costs one memory latency whatever the chunk count; the
// second plane is read only when some chunk of the launch was stored in two.
template <int D, int W, int MC>
__global__ __launch_bounds__(W * 64) void k_vscore(const uint32_t *__restrict__ part, int chunks,
                                                   const uint32_t *__restrict__ fit,
                                                   const uint64_t *__restrict__ keys, int64_t M,
                                                   int64_t n_p, int64_t n_q, VBest *__restrict__ bb)
{
    __shared__ uint64_t red[W * 64 * 12 / 8];
    constexpr int BINS = Geo<D>::BINS;
    constexpr int HB = BINS * 64;
    const int lane = threadIdx.x & 63;
    const int64_t groups = gridDim.x;
    const size_t row = (size_t)groups * HB;  // one chunk's rows
    const size_t plane = (size_t)chunks * row;
    uint32_t wide = 0;  // chunks stored in two planes
    if (fit)
        for (int c = 0; c < chunks; ++c) wide |= (fit[c] != 0u ? 1u : 0u) << c;
    wide = __builtin_amdgcn_readfirstlane(wide);
    const uint32_t *g = part + (size_t)blockIdx.x * HB + lane;
    vfinish<D, W>(
        [&](int j, uint64_t &cp, uint64_t &cq) {
            uint32_t v[MC];
#pragma unroll
            for (int c = 0; c < MC; ++c) v[c] = g[(size_t)(c < chunks ? c : chunks - 1) * row + (size_t)j * 64];
            uint32_t sp = 0, sq = 0;
            if (wide) {
                uint32_t q[MC];
#pragma unroll
                for (int c = 0; c < MC; ++c)
                    q[c] = g[plane + (size_t)(c < chunks ? c : chunks - 1) * row + (size_t)j * 64];
#pragma unroll
                for (int c = 0; c < MC; ++c) {
                    const bool on = c < chunks, two = (wide >> c) & 1u;
                    sp += on ? (two ? v[c] : (v[c] & 0xffffu)) : 0u;
                    sq += on ? (two ? q[c] : (v[c] >> 16)) : 0u;
                }
            } else {
#pragma unroll
                for (int c = 0; c < MC; ++c) {
                    const bool on = c < chunks;
                    sp += on ? (v[c] & 0xffffu) : 0u;
                    sq += on ? (v[c] >> 16) : 0u;
                }
            }
            cp = sp;
            cq = sq;
        },
        red, keys, M, n_p, n_q, blockIdx.x, bb);
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

// Whether V^d voxels fit the table's slots, so that the key can be the slot.
static bool vox_dense(int d, int V, int64_t slots)
{
    uint64_t cells = 1;
    for (int m = 0; m < d; ++m) {
        cells *= (uint64_t)V;
        if (cells > (uint64_t)slots) return false;
    }
    return true;
}

template <int D>
static hipError_t launch_vox_front_d(const float *Z, int64_t N, int64_t n_p, int V, uint32_t *mm,
                                     uint32_t *part, uint64_t *tab_key, uint32_t *tab_cnt, int64_t slots,
                                     uint32_t *counter, uint64_t *keys, uint64_t *inc, hipStream_t s)
{
    const int dense = vox_dense(D, V, slots) ? 1 : 0;
    hipLaunchKernelGGL(k_vox_init, dim3(grid_for(slots)), dim3(256), 0, s, mm, D, tab_key, tab_cnt,
                       slots, counter);
    const unsigned rows = grid_for(N, 256, VOX_EXTENT_ROWS);
    hipLaunchKernelGGL(k_vox_minmax<D>, dim3(rows), dim3(256), 0, s, Z, N, part);
    hipLaunchKernelGGL(k_vox_minmax_final<D>, dim3(1), dim3(256), 0, s, part, (int)rows, mm);
    hipLaunchKernelGGL(k_vox_insert<D>, dim3(grid_for(N)), dim3(256), 0, s, Z, N, n_p, V, mm, tab_key,
                       tab_cnt, (uint64_t)(slots - 1), dense);
    hipLaunchKernelGGL(k_vox_compact, dim3(grid_for(slots, COMPACT_THREADS, 256)), dim3(COMPACT_THREADS), 0, s,
                       tab_key, tab_cnt, slots, dense, counter, keys, inc);
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


// Default shape of the weighted sweep: 8 waves per block, and point chunks
// enough for about four blocks per CU when the filled voxels are few, each
// chunk at least 512 voxels.
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

static int vsweep_mode(const VSweepPlan &p, int64_t n_p, int64_t n_q)
{
    if (n_p <= 65535 && n_q <= 65535) return VFIT_NARROW;
    return p.chunks == 1 ? VFIT_WIDE : VFIT_PER_CHUNK;
}

bool vsweep_plan_ok(const VSweepPlan &p, int64_t M, int d)
{
    // with two groups scored in the block, the reduction space (at the start
    // of the histograms) must leave the second group's histogram alone
    const size_t hist = ((size_t)1 << d) * 64 * 4, red = (size_t)p.waves * 64 * 12;
    return (p.waves == 4 || p.waves == 8 || p.waves == 16) && (p.per_block == 1 || p.per_block == 2) &&
           p.chunks >= 1 && p.chunks <= VSWEEP_MAX_CHUNKS && p.chunks <= M &&
           vsweep_lds(d, p.waves, 2) <= (size_t)MAX_LDS_BYTES && (p.per_block == 1 || red <= hist);
}

bool vsweep_uses_bytes(int d, int V) { return vsweep_bytes(d, V); }

size_t vsweep_partial_bytes(int64_t M, int d, const VSweepPlan &p)
{
    if (p.chunks <= 1) return 0;
    // two planes of [chunk][group][bin][lane] words (the second for the c_Q
    // of chunks too heavy for one pass)
    return 2 * (size_t)p.chunks * (size_t)((M + 63) / 64) * ((size_t)1 << d) * 64 * sizeof(uint32_t);
}

template <int D, int W, int G, bool B8>
static hipError_t launch_vsweep_w(const uint64_t *keys, const uint64_t *inc, int64_t M, int chunks, int64_t n_p,
                                  int64_t n_q, const uint32_t *RV, const uint32_t *W32, int mode, const uint32_t *fit, void *bb,
                                  void *partial, hipStream_t s)
{
    const size_t lds = vsweep_lds(D, W, mode == VFIT_WIDE ? 2 : G);
    if (lds > (size_t)MAX_LDS_BYTES || (mode == VFIT_WIDE && (G != 1 || chunks != 1))) return hipErrorInvalidValue;
    static std::once_flag attr;
    if (lds > 64 * 1024)
        std::call_once(attr, [] {
            if (hipFuncSetAttribute((const void *)k_vsweep<D, W, G, B8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    MAX_LDS_BYTES) != hipSuccess)
                (void)hipGetLastError();
        });
    const int64_t groups = (M + 63) / 64;
    // the partial counts take the chunks' counts; a single chunk scores in the block
    const bool via_partial = chunks > 1;
    uint32_t *Pp = via_partial ? (uint32_t *)partial : nullptr;
    if (via_partial && !Pp) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_vsweep<D, W, G, B8>), dim3((unsigned)((groups + G - 1) / G), (unsigned)chunks), dim3(W * 64),
                       lds, s, RV, W32, inc, keys, M, n_p, n_q, mode, fit, Pp, (VBest *)bb);
    if (via_partial) {
        const uint32_t *f = mode == VFIT_PER_CHUNK ? fit : nullptr;
        if (chunks <= 4)
            hipLaunchKernelGGL((k_vscore<D, W, 4>), dim3((unsigned)groups), dim3(W * 64), 0, s, (const uint32_t *)Pp,
                               chunks, f, keys, M, n_p, n_q, (VBest *)bb);
        else if (chunks <= 8)
            hipLaunchKernelGGL((k_vscore<D, W, 8>), dim3((unsigned)groups), dim3(W * 64), 0, s, (const uint32_t *)Pp,
                               chunks, f, keys, M, n_p, n_q, (VBest *)bb);
        else
            hipLaunchKernelGGL((k_vscore<D, W, VSWEEP_MAX_CHUNKS>), dim3((unsigned)groups), dim3(W * 64), 0, s,
                               (const uint32_t *)Pp, chunks, f, keys, M, n_p, n_q, (VBest *)bb);
    }
    return hipGetLastError();
}

template <int D, int W, bool B8>
static hipError_t launch_vsweep_g(int G, const uint64_t *keys, const uint64_t *inc, int64_t M, int chunks,
                                  int64_t n_p, int64_t n_q, const uint32_t *RV, const uint32_t *W32, int mode, const uint32_t *fit,
                                  void *bb, void *partial, hipStream_t s)
{
    if (G == 2 && mode != VFIT_WIDE)
        return launch_vsweep_w<D, W, 2, B8>(keys, inc, M, chunks, n_p, n_q, RV, W32, mode, fit, bb, partial, s);
    return launch_vsweep_w<D, W, 1, B8>(keys, inc, M, chunks, n_p, n_q, RV, W32, mode, fit, bb, partial, s);
}

template <int D, bool B8>
static hipError_t launch_vsweep_e(const uint64_t *keys, const uint64_t *inc, int64_t M, const VSweepPlan &p,
                                  int V, int64_t n_p, int64_t n_q, uint32_t *RV, const uint32_t *fitp, int mode,
                                  void *bb, void *partial, hipStream_t s)
{
    // the counts words follow the M voxels' coordinate words
    uint32_t *W32 = RV + M * VLayout<D, B8>::STRIDE;
    hipLaunchKernelGGL((k_vox_encode<D, B8>), dim3(grid_for(M)), dim3(256), 0, s, keys, inc, M, V, RV, W32);
    switch (p.waves) {
    case 4: return launch_vsweep_g<D, 4, B8>(p.per_block, keys, inc, M, p.chunks, n_p, n_q, RV, W32, mode, fitp, bb, partial, s);
    case 8: return launch_vsweep_g<D, 8, B8>(p.per_block, keys, inc, M, p.chunks, n_p, n_q, RV, W32, mode, fitp, bb, partial, s);
    case 16: return launch_vsweep_g<D, 16, B8>(p.per_block, keys, inc, M, p.chunks, n_p, n_q, RV, W32, mode, fitp, bb, partial, s);
    default: return hipErrorInvalidValue;
    }
}

template <int D>
static hipError_t launch_vsweep_d(const uint64_t *keys, const uint64_t *inc, int64_t M, const VSweepPlan &p,
                                  int V, int64_t n_p, int64_t n_q, uint32_t *RV, uint32_t *fit, void *bb,
                                  void *partial, uint32_t *flags, ResultDev *out, hipStream_t s)
{
    // chunks of more than 65535 points of a sample cannot take the one-pass
    // bins: with both samples that small no chunk can hold so many; a single
    // chunk holds them all
    const uint32_t *fitp = nullptr;
    const int mode = vsweep_mode(p, n_p, n_q);
    if (mode == VFIT_PER_CHUNK) {
        hipLaunchKernelGGL(k_vchunk_fit, dim3((unsigned)p.chunks), dim3(256), 0, s, inc, M, p.chunks, fit);
        fitp = fit;
    }
    hipError_t e;
    if constexpr (D <= 7) {
        if (vsweep_bytes(D, V))
            e = launch_vsweep_e<D, true>(keys, inc, M, p, V, n_p, n_q, RV, fitp, mode, bb, partial, s);
        else
            e = launch_vsweep_e<D, false>(keys, inc, M, p, V, n_p, n_q, RV, fitp, mode, bb, partial, s);
    } else {
        e = launch_vsweep_e<D, false>(keys, inc, M, p, V, n_p, n_q, RV, fitp, mode, bb, partial, s);
    }
    if (e != hipSuccess) return e;
    const int64_t groups = (M + 63) / 64;
    hipLaunchKernelGGL(k_vreduce, dim3(1), dim3(1024), 0, s, (const VBest *)bb, groups, flags, out);
    return hipGetLastError();
}

size_t vdks_best_bytes(int64_t M) { return (size_t)((M + 63) / 64) * sizeof(VBest); }

hipError_t launch_vsweep(const uint64_t *keys, const uint64_t *inc, int64_t M, int d, int V, int64_t n_p,
                         int64_t n_q, const VSweepPlan &plan, uint32_t *RV, uint32_t *fit, void *bb, void *partial,
                         uint32_t *flags, ResultDev *out, hipStream_t s)
{
    if (M < 1 || M > 0x7fffffff || !vsweep_plan_ok(plan, M, d)) return hipErrorInvalidValue;
    switch (d) {
#define DDKS_VS(DD) \
    case DD: return launch_vsweep_d<DD>(keys, inc, M, plan, V, n_p, n_q, RV, fit, bb, partial, flags, out, s);
        DDKS_VS(1) DDKS_VS(2) DDKS_VS(3) DDKS_VS(4) DDKS_VS(5) DDKS_VS(6) DDKS_VS(7) DDKS_VS(8)
#undef DDKS_VS
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ddks
