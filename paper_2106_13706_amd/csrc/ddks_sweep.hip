// gfx950 kernels for the exact ddKS orthant-counting sweep (arXiv:2106.13706,
// Sec. 2.1 Eq. ddks_tensor_definition, Eq. g, Eq. membership, Eq. d1).
//
// Work decomposition: one origin per lane, 64 origins per wave; every wave of
// a block holds the same 64 origins and sweeps its own share of the points
// (an equal part of the chunk's first-sample points and of its second-sample
// points).  The block's waves add into H shared LDS histograms (wave w into
// histogram w mod H; LDS atomics are atomic across waves), H chosen by the
// host as the smallest power of two that keeps every per-sample counter of a
// histogram within 16 bits, so usually one histogram serves the whole block
// and the LDS a block needs does not grow with its wave count.  Only the
// block's result leaves the CU.  Points are read with wave-uniform (scalar) loads straight into
// SGPRs, so a point costs no VGPR traffic; each lane compares it with its own
// origin:
//
//   fp32 path: v_sub_f32 (x - o) is exact in sign: zero only when x == o,
//              and then +0 (-0 was mapped to +0 on ingest; subnormals are
//              kept: the kernels run with fp32 denormals preserved);
//              v_cvt_pkrtz_f16_f32 packs the signs of two differences into
//              bits 15 and 31 of one register (rounding toward zero never
//              flips a sign).
//   rank path: coordinates replaced by per-dimension dense ranks biased to
//              int16, two dimensions per word; v_pk_sub_i16 with saturation
//              gives both signs in one instruction.
//
// v_perm_b32 gathers four sign bits into sign-filled bytes (0xff where
// x_m < o_m), v_dot4_i32_i8 against per-dimension weights turns them into
// -(sum of 2^m over the dimensions where x_m < o_m), and one v_lshl_add forms
// the LDS address of the orthant bin.  Histograms are lane-minor
// (bin * 64 + lane), so a ds_add_u32 from a wave touches 64 distinct banks
// slots whatever the codes are.  Counts of both samples share one 32-bit
// counter: +1 for a point of P, +65536 for a point of Q (no histogram ever
// receives more than 65535 points of either sample).
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>

#include "ddks_device.h"

namespace ddks {

// Block finish: thread (wave w, lane) owns bins j = w, w+W, ... of origin
// group*64+lane; get(j) returns its (c_P, c_Q).  Scores every bin, writes the
// counts if requested, reduces to the block's best.  scratch: >= W*64*16 bytes.
template <int D, int W, typename Get>
__device__ __forceinline__ void finish_block(Get get, int64_t group, int64_t N, int64_t n_p,
                                             int64_t n_q, BlockBest *block_best,
                                             uint32_t *counts, uint32_t *scratch)
{
    constexpr int BINS = Geo<D>::BINS;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t k = group * 64 + lane;
    const bool valid = k < N;
    uint64_t best = 0;
    int32_t bcode = 0x7fffffff;
    for (int j = w; j < BINS; j += W) {
        uint2 c = get(j);
        const int code = j ^ Geo<D>::FLIP;
        uint64_t s = score(c.x, c.y, n_p, n_q);
        if (s > best || (s == best && code < bcode)) {
            best = s;
            bcode = code;
        }
        if (counts && valid) {
            *reinterpret_cast<uint2 *>(counts + ((size_t)k * BINS + code) * 2) = c;
        }
    }
    __syncthreads();  // every read of the histograms is done; scratch may alias them
    uint64_t *sn = reinterpret_cast<uint64_t *>(scratch);
    int32_t *sc = reinterpret_cast<int32_t *>(scratch + 2 * W * 64);
    sn[w * 64 + lane] = best;
    sc[w * 64 + lane] = bcode;
    __syncthreads();
    if (w == 0) {
        for (int v = 1; v < W; ++v) {
            uint64_t n2 = sn[v * 64 + lane];
            int32_t c2 = sc[v * 64 + lane];
            if (n2 > best || (n2 == best && c2 < bcode)) {
                best = n2;
                bcode = c2;
            }
        }
        uint32_t org = valid ? (uint32_t)k : 0xffffffffu;
        if (!valid) {
            best = 0;
            bcode = 0x7fffffff;
        }
        wave_best(best, org, bcode);
        if (lane == 0) {
            BlockBest bb;
            bb.num = best;
            bb.origin = org;
            bb.code = bcode;
            block_best[group] = bb;
        }
    }
}

// One block of the sweep: origins group*64 .. group*64+63 against the points
// of chunk `chunk` (of nchunks), split across the W waves, which add into
// `hists` LDS histograms (1 <= hists <= W, a power of two).  With nchunks == 1
// the block scores in place and writes block_best[group] (and counts);
// otherwise it writes its partial counts: one uint32 (c_P | c_Q << 16) per
// entry when a chunk holds at most 65535 points, else a uint2.
template <int D, int PATH, int W>
__device__ __forceinline__ void sweep_block(const void *__restrict__ Zv, int64_t N, int64_t n_p,
                                            int64_t n_q, int64_t chunk_len, int64_t chunk,
                                            int64_t nchunks, int64_t group, int64_t groups,
                                            int hists, void *__restrict__ partial,
                                            BlockBest *__restrict__ block_best,
                                            uint32_t *__restrict__ counts, uint32_t *smem)
{
    typedef typename Layout<PATH, D>::T T;
    constexpr int BINS = Geo<D>::BINS;
    const T *__restrict__ Z = static_cast<const T *>(Zv);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int H = __builtin_amdgcn_readfirstlane(hists);

    constexpr bool PAIRS = PairGeo<D>::ON;
    constexpr int SLOTS = PAIRS ? PairGeo<D>::SLOTS : BINS;  // 32-bit words per lane per histogram
    for (int i = threadIdx.x; i < H * SLOTS * 64; i += W * 64) smem[i] = 0;

    int64_t k = group * 64 + lane;
    Origin<PATH, D> org;
    org.load(Z, k < N ? k : N - 1);
    __syncthreads();

    // This wave's shares of the chunk's points of P and of Q.
    const int64_t c0 = chunk * chunk_len;
    const int64_t c1 = (c0 + chunk_len < N) ? c0 + chunk_len : N;
    const int64_t p1 = c1 < n_p ? c1 : n_p;      // P part: [c0, p1)
    const int64_t q0 = c0 > n_p ? c0 : n_p;      // Q part: [q0, c1)
    const int64_t np_c = p1 > c0 ? p1 - c0 : 0;
    const int64_t nq_c = c1 > q0 ? c1 - q0 : 0;
    const int64_t perp = (np_c + W - 1) / W, perq = (nq_c + W - 1) / W;
    int64_t pa = (int64_t)w * perp, pb = pa + perp;
    int64_t qa = (int64_t)w * perq, qb = qa + perq;
    pa = pa < np_c ? pa : np_c;
    pb = pb < np_c ? pb : np_c;
    qa = qa < nq_c ? qa : nq_c;
    qb = qb < nq_c ? qb : nq_c;
    // keep the ranges in SGPRs (each share is < 2^31 points)
    pa = __builtin_amdgcn_readfirstlane((int)pa) + c0;
    pb = __builtin_amdgcn_readfirstlane((int)pb) + c0;
    qa = __builtin_amdgcn_readfirstlane((int)qa) + q0;
    qb = __builtin_amdgcn_readfirstlane((int)qb) + q0;

    const int hist = w & (H - 1);
    if constexpr (PAIRS) {
        const uint32_t pbase =
            (uint32_t)(uintptr_t)(lds_u32 *)(smem + (hist * SLOTS + PairGeo<D>::PKOFF) * 64 + lane);
        const uint32_t sbase = (uint32_t)(uintptr_t)(lds_u32 *)(
            smem + (hist * SLOTS + PairGeo<D>::PBINS + Geo<D>::KOFF) * 64 + lane);
        sweep_range_pairs<PATH, D>(Z, pa, pb, org, pbase, sbase, 1u);
        sweep_range_pairs<PATH, D>(Z, qa, qb, org, pbase, sbase, 0x10000u);
    } else {
        const uint32_t base =
            (uint32_t)(uintptr_t)(lds_u32 *)(smem + (hist * BINS + Geo<D>::KOFF) * 64 + lane);
        sweep_range<PATH, D>(Z, pa, pb, org, base, 1u);
        sweep_range<PATH, D>(Z, qa, qb, org, base, 0x10000u);
    }
    __syncthreads();

    // (c_P, c_Q) of orthant j: with pair tables, the row of j (j first in the
    // pair), its column (j second; the diagonal bin counts two points of j),
    // and the single-point bin.
    auto get = [&](int j) {
        uint32_t cp = 0, cq = 0;
        for (int v = 0; v < H; ++v) {
            if constexpr (PAIRS) {
                constexpr int F = PairGeo<D>::PFLIP;
                const uint32_t *t = smem + v * SLOTS * 64 + lane;
#pragma unroll
                for (int k = 0; k < BINS; ++k) {
                    const uint32_t r = t[((j * BINS + k) ^ F) * 64], c = t[((k * BINS + j) ^ F) * 64];
                    cp += (r & 0xffffu) + (c & 0xffffu);
                    cq += (r >> 16) + (c >> 16);
                }
                const uint32_t h = t[(PairGeo<D>::PBINS + j) * 64];
                cp += h & 0xffffu;
                cq += h >> 16;
            } else {
                uint32_t h = smem[(v * BINS + j) * 64 + lane];
                cp += h & 0xffffu;
                cq += h >> 16;
            }
        }
        return make_uint2(cp, cq);
    };
    if (nchunks == 1) {
        finish_block<D, W>(get, group, N, n_p, n_q, block_best, counts, smem);
    } else if (chunk_len <= 65535) {
        uint32_t *p32 = static_cast<uint32_t *>(partial);
        for (int j = w; j < BINS; j += W) {
            const uint2 c = get(j);
            p32[((chunk * groups + group) * BINS + j) * 64 + lane] = c.x | (c.y << 16);
        }
    } else {
        uint2 *p64 = static_cast<uint2 *>(partial);
        for (int j = w; j < BINS; j += W) p64[((chunk * groups + group) * BINS + j) * 64 + lane] = get(j);
    }
}

// gfx950 keeps 8 waves per SIMD resident only for kernels of at most 80
// scalar registers (81-96 admit 7, 97-112 six), where the compiler's
// occupancy estimate allows 8 up to 96.  The sweep's software pipeline holds
// two blocks of point data in scalar registers (about 106 in all); capped at
// 80 (the attribute's count leaves out VCC), the values set up before the
// loops go to vector-register lanes instead, none inside the loops, and two
// 16-wave blocks share a CU.
#define SWEEP_SGPR_LIMIT __attribute__((amdgpu_num_sgpr(82)))

template <int D, int PATH, int W>
__global__ __launch_bounds__(W * 64) SWEEP_SGPR_LIMIT void k_sweep(const void *__restrict__ Zv, int64_t N,
                                                  int64_t n_p, int64_t n_q, int64_t chunk_len,
                                                  int64_t groups, int hists,
                                                  void *__restrict__ partial,
                                                  BlockBest *__restrict__ block_best,
                                                  uint32_t *__restrict__ counts)
{
    extern __shared__ uint32_t smem[];
    sweep_block<D, PATH, W>(Zv, N, n_p, n_q, chunk_len, blockIdx.y, gridDim.y, blockIdx.x, groups,
                            hists, partial, block_best, counts, smem);
}

// Many tests of one dimension in one launch: block i sweeps work item
// items[i] = (test, origin group), each test in a single chunk.
template <int D, int PATH, int W>
__global__ __launch_bounds__(W * 64) void k_sweep_packed(const PackedTest *__restrict__ tests,
                                                         const int2 *__restrict__ items,
                                                         BlockBest *__restrict__ block_best)
{
    extern __shared__ uint32_t smem[];
    const int2 it = items[blockIdx.x];
    const PackedTest t = tests[it.x];
    sweep_block<D, PATH, W>(t.Z, t.N, t.n_p, t.n_q, t.N, 0, 1, it.y, t.groups, t.hists, nullptr,
                            block_best + t.bb_offset, nullptr, smem);
}

// packed != 0: the partial counts are uint32 (c_P | c_Q << 16), else uint2.
template <int D, int W>
__global__ __launch_bounds__(W * 64) void k_score(int64_t N, int64_t n_p, int64_t n_q,
                                                  int64_t chunks, int64_t groups, int packed,
                                                  const void *__restrict__ partial,
                                                  BlockBest *__restrict__ block_best,
                                                  uint32_t *__restrict__ counts)
{
    constexpr int BINS = Geo<D>::BINS;
    __shared__ uint32_t scratch[W * 64 * 4];
    const int lane = threadIdx.x & 63;
    const int64_t group = blockIdx.x;
    auto get = [&](int j) {
        uint32_t cp = 0, cq = 0;
        if (packed) {
            const uint32_t *p32 = static_cast<const uint32_t *>(partial);
            for (int64_t s = 0; s < chunks; ++s) {
                const uint32_t c = p32[((s * groups + group) * BINS + j) * 64 + lane];
                cp += c & 0xffffu;
                cq += c >> 16;
            }
        } else {
            const uint2 *p64 = static_cast<const uint2 *>(partial);
            for (int64_t s = 0; s < chunks; ++s) {
                const uint2 c = p64[((s * groups + group) * BINS + j) * 64 + lane];
                cp += c.x;
                cq += c.y;
            }
        }
        return make_uint2(cp, cq);
    };
    finish_block<D, W>(get, group, N, n_p, n_q, block_best, counts, scratch);
}

// done (nullable, coherent host memory): set to 1 once *out is written, so
// that a host waiting on this result alone can poll it.
__global__ __launch_bounds__(1024) void k_reduce(const BlockBest *__restrict__ bb, int64_t n,
                                                 uint32_t *__restrict__ flags,
                                                 ResultDev *__restrict__ out, uint32_t *done)
{
    __shared__ uint64_t sn[16];
    __shared__ uint32_t so[16];
    __shared__ int32_t sc[16];
    uint64_t best = 0;
    uint32_t org = 0xffffffffu;
    int32_t code = 0x7fffffff;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        BlockBest b = bb[i];
        if (better(b.num, b.origin, b.code, best, org, code)) {
            best = b.num;
            org = b.origin;
            code = b.code;
        }
    }
    wave_best(best, org, code);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sn[w] = best;
        so[w] = org;
        sc[w] = code;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < (int)(blockDim.x >> 6); ++v) {
            if (better(sn[v], so[v], sc[v], best, org, code)) {
                best = sn[v];
                org = so[v];
                code = sc[v];
            }
        }
        out->num = best;
        out->origin = (int64_t)org;
        out->code = code;
        out->flags = *flags;
        *flags = 0u;
        if (done) {
            __threadfence_system();  // the result reaches host memory first
            __hip_atomic_store(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// One block per packed test: reduce its block results into out[test].
__global__ __launch_bounds__(256) void k_reduce_packed(const PackedTest *__restrict__ tests,
                                                       const BlockBest *__restrict__ bb,
                                                       ResultDev *__restrict__ out)
{
    __shared__ uint64_t sn[4];
    __shared__ uint32_t so[4];
    __shared__ int32_t sc[4];
    const PackedTest t = tests[blockIdx.x];
    uint64_t best = 0;
    uint32_t org = 0xffffffffu;
    int32_t code = 0x7fffffff;
    for (int64_t i = threadIdx.x; i < t.groups; i += blockDim.x) {
        BlockBest b = bb[t.bb_offset + i];
        if (better(b.num, b.origin, b.code, best, org, code)) {
            best = b.num;
            org = b.origin;
            code = b.code;
        }
    }
    wave_best(best, org, code);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sn[w] = best;
        so[w] = org;
        sc[w] = code;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 4; ++v)
            if (better(sn[v], so[v], sc[v], best, org, code)) {
                best = sn[v];
                org = so[v];
                code = sc[v];
            }
        ResultDev r;
        r.num = best;
        r.origin = (int64_t)org;
        r.code = code;
        r.flags = 0;
        r.ge = 0;
        out[blockIdx.x] = r;
    }
}

__global__ void k_ingest_f32(const float *P, int64_t np_elems, const float *Q, int64_t total,
                             float *Z, uint32_t *flags)
{
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        float v = i < np_elems ? P[i] : Q[i - np_elems];
        if (!__builtin_isfinite(v)) bad = 1u;
        Z[i] = v + 0.0f;  // maps -0 to +0, leaves every other value (subnormals included) as is
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, 1u);
}

// ---------------------------------------------------------------- host side

int point_words(int path, int d)
{
    if (path == PATH_F32) return d;
    return d <= 2 ? 1 : (d <= 4 ? 2 : 4);
}

size_t hist_lds_bytes(int d, int hists)
{
    // d <= 4: a BINS x BINS pair table and BINS single-point bins per histogram
    const size_t bins = (size_t)1 << d;
    const size_t slots = d <= 4 ? bins * bins + bins : bins;
    return (size_t)hists * slots * 64 * 4;
}

size_t sweep_lds_bytes(const SweepPlan &p)
{
    size_t hist = hist_lds_bytes(p.d, p.hists);
    size_t fin = (size_t)p.waves * 64 * 16;
    return hist > fin ? hist : fin;
}

int sweep_hists(int d, int waves, int64_t chunk_len, int64_t n_p, int64_t n_q)
{
    // A wave sweeps at most ceil(m / waves) points of a sample with m points
    // in the chunk, and at most ceil(waves / h) waves share each of h
    // histograms (wave w adds into histogram w mod h).
    const int64_t mp = chunk_len < n_p ? chunk_len : n_p;
    const int64_t mq = chunk_len < n_q ? chunk_len : n_q;
    const int64_t perp = (mp + waves - 1) / waves, perq = (mq + waves - 1) / waves;
    for (int h = 1; h <= waves; h *= 2) {
        const int64_t share = (waves + h - 1) / h;
        if (share * perp <= 65535 && share * perq <= 65535)
            return hist_lds_bytes(d, h) <= (size_t)MAX_LDS_BYTES ? h : 0;
    }
    return 0;
}

int max_waves_for_d(int /*d*/) { return 16; }

hipError_t launch_ingest_f32(const float *P, int64_t n_p, const float *Q, int64_t n_q, int d,
                             float *Z, uint32_t *flags, hipStream_t s)
{
    int64_t total = (n_p + n_q) * d;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_ingest_f32, dim3((unsigned)blocks), dim3(256), 0, s, P, n_p * d, Q,
                       total, Z, flags);
    return hipGetLastError();
}

// Lets a kernel instance use more than the default 64 KB of dynamic LDS (once
// per instance, whichever thread launches it first; if the runtime refuses,
// the launch reports the real error).
static void allow_big_lds(const void *kernel, std::once_flag &once)
{
    std::call_once(once, [kernel] {
        if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, MAX_LDS_BYTES) !=
            hipSuccess)
            (void)hipGetLastError();
    });
}

template <int D, int PATH, int W>
static hipError_t launch_sweep_t(const SweepPlan &p, const void *Z, int64_t N, int64_t n_p,
                                 int64_t n_q, void *partial, BlockBest *bb, uint32_t *counts,
                                 hipStream_t s)
{
    size_t lds = sweep_lds_bytes(p);
    static std::once_flag attr_set;
    if (lds > 64 * 1024) allow_big_lds((const void *)k_sweep<D, PATH, W>, attr_set);
    dim3 grid((unsigned)p.groups, (unsigned)p.chunks);
    hipLaunchKernelGGL((k_sweep<D, PATH, W>), grid, dim3(W * 64), lds, s, Z, N, n_p, n_q,
                       p.chunk_len, p.groups, p.hists, partial, bb, counts);
    return hipGetLastError();
}

template <int D, int PATH>
static hipError_t launch_sweep_w(const SweepPlan &p, const void *Z, int64_t N, int64_t n_p,
                                 int64_t n_q, void *partial, BlockBest *bb, uint32_t *counts,
                                 hipStream_t s)
{
    switch (p.waves) {
    case 1: return launch_sweep_t<D, PATH, 1>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 2: return launch_sweep_t<D, PATH, 2>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 4: return launch_sweep_t<D, PATH, 4>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 8: return launch_sweep_t<D, PATH, 8>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 12: return launch_sweep_t<D, PATH, 12>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 16: return launch_sweep_t<D, PATH, 16>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    default: return hipErrorInvalidValue;
    }
}

template <int PATH>
static hipError_t launch_sweep_p(const SweepPlan &p, const void *Z, int64_t N, int64_t n_p,
                                 int64_t n_q, void *partial, BlockBest *bb, uint32_t *counts,
                                 hipStream_t s)
{
    switch (p.d) {
    case 1: return launch_sweep_w<1, PATH>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 2: return launch_sweep_w<2, PATH>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 3: return launch_sweep_w<3, PATH>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 4: return launch_sweep_w<4, PATH>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 5: return launch_sweep_w<5, PATH>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 6: return launch_sweep_w<6, PATH>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 7: return launch_sweep_w<7, PATH>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    case 8: return launch_sweep_w<8, PATH>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(const SweepPlan &p, const void *Z, int64_t N, int64_t n_p, int64_t n_q,
                        void *partial, BlockBest *bb, uint32_t *counts, hipStream_t s)
{
    if (p.groups < 1 || p.chunks < 1 || p.chunk_len < 1 || p.groups * 64 < N ||
        p.chunks * p.chunk_len < N || p.groups > 0x7fffffff || p.chunks > 65535)
        return hipErrorInvalidValue;
    // the 16-bit counters must not overflow and the histograms must fit in LDS
    const int hmin = sweep_hists(p.d, p.waves, p.chunk_len, n_p, n_q);
    if (hmin == 0 || p.hists < hmin || p.hists > p.waves || (p.hists & (p.hists - 1)) ||
        sweep_lds_bytes(p) > (size_t)MAX_LDS_BYTES)
        return hipErrorInvalidValue;
    if (p.path == PATH_F32) return launch_sweep_p<PATH_F32>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    if (p.path == PATH_R16) return launch_sweep_p<PATH_R16>(p, Z, N, n_p, n_q, partial, bb, counts, s);
    return hipErrorInvalidValue;
}

template <int D, int PATH, int W>
static hipError_t launch_packed_t(const PackedTest *tests, const int2 *items, int64_t nitems,
                                  int max_hists, BlockBest *bb, hipStream_t s)
{
    SweepPlan p;
    p.d = D;
    p.waves = W;
    p.hists = max_hists;
    const size_t lds = sweep_lds_bytes(p);
    if (lds > (size_t)MAX_LDS_BYTES) return hipErrorInvalidValue;
    static std::once_flag attr_set;
    if (lds > 64 * 1024) allow_big_lds((const void *)k_sweep_packed<D, PATH, W>, attr_set);
    hipLaunchKernelGGL((k_sweep_packed<D, PATH, W>), dim3((unsigned)nitems), dim3(W * 64), lds, s,
                       tests, items, bb);
    return hipGetLastError();
}

template <int D, int PATH>
static hipError_t launch_packed_w(int waves, const PackedTest *tests, const int2 *items, int64_t nitems,
                                  int max_hists, BlockBest *bb, hipStream_t s)
{
    switch (waves) {
    case 4: return launch_packed_t<D, PATH, 4>(tests, items, nitems, max_hists, bb, s);
    case 8: return launch_packed_t<D, PATH, 8>(tests, items, nitems, max_hists, bb, s);
    case 16: return launch_packed_t<D, PATH, 16>(tests, items, nitems, max_hists, bb, s);
    default: return hipErrorInvalidValue;
    }
}

bool packed_waves_ok(int waves) { return waves == 4 || waves == 8 || waves == 16; }

hipError_t launch_sweep_packed(int path, int d, int waves, const PackedTest *tests, const int2 *items,
                               int64_t nitems, int max_hists, BlockBest *bb, hipStream_t s)
{
    if (nitems < 1 || nitems > 0x7fffffff || !packed_waves_ok(waves)) return hipErrorInvalidValue;
    if (max_hists < 1 || max_hists > waves || (max_hists & (max_hists - 1)))
        return hipErrorInvalidValue;
#define DDKS_PACKED_CASE(DD)                                                                          \
    case DD:                                                                                          \
        return path == PATH_F32                                                                       \
                   ? launch_packed_w<DD, PATH_F32>(waves, tests, items, nitems, max_hists, bb, s)     \
                   : launch_packed_w<DD, PATH_R16>(waves, tests, items, nitems, max_hists, bb, s);
    if (path != PATH_F32 && path != PATH_R16) return hipErrorInvalidValue;
    switch (d) {
        DDKS_PACKED_CASE(1)
        DDKS_PACKED_CASE(2)
        DDKS_PACKED_CASE(3)
        DDKS_PACKED_CASE(4)
        DDKS_PACKED_CASE(5)
        DDKS_PACKED_CASE(6)
        DDKS_PACKED_CASE(7)
        DDKS_PACKED_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef DDKS_PACKED_CASE
}

hipError_t launch_reduce_packed(const PackedTest *tests, int64_t ntests, const BlockBest *bb,
                                ResultDev *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_packed, dim3((unsigned)ntests), dim3(256), 0, s, tests, bb, out);
    return hipGetLastError();
}

template <int D>
static hipError_t launch_score_d(const SweepPlan &p, int64_t N, int64_t n_p, int64_t n_q,
                                 const void *partial, BlockBest *bb, uint32_t *counts,
                                 hipStream_t s)
{
    hipLaunchKernelGGL((k_score<D, 4>), dim3((unsigned)p.groups), dim3(256), 0, s, N, n_p, n_q,
                       p.chunks, p.groups, partial_packed(p) ? 1 : 0, partial, bb, counts);
    return hipGetLastError();
}

hipError_t launch_score(const SweepPlan &p, int64_t N, int64_t n_p, int64_t n_q,
                        const void *partial, BlockBest *bb, uint32_t *counts, hipStream_t s)
{
    switch (p.d) {
    case 1: return launch_score_d<1>(p, N, n_p, n_q, partial, bb, counts, s);
    case 2: return launch_score_d<2>(p, N, n_p, n_q, partial, bb, counts, s);
    case 3: return launch_score_d<3>(p, N, n_p, n_q, partial, bb, counts, s);
    case 4: return launch_score_d<4>(p, N, n_p, n_q, partial, bb, counts, s);
    case 5: return launch_score_d<5>(p, N, n_p, n_q, partial, bb, counts, s);
    case 6: return launch_score_d<6>(p, N, n_p, n_q, partial, bb, counts, s);
    case 7: return launch_score_d<7>(p, N, n_p, n_q, partial, bb, counts, s);
    case 8: return launch_score_d<8>(p, N, n_p, n_q, partial, bb, counts, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce(const BlockBest *bb, int64_t nblocks, uint32_t *flags, ResultDev *out,
                         hipStream_t s, uint32_t *done)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, bb, nblocks, flags, out, done);
    return hipGetLastError();
}

}  // namespace ddks
