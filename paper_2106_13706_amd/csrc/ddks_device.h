// Device building blocks of the orthant-counting sweep shared by the
// single-test, permutation and serving kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ddks_internal.h"

namespace ddks {

typedef short short2_t __attribute__((ext_vector_type(2)));

template <int D>
struct Geo {
    static constexpr int BINS = 1 << D;
    static constexpr int NREG = (D + 1) / 2;   // sign registers, two dimensions each
    static constexpr int NPERM = (D + 3) / 4;  // v_perm/v_dot4 groups, four dimensions each
    // Dimension 7's weight does not fit a signed byte; it is given weight -128,
    // which flips that bit of the bin index relative to the orthant code.
    static constexpr int FLIP = (D == 8) ? 0x80 : 0;
    static constexpr int KOFF = (D == 8) ? 127 : (BINS - 1);  // bin = dot-sum + KOFF
};

// v_perm_b32 selector for group q: byte i takes the sign of dimension 4q+i
// (8/9: bit 15/31 of src1 = register 2q; 10/11: bit 15/31 of src0 = register
// 2q+1) and 0x00 (selector 12) for dimensions beyond D.
__host__ __device__ constexpr uint32_t perm_sel(int D, int q)
{
    uint32_t sel = 0;
    for (int i = 0; i < 4; ++i) {
        int m = 4 * q + i;
        uint32_t b = (m < D) ? (uint32_t)(8 + i) : 12u;
        sel |= b << (8 * i);
    }
    return sel;
}

// Signed-byte weights for group q: 2^m, and -128 for m = 7.
__host__ __device__ constexpr uint32_t dot_wts(int D, int q)
{
    uint32_t w = 0;
    for (int i = 0; i < 4; ++i) {
        int m = 4 * q + i;
        uint32_t b = 0;
        if (m < D) b = (m == 7) ? 0x80u : (uint32_t)(1u << m);
        w |= (b & 0xffu) << (8 * i);
    }
    return w;
}

// Pair histograms (d <= 4).  Consecutive points p, p' of a wave's range are
// counted together in one bin of a BINS x BINS table, bin (code(p) * BINS +
// code(p')), so one LDS atomic serves two points; a per-orthant count is then
// its row sum plus its column sum (plus the single-point bins of a range's
// leftover points).  The pair index comes from the same v_dot4 chain as a
// point of 2d dimensions: the first point's dimensions weighted 2^m * BINS,
// the second's 2^m.  At d = 4 the first point's weight 128 does not fit a
// signed byte and is given -128, which flips bit 7 of the table index (as
// dimension 7 does at d = 8).
template <int D>
struct PairGeo {
    static constexpr bool ON = D <= 4;
    static constexpr int BINS = 1 << D;
    static constexpr int PBINS = BINS * BINS;
    static constexpr int PFLIP = (D == 4) ? 0x80 : 0;
    static constexpr int PKOFF = (D == 4) ? 127 : (PBINS - 1);  // table index = dot-sum + PKOFF
    static constexpr int SLOTS = PBINS + BINS;                 // table, then single-point bins
};

// Signed-byte weights of a pair's first point: 2^m * BINS, -128 for 128.
__host__ __device__ constexpr uint32_t pair_wts_hi(int D)
{
    uint32_t w = 0;
    for (int m = 0; m < D && m < 4; ++m) {
        uint32_t b = (uint32_t)(1u << m) << D;
        w |= (b & 0xffu) << (8 * m);
    }
    return w;
}

typedef __attribute__((address_space(3))) uint32_t lds_u32;

// ---------------------------------------------------------------------------
// Inline-asm building blocks.  A gfx950 pipeline hazard is invisible to the
// compiler inside asm, so each asm block carries a whole dependent chain with
// the spacing built in: a v_dot4 result needs three intervening instructions
// before a VALU reads it; the dots of four points are issued back to back,
// then their address computations, so every read is at least three
// instructions later.
// ---------------------------------------------------------------------------

// sign(x - o) of two rank-encoded dimensions (int16, saturating) into bits 15 and 31.
__device__ __forceinline__ uint32_t sgn2_r16(uint32_t x, uint32_t o)
{
    short2_t t = __builtin_elementwise_sub_sat(__builtin_bit_cast(short2_t, x),
                                               __builtin_bit_cast(short2_t, o));
    return __builtin_bit_cast(uint32_t, t);
}

// Sign-filled bytes of perm group q (v_perm_b32 sign selectors).
template <int D>
__device__ __forceinline__ uint32_t group_bytes(const uint32_t (&r)[Geo<D>::NREG], int q)
{
    constexpr int NR = Geo<D>::NREG;
    if (q == 0) return __builtin_amdgcn_perm(NR > 1 ? r[NR > 1 ? 1 : 0] : 0u, r[0], perm_sel(D, 0));
    return __builtin_amdgcn_perm(NR > 3 ? r[NR > 3 ? 3 : 2] : 0u, r[NR > 2 ? 2 : 0], perm_sel(D, 1));
}

#define DOT0(d, r, w) "v_dot4_i32_i8 " d ", " r ", " w ", 0\n\t"
#define DOTC(d, r, w) "v_dot4_i32_i8 " d ", " r ", " w ", " d "\n\t"
#define ADDR(d, b) "v_lshl_add_u32 " d ", " d ", %[sh], " b "\n\t"

// LDS byte addresses of the bins of four points: base + (dot-sum << SH)
// (SH = 8 for 4-byte bins of 64 lanes, 9 for 8-byte bins).
template <int NPERM, int SH = 8>
__device__ __forceinline__ void addr4(const uint32_t (&R)[2][4], uint32_t base, uint32_t (&a)[4],
                                      uint32_t w0, uint32_t w1)
{
    if constexpr (NPERM == 1) {
        asm(DOT0("%0", "%4", "%8") DOT0("%1", "%5", "%8") DOT0("%2", "%6", "%8")
                DOT0("%3", "%7", "%8") ADDR("%0", "%9") ADDR("%1", "%9") ADDR("%2", "%9")
                    ADDR("%3", "%9")
            : "=&v"(a[0]), "=&v"(a[1]), "=&v"(a[2]), "=&v"(a[3])
            : "v"(R[0][0]), "v"(R[0][1]), "v"(R[0][2]), "v"(R[0][3]), "s"(w0), "v"(base),
              [sh] "i"(SH));
    } else {
        asm(DOT0("%0", "%4", "%12") DOT0("%1", "%5", "%12") DOT0("%2", "%6", "%12")
                DOT0("%3", "%7", "%12") DOTC("%0", "%8", "%13") DOTC("%1", "%9", "%13")
                    DOTC("%2", "%10", "%13") DOTC("%3", "%11", "%13") ADDR("%0", "%14")
                        ADDR("%1", "%14") ADDR("%2", "%14") ADDR("%3", "%14")
            : "=&v"(a[0]), "=&v"(a[1]), "=&v"(a[2]), "=&v"(a[3])
            : "v"(R[0][0]), "v"(R[0][1]), "v"(R[0][2]), "v"(R[0][3]), "v"(R[1][0]),
              "v"(R[1][1]), "v"(R[1][2]), "v"(R[1][3]), "s"(w0), "s"(w1), "v"(base),
              [sh] "i"(SH));
    }
}

// addr4<2> with the second group's weight alternating between points: points
// 0, 2 take w1e and points 1, 3 take w1o (two points whose second groups share
// one register).
template <int SH = 8>
__device__ __forceinline__ void addr4_w2(const uint32_t (&R)[2][4], uint32_t base, uint32_t (&a)[4],
                                         uint32_t w0, uint32_t w1e, uint32_t w1o)
{
    asm(DOT0("%0", "%4", "%12") DOT0("%1", "%5", "%12") DOT0("%2", "%6", "%12")
            DOT0("%3", "%7", "%12") DOTC("%0", "%8", "%13") DOTC("%1", "%9", "%14")
                DOTC("%2", "%10", "%13") DOTC("%3", "%11", "%14") ADDR("%0", "%15")
                    ADDR("%1", "%15") ADDR("%2", "%15") ADDR("%3", "%15")
        : "=&v"(a[0]), "=&v"(a[1]), "=&v"(a[2]), "=&v"(a[3])
        : "v"(R[0][0]), "v"(R[0][1]), "v"(R[0][2]), "v"(R[0][3]), "v"(R[1][0]), "v"(R[1][1]),
          "v"(R[1][2]), "v"(R[1][3]), "s"(w0), "s"(w1e), "s"(w1o), "v"(base), [sh] "i"(SH));
}

// The same for a single point, with the wait states written out.
template <int NPERM, int SH = 8>
__device__ __forceinline__ uint32_t addr1(uint32_t R0, uint32_t R1, uint32_t base, uint32_t w0,
                                          uint32_t w1)
{
    uint32_t a;
    if constexpr (NPERM == 1) {
        asm(DOT0("%0", "%1", "%2") "s_nop 2\n\t" ADDR("%0", "%3")
            : "=&v"(a) : "v"(R0), "s"(w0), "v"(base), [sh] "i"(SH));
    } else {
        asm(DOT0("%0", "%1", "%3") "s_nop 2\n\t" DOTC("%0", "%2", "%4") "s_nop 2\n\t" ADDR("%0", "%5")
            : "=&v"(a) : "v"(R0), "v"(R1), "s"(w0), "s"(w1), "v"(base), [sh] "i"(SH));
    }
    return a;
}

__device__ __forceinline__ void lds_add(uint32_t byte_addr, uint32_t v)
{
    __hip_atomic_fetch_add((lds_u32 *)(uintptr_t)byte_addr, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Point element type and words per point for each path.
template <int PATH, int D>
struct Layout;
template <int D>
struct Layout<PATH_F32, D> {
    typedef float T;
    static constexpr int PW = D;  // floats per point
};
template <int D>
struct Layout<PATH_R16, D> {
    typedef uint32_t T;
    static constexpr int PW = (D <= 2) ? 1 : (D <= 4 ? 2 : 4);  // padded to a power of two
};

// Points per unrolled block: a multiple of four, about 32 scalar registers of point data.
template <int PATH, int D>
struct Unroll {
    static constexpr int PW = Layout<PATH, D>::PW;
    static constexpr int U0 = ((32 / PW) / 4) * 4;
    static constexpr int U = U0 < 4 ? 4 : U0;
};

// The origin held by a lane.
template <int PATH, int D>
struct Origin;
template <int D>
struct Origin<PATH_F32, D> {
    float o[D];
    __device__ void load(const float *Z, int64_t k)
    {
#pragma unroll
        for (int m = 0; m < D; ++m) o[m] = Z[k * D + m];
    }
};
template <int D>
struct Origin<PATH_R16, D> {
    static constexpr int PW = Layout<PATH_R16, D>::PW;
    uint32_t o[PW];
    __device__ void load(const uint32_t *Z, int64_t k)
    {
#pragma unroll
        for (int m = 0; m < PW; ++m) o[m] = Z[k * PW + m];
    }
};

// fp32 signs by subtraction: with gradual underflow x - o is zero only when
// x == o (and then +0), so its sign bit is [x < o]; v_cvt_pkrtz_f16_f32 keeps
// the signs of two differences (rounding toward zero never flips a sign) in
// bits 15 and 31.
template <int D>
__device__ __forceinline__ void signs_sub(const float *x, const float *o, uint32_t (&r)[Geo<D>::NREG])
{
#pragma unroll
    for (int p = 0; p < Geo<D>::NREG; ++p) {
        const float a = x[2 * p] - o[2 * p];
        const float b = (2 * p + 1 < D) ? x[2 * p + 1] - o[2 * p + 1] : 0.0f;
        r[p] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a, b));
    }
}

// Sign registers of point x (PW words at xs) against the lane's origin.
template <int PATH, int D>
__device__ __forceinline__ void signs(const typename Layout<PATH, D>::T *xs,
                                      const Origin<PATH, D> &org, uint32_t (&r)[Geo<D>::NREG])
{
    if constexpr (PATH == PATH_F32) {
        signs_sub<D>(xs, org.o, r);
    } else {
#pragma unroll
        for (int p = 0; p < Geo<D>::NREG; ++p) r[p] = sgn2_r16(xs[p], org.o[p]);
    }
}

// LDS bin addresses of U consecutive points held in buf (U a multiple of 4).
template <int PATH, int D, int U>
__device__ __forceinline__ void block_addrs(const typename Layout<PATH, D>::T *buf,
                                            const Origin<PATH, D> &org, uint32_t base,
                                            uint32_t (&a)[U])
{
    constexpr int PW = Layout<PATH, D>::PW;
    constexpr int NP = Geo<D>::NPERM;
    const uint32_t w0 = dot_wts(D, 0), w1 = dot_wts(D, 1);
#pragma unroll
    for (int g = 0; g < U; g += 4) {
        uint32_t R[2][4];
        uint32_t q[4];
        if constexpr (D == 5 || D == 6) {
            // The second group holds dimensions 4 (and 5) only: one v_perm
            // serves two points, bytes 0-1 the first's, bytes 2-3 the second's.
            constexpr uint32_t SEL = D == 6 ? 0x0b0a0908u : 0x0c0a0c08u;
#pragma unroll
            for (int u = 0; u < 4; u += 2) {
                uint32_t r0[Geo<D>::NREG], r1[Geo<D>::NREG];
                signs<PATH, D>(buf + (g + u) * PW, org, r0);
                signs<PATH, D>(buf + (g + u + 1) * PW, org, r1);
                R[0][u] = group_bytes<D>(r0, 0);
                R[0][u + 1] = group_bytes<D>(r1, 0);
                R[1][u] = R[1][u + 1] = __builtin_amdgcn_perm(r1[2], r0[2], SEL);
            }
            addr4_w2(R, base, q, w0, w1, w1 << 16);
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                uint32_t r[Geo<D>::NREG];
                signs<PATH, D>(buf + (g + u) * PW, org, r);
                R[0][u] = group_bytes<D>(r, 0);
                R[1][u] = NP > 1 ? group_bytes<D>(r, 1) : 0u;
            }
            addr4<NP>(R, base, q, w0, w1);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) a[g + u] = q[u];
    }
}

// Pair-table addresses of U/2 pairs of consecutive points held in buf (U a
// multiple of 8): the dot chain of two 4-dimension groups, first point's
// bytes against pair_wts_hi, second point's against dot_wts.
template <int PATH, int D, int U>
__device__ __forceinline__ void block_pair_addrs(const typename Layout<PATH, D>::T *buf,
                                                 const Origin<PATH, D> &org, uint32_t pbase,
                                                 uint32_t (&a)[U / 2])
{
    static_assert(PairGeo<D>::ON && U % 8 == 0, "pairs of four per chain");
    constexpr int PW = Layout<PATH, D>::PW;
    const uint32_t wh = pair_wts_hi(D), wl = dot_wts(D, 0);
#pragma unroll
    for (int g = 0; g < U / 2; g += 4) {
        uint32_t R[2][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uint32_t r0[Geo<D>::NREG], r1[Geo<D>::NREG];
            signs<PATH, D>(buf + (2 * (g + u)) * PW, org, r0);
            signs<PATH, D>(buf + (2 * (g + u) + 1) * PW, org, r1);
            R[0][u] = group_bytes<D>(r0, 0);
            R[1][u] = group_bytes<D>(r1, 0);
        }
        uint32_t q[4];
        addr4<2>(R, pbase, q, wh, wl);
#pragma unroll
        for (int u = 0; u < 4; ++u) a[g + u] = q[u];
    }
}

// d <= 2: a point has at most two sign bits (bits 15 and 31 of its one sign
// register), so one v_perm_b32 gathers both points of a pair: bytes 0, 1 the
// first point's dimensions, bytes 2, 3 the second's, and one v_dot4 against
// the weights (2^m * BINS for the first point, 2^m for the second) gives the
// table index.
__host__ __device__ constexpr uint32_t pair_wts_merged(int D)
{
    uint32_t w = 0;
    for (int m = 0; m < D && m < 2; ++m) {
        w |= ((uint32_t)(1u << m) << D) << (8 * m);  // first point
        w |= (uint32_t)(1u << m) << (8 * (m + 2));     // second point
    }
    return w;
}

template <int PATH, int D, int U>
__device__ __forceinline__ void block_pair_addrs_merged(const typename Layout<PATH, D>::T *buf,
                                                        const Origin<PATH, D> &org, uint32_t pbase,
                                                        uint32_t (&a)[U / 2])
{
    static_assert(D <= 2 && U % 8 == 0, "pairs of four per chain");
    constexpr int PW = Layout<PATH, D>::PW;
    // selector 8/9: bit 15/31 of src1 (first point), 10/11: of src0 (second)
    constexpr uint32_t SEL = 0x0b0a0908u;
    const uint32_t w = pair_wts_merged(D);
#pragma unroll
    for (int g = 0; g < U / 2; g += 4) {
        uint32_t R[2][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            uint32_t r0[Geo<D>::NREG], r1[Geo<D>::NREG];
            signs<PATH, D>(buf + (2 * (g + u)) * PW, org, r0);
            signs<PATH, D>(buf + (2 * (g + u) + 1) * PW, org, r1);
            R[0][u] = __builtin_amdgcn_perm(r1[0], r0[0], SEL);
            R[1][u] = 0u;
        }
        uint32_t q[4];
        addr4<1>(R, pbase, q, w, 0u);
#pragma unroll
        for (int u = 0; u < 4; ++u) a[g + u] = q[u];
    }
}

// Waits for every outstanding LDS and scalar-memory operation of the wave
// (lgkmcnt = 0; vector-memory and export counters left alone).
__device__ __forceinline__ void wait_lgkm() { __builtin_amdgcn_s_waitcnt(0xc07f); }

// Sweeps points [lo, hi) of Z against the lane's origin, adding inc to the
// lane's bin of each point.  base: LDS byte address of bin KOFF of this lane.
//
// Software-pipelined: the scalar loads of block i+1 are issued before block
// i's addresses are computed, and the wait before block i's LDS atomics then
// covers only loads and atomics issued a whole block earlier.  (Scalar loads
// and LDS operations share one wait counter, so waiting for a block's points
// right after loading them would also wait for the atomics just issued.)
template <int PATH, int D>
__device__ __forceinline__ void sweep_range(const typename Layout<PATH, D>::T *__restrict__ Z,
                                            int64_t lo, int64_t hi, const Origin<PATH, D> &org,
                                            uint32_t base, uint32_t inc)
{
    typedef typename Layout<PATH, D>::T T;
    constexpr int PW = Layout<PATH, D>::PW;
    constexpr int U = Unroll<PATH, D>::U;
    constexpr int NP = Geo<D>::NPERM;
    int64_t i = lo;
    int64_t nblk = hi > lo ? (hi - lo) / U : 0;
    if (nblk & 1) {  // an odd block first, so the pipelined loop runs in pairs
        T buf[U * PW];
#pragma unroll
        for (int e = 0; e < U * PW; ++e) buf[e] = Z[i * PW + e];
        uint32_t a[U];
        block_addrs<PATH, D, U>(buf, org, base, a);
#pragma unroll
        for (int u = 0; u < U; ++u) lds_add(a[u], inc);
        i += U;
        --nblk;
    }
    if (nblk > 0) {
        // Two blocks per trip and no exit in between, so no load can be moved
        // past the block that consumes it.  The last trip's prefetch is clamped
        // to the last full block (a redundant, in-bounds load).
        const int64_t last = hi - U;
        T bufA[U * PW], bufB[U * PW];
#pragma unroll
        for (int e = 0; e < U * PW; ++e) bufA[e] = Z[i * PW + e];
        // Settle everything issued before the loop here, once: otherwise the
        // counter state merged at the loop head forces a full wait (on this
        // trip's ds_adds as well) at the top of every trip.
        __builtin_amdgcn_s_waitcnt(0);
        for (int64_t t = 0; t < nblk; t += 2) {
#pragma unroll
            for (int e = 0; e < U * PW; ++e) bufB[e] = Z[(i + U) * PW + e];
            uint32_t a[U];
            block_addrs<PATH, D, U>(bufA, org, base, a);
            wait_lgkm();
#pragma unroll
            for (int u = 0; u < U; ++u) lds_add(a[u], inc);
            const int64_t na = (i + 2 * U < last) ? i + 2 * U : last;
#pragma unroll
            for (int e = 0; e < U * PW; ++e) bufA[e] = Z[na * PW + e];
            block_addrs<PATH, D, U>(bufB, org, base, a);
            wait_lgkm();
#pragma unroll
            for (int u = 0; u < U; ++u) lds_add(a[u], inc);
            i += 2 * U;
        }
    }
    const uint32_t w0 = dot_wts(D, 0), w1 = dot_wts(D, 1);
    for (; i < hi; ++i) {
        const T *xs = Z + i * PW;
        T buf[PW];
#pragma unroll
        for (int e = 0; e < PW; ++e) buf[e] = xs[e];
        uint32_t r[Geo<D>::NREG];
        signs<PATH, D>(buf, org, r);
        uint32_t R0 = group_bytes<D>(r, 0);
        uint32_t R1 = NP > 1 ? group_bytes<D>(r, 1) : 0u;
        lds_add(addr1<NP>(R0, R1, base, w0, w1), inc);
    }
}

template <int PATH, int D, int U>
__device__ __forceinline__ void pair_addrs(const typename Layout<PATH, D>::T *buf, const Origin<PATH, D> &org,
                                           uint32_t pbase, uint32_t (&a)[U / 2])
{
    if constexpr (D <= 2)
        block_pair_addrs_merged<PATH, D, U>(buf, org, pbase, a);
    else
        block_pair_addrs<PATH, D, U>(buf, org, pbase, a);
}

// sweep_range with pair histograms (d <= 4): the same software pipeline over
// blocks of U points, each block adding U/2 pairs into the table at pbase (the
// LDS byte address of table index PKOFF of this lane); leftover points of the
// range go one by one to the single-point bins at sbase (bin KOFF).
template <int PATH, int D>
__device__ __forceinline__ void sweep_range_pairs(const typename Layout<PATH, D>::T *__restrict__ Z,
                                                  int64_t lo, int64_t hi, const Origin<PATH, D> &org,
                                                  uint32_t pbase, uint32_t sbase, uint32_t inc)
{
    typedef typename Layout<PATH, D>::T T;
    constexpr int PW = Layout<PATH, D>::PW;
    constexpr int U0 = Unroll<PATH, D>::U;
    constexpr int U = U0 < 8 ? 8 : U0 / 8 * 8;
    int64_t i = lo;
    int64_t nblk = hi > lo ? (hi - lo) / U : 0;
    if (nblk & 1) {
        T buf[U * PW];
#pragma unroll
        for (int e = 0; e < U * PW; ++e) buf[e] = Z[i * PW + e];
        uint32_t a[U / 2];
        pair_addrs<PATH, D, U>(buf, org, pbase, a);
#pragma unroll
        for (int u = 0; u < U / 2; ++u) lds_add(a[u], inc);
        i += U;
        --nblk;
    }
    if (nblk > 0) {
        const int64_t last = hi - U;
        T bufA[U * PW], bufB[U * PW];
#pragma unroll
        for (int e = 0; e < U * PW; ++e) bufA[e] = Z[i * PW + e];
        __builtin_amdgcn_s_waitcnt(0);
        for (int64_t t = 0; t < nblk; t += 2) {
#pragma unroll
            for (int e = 0; e < U * PW; ++e) bufB[e] = Z[(i + U) * PW + e];
            uint32_t a[U / 2];
            pair_addrs<PATH, D, U>(bufA, org, pbase, a);
            wait_lgkm();
#pragma unroll
            for (int u = 0; u < U / 2; ++u) lds_add(a[u], inc);
            const int64_t na = (i + 2 * U < last) ? i + 2 * U : last;
#pragma unroll
            for (int e = 0; e < U * PW; ++e) bufA[e] = Z[na * PW + e];
            pair_addrs<PATH, D, U>(bufB, org, pbase, a);
            wait_lgkm();
#pragma unroll
            for (int u = 0; u < U / 2; ++u) lds_add(a[u], inc);
            i += 2 * U;
        }
    }
    const uint32_t w0 = dot_wts(D, 0);
    for (; i < hi; ++i) {
        T buf[PW];
#pragma unroll
        for (int e = 0; e < PW; ++e) buf[e] = Z[i * PW + e];
        uint32_t r[Geo<D>::NREG];
        signs<PATH, D>(buf, org, r);
        lds_add(addr1<1>(group_bytes<D>(r, 0), 0u, sbase, w0, 0u), inc);
    }
}

// Key order of the maximum: larger num first, then lower origin, then lower code.
__device__ __forceinline__ bool better(uint64_t an, uint32_t ao, int32_t ac, uint64_t bn,
                                       uint32_t bo, int32_t bc)
{
    if (an != bn) return an > bn;
    if (ao != bo) return ao < bo;
    return ac < bc;
}

__device__ __forceinline__ uint64_t score(uint32_t cp, uint32_t cq, int64_t n_p, int64_t n_q)
{
    int64_t a = (int64_t)cp * n_q - (int64_t)cq * n_p;
    return (uint64_t)(a < 0 ? -a : a);
}

// Wave-wide arg-max of (num, origin, code) with the key order above.
__device__ __forceinline__ void wave_best(uint64_t &n, uint32_t &o, int32_t &c)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        uint64_t n2 = __shfl_xor(n, off, 64);
        uint32_t o2 = __shfl_xor(o, off, 64);
        int32_t c2 = __shfl_xor(c, off, 64);
        if (better(n2, o2, c2, n, o, c)) {
            n = n2;
            o = o2;
            c = c2;
        }
    }
}

}  // namespace ddks
