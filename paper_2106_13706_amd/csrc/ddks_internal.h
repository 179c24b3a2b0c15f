// Internal interface between the host runtime and the gfx950 kernels of libddks.
// Not part of the public ABI (include/ddks.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddks {

// Per-block best (origin group) and the final result, as the device writes them.
struct BlockBest {
    uint64_t num;     // max |c_P*n_Q - c_Q*n_P| within the block
    uint32_t origin;  // lowest maximising origin (P-then-Q index); 0xffffffff if none
    int32_t code;     // lowest maximising orthant code of that origin
};

struct ResultDev {
    uint64_t num;
    int64_t origin;
    int32_t code;
    uint32_t flags;  // bit 0: a non-finite input value was seen; bit 1: malformed label row
    uint64_t ge;     // permutation batch: relabellings with numerator >= num
};

enum Path : int { PATH_F32 = 0, PATH_R16 = 1 };

// One test of a packed (serving) launch.
struct PackedTest {
    const void *Z;      // device points, P then Q, N x d fp32 (-0 already mapped to +0)
    int64_t N, n_p, n_q;
    int64_t groups;     // ceil(N / 64)
    int64_t bb_offset;  // first BlockBest slot of this test
    int32_t hists;      // LDS histograms per block (sweep_hists for the launch's waves, N)
    int32_t path;       // PATH_F32 (Z fp32) or PATH_R16 (Z rank-encoded)
};

// LDS a block may use (gfx950: 160 KB per CU, all of it addressable by one block).
constexpr int MAX_LDS_BYTES = 160 * 1024;
// Waves per block of the packed (many-test) sweep: the default, and the
// largest (which bounds the tests admitted to packed launches).
constexpr int PACKED_WAVES = 8;
constexpr int PACKED_MAX_WAVES = 16;

// Launch shape of one sweep.
struct SweepPlan {
    int path = PATH_F32;
    int d = 1;
    int waves = 4;          // waves per block (1, 2, 4, 8, 16), all on the same 64 origins
    int hists = 1;          // LDS histograms per block (power of two <= waves)
    int64_t groups = 0;     // ceil(N / 64) origin groups
    int64_t chunks = 1;     // point-range chunks (grid.y)
    int64_t chunk_len = 0;  // points per chunk
};

// Partial counts of a multi-chunk plan, one entry per (chunk, group, bin,
// lane): a uint32 with c_P in the low and c_Q in the high half when no chunk
// holds more than 65535 points (each half then fits), else a uint2 (c_P, c_Q).
inline bool partial_packed(const SweepPlan &p) { return p.chunk_len <= 65535; }
inline size_t partial_bytes(const SweepPlan &p)
{
    return (size_t)p.chunks * p.groups * ((size_t)1 << p.d) * 64 * (partial_packed(p) ? 4 : 8);
}

// Words (4-byte) per point in the device point buffer.
int point_words(int path, int d);

// Bytes of dynamic LDS a sweep block of this plan uses.
size_t sweep_lds_bytes(const SweepPlan &p);

// Largest waves-per-block of the sweep kernels.
int max_waves_for_d(int d);

// Bytes of LDS of `hists` histograms of dimension d.
size_t hist_lds_bytes(int d, int hists);

// Smallest number of histograms per block (a power of two <= waves) with
// which no 16-bit per-sample counter can overflow when chunks of chunk_len
// points of a test with n_p + n_q points are swept by `waves` waves; 0 if
// even one histogram per wave is not enough or the histograms do not fit in
// LDS.
int sweep_hists(int d, int waves, int64_t chunk_len, int64_t n_p, int64_t n_q);

// ---------------------------------------------------------------- launches
// All return the HIP error of the launch (hipSuccess on success).

// Copies P then Q into Z (N x d fp32), mapping -0 to +0 and setting bit 0 of
// *flags if any value is not finite.  P/Q may alias Z (in-place).
hipError_t launch_ingest_f32(const float *P, int64_t n_p, const float *Q, int64_t n_q, int d,
                             float *Z, uint32_t *flags, hipStream_t s);

// Words of the device control block of launch_rank16.
constexpr int RANK_CTL_WORDS = 16;

// Encodes Z (N x d fp32, -0 already mapped to +0) as per-dimension ranks
// biased to int16, two dimensions per word, point_words(PATH_R16, d) words per
// point, into R.  scratch: rank16_scratch_bytes(N, d) bytes.  ctl: a device
// block of RANK_CTL_WORDS words.  For N <= 65536 the ranks always fit; for
// larger N, ctl[0] receives the largest per-dimension count of distinct values
// and ctl[1 + m] dimension m's, and the encoding is valid only when all are
// <= 65536 (otherwise see launch_rank16_shift).
hipError_t launch_rank16(const float *Z, int64_t N, int d, uint32_t *R, void *scratch,
                         uint32_t *ctl, hipStream_t s);
// The same encoding for N = n_p + n_q <= 65536 read straight from P then Q
// (device pointers, n x d fp32; -0 taken as +0), so that no ingested copy is
// needed; flags (nullable): bit 0 is set if a value is NaN or infinite.
hipError_t launch_rank16_pq(const float *P, int64_t n_p, const float *Q, int64_t n_q, int d, uint32_t *R,
                            void *scratch, uint32_t *flags, hipStream_t s);
size_t rank16_scratch_bytes(int64_t N, int d);

// N > 65536, after launch_rank16: tables in its scratch.  S: per dimension the
// N (order key << 32 | index) pairs in sorted order; R32: N x d full dense
// ranks; RS: per dimension the first sorted position of each rank (d x
// (N + 1), entry [distinct] = N).
struct RankTables {
    const uint64_t *S = nullptr;
    uint32_t *R32 = nullptr, *RS = nullptr;
};
RankTables rank16_tables(void *scratch, int64_t N, int d);

// For each dimension m with more than 65536 distinct values and N <= 65536 <<
// shift_m (shift_m = 4-bit field m of `shifts`, 0 for the other dimensions):
// replaces the rank in the tables' R32 by F, the first sorted position of the
// point's value, and its 16-bit code in R by F >> shift_m.  Compares on the
// codes are exact up to the points that launch_rank_fixups corrects.
hipError_t launch_rank16_shift(int64_t N, int d, uint32_t *R, void *scratch, uint32_t shifts, hipStream_t s);

// After a sweep of the shifted encoding with plan.chunks >= 2 (before
// launch_score): for every origin o, each point x with o's code and a smaller
// value in some shifted dimension was counted in the orthant of the code
// compares; moves it to its exact orthant in the partial counts of the chunk
// that holds x (at most 2^shift_m - 1 points per origin and dimension).
hipError_t launch_rank_fixups(const SweepPlan &plan, const RankTables &t, int64_t N, int64_t n_p,
                              uint32_t shifts, void *partial, hipStream_t s);

// The O(2^d N^2) sweep.  With plan.chunks == 1 the epilogue scores in place and
// writes block_best[group]; otherwise it writes per-chunk partial counts
// ([chunks][groups][2^d][64] entries, see partial_packed; partial_bytes(plan)
// bytes) for launch_score.
// counts (nullable, device): [N][2^d][2] uint32, written when chunks == 1.
hipError_t launch_sweep(const SweepPlan &plan, const void *Z, int64_t N, int64_t n_p,
                        int64_t n_q, void *partial, BlockBest *block_best, uint32_t *counts,
                        hipStream_t s);

// Sums the partial counts of a multi-chunk sweep, scores, writes block_best
// (and counts if non-null).
hipError_t launch_score(const SweepPlan &plan, int64_t N, int64_t n_p, int64_t n_q,
                        const void *partial, BlockBest *block_best, uint32_t *counts,
                        hipStream_t s);

// Reduces block_best[0..nblocks) with the tie rule (num desc, origin asc,
// code asc) into *out, copies *flags into out->flags and clears *flags.
// done (nullable, coherent pinned host memory): set to 1 after *out.
hipError_t launch_reduce(const BlockBest *block_best, int64_t nblocks, uint32_t *flags,
                         ResultDev *out, hipStream_t s, uint32_t *done = nullptr);

// ---------------------------------------------------------------- packed tests

// One launch over work items (test, origin group) of tests of dimension d on
// one path, each test swept in a single chunk by `waves` waves (4, 8 or 16;
// packed_waves_ok) with test.hists histograms (nonzero sweep_hists(d, waves,
// N, n_p, n_q)); block results go to bb[test.bb_offset + group].  max_hists:
// the largest test.hists of the launch (sizes the LDS).
bool packed_waves_ok(int waves);
hipError_t launch_sweep_packed(int path, int d, int waves, const PackedTest *tests, const int2 *items,
                               int64_t nitems, int max_hists, BlockBest *bb, hipStream_t s);
// out[t] = the test's maximum with the tie rule, for t < ntests.
hipError_t launch_reduce_packed(const PackedTest *tests, int64_t ntests, const BlockBest *bb,
                                ResultDev *out, hipStream_t s);

// ---------------------------------------------------------------- permutation test

// LDS bytes of one permutation-kernel wave (pb relabellings per wave).
size_t perm_lds_bytes(int d, int pb);
// Largest relabellings-per-wave group for dimension d (8 for d <= 6, else 4).
int perm_max_group(int d);

// Checks every label row (bit 1 of *flags when a row is malformed), builds the
// per-point increments inc [ceil(B/pb)][n][pb/4] and clears nums[B].
hipError_t launch_perm_prepare(const uint32_t *labels, int64_t n, int B, int64_t n_p, int pb,
                               uint64_t *inc, uint32_t *flags, unsigned long long *nums,
                               hipStream_t s);

// nums[b] = max over origins and orthants of |c_P*n_Q - c_Q*n_P| for relabelling b
// (atomic max; nums must start at zero).  obs_counts: [N][2^d][2] counts of any
// one split of the same pooled points (only c_P + c_Q is used).  n_p <= 65535.
// pb relabellings per block (inc built for the same pb), `waves` waves per
// block sharing its 64 origins and counters; perm_shape_ok tells which.
constexpr int PERM_DEFAULT_WAVES = 8;
bool perm_shape_ok(int d, int pb, int waves);
hipError_t launch_perm(int path, int d, int pb, int waves, const void *Z, int64_t N, int64_t n_p,
                       const uint64_t *inc, int B, const uint32_t *obs_counts,
                       unsigned long long *nums, hipStream_t s);

// Sorts each column m < C of X (N x C fp32, finite, -0 already +0): the pairs
// (order-preserving key of X[i][m]) << 32 | i ascending in S[m * N + p],
// S = *S_out inside scratch (sort_columns_scratch_bytes(N, C) bytes).
size_t sort_columns_scratch_bytes(int64_t N, int C);
hipError_t launch_sort_columns(const float *X, int64_t N, int C, void *scratch, uint64_t **S_out,
                               hipStream_t s);

// ---------------------------------------------------------------- rdKS

// Scratch bytes of launch_rdks for N points in d dimensions.
size_t rdks_scratch_bytes(int64_t N, int d);

// rdKS of Z (N x d, first n_p rows the first sample, -0 already +0): per
// corner numerators in corner_num[d + 1], and *out = (the largest, the lowest
// maximising corner, code 0, *flags), *flags cleared.
hipError_t launch_rdks(const float *Z, int64_t N, int64_t n_p, int d, void *scratch,
                       unsigned long long *corner_num, uint32_t *flags, ResultDev *out, hipStream_t s);

// ---------------------------------------------------------------- vdKS

// Slots of the voxel hash table for N points (a power of two >= 2 N).
size_t vdks_table_slots(int64_t N);
// Bytes of the per-block results of the voxel sweep over M filled voxels.
size_t vdks_best_bytes(int64_t M);

// Per-dimension extent of Z (N x d, -0 already mapped to +0), each point's
// voxel key sum_m v_m V^m merged into the table (slots entries: keys, then 2
// counts each), and the filled voxels compacted into keys[] and inc[]
// (c_P | c_Q << 32), their number in *counter.  mm: 2 d words of scratch;
// part: VOX_EXTENT_ROWS x 2 d words of scratch (per-block extents).
constexpr int VOX_EXTENT_ROWS = 256;
hipError_t launch_vox_front(const float *Z, int64_t N, int64_t n_p, int d, int V, uint32_t *mm,
                            uint32_t *part, uint64_t *tab_key, uint32_t *tab_cnt, int64_t slots, uint32_t *counter,
                            uint64_t *keys, uint64_t *inc, hipStream_t s);

// Launch shape of the weighted sweep: waves per block (4, 8 or 16; they
// share the block's origins), origin groups of 64 per block (1 or 2), and
// point chunks (1..VSWEEP_MAX_CHUNKS; with more than one the chunks' counts go
// through partial sums).
constexpr int VSWEEP_MAX_CHUNKS = 16;
struct VSweepPlan {
    int waves = 8;
    int chunks = 1;
    int per_block = 1;  // origin groups per block (1 or 2): each voxel load serves all of them
};
VSweepPlan vsweep_default_plan(int64_t M);
bool vsweep_plan_ok(const VSweepPlan &p, int64_t M, int d);
// Whether the weighted sweep codes the voxel coordinates one byte each (at
// most 128 voxels per dimension, d <= 7) rather than as int16.
bool vsweep_uses_bytes(int d, int V);
// Words per filled voxel of the weighted sweep's encoding.
int vox_words(int d);

// The weighted sweep over the M filled voxels (RV: M x vox_words(d) words of
// scratch for the encoding, fit: VSWEEP_MAX_CHUNKS words of scratch, bb:
// vdks_best_bytes(M), partial: vsweep_partial_bytes(M, d, plan) of scratch,
// null when that is 0); *out = (num, lowest maximising voxel key, its lowest
// code, *flags), *flags cleared.
size_t vsweep_partial_bytes(int64_t M, int d, const VSweepPlan &plan);
hipError_t launch_vsweep(const uint64_t *keys, const uint64_t *inc, int64_t M, int d, int V, int64_t n_p,
                         int64_t n_q, const VSweepPlan &plan, uint32_t *RV, uint32_t *fit, void *bb, void *partial,
                         uint32_t *flags, ResultDev *out, hipStream_t s);

// ---------------------------------------------------------------- significance

// Rate models of the analytic significance (Sec. 3).
enum : int { SIG_MODEL_BINOMIAL = 0, SIG_MODEL_POISSON = 1 };

// Waves of the significance tail kernel in flight for n_q (a multiple of 4).
int significance_rows(int64_t n_q, int model);
// Scratch bytes for launch_significance with `rows` waves in flight.
size_t significance_scratch_bytes(int64_t n_p, int64_t n_q, int rows, int model);

// *S = analytic significance of num/(n_p n_q) from counts [N][2^d][2] (fp64),
// with num read from *num_dev when num_dev is not null (a device word written
// earlier on the same stream).  model: SIG_MODEL_*.  Sets bit 2 of *flags if
// a second-sample count exceeds n_q.
hipError_t launch_significance(const uint32_t *counts, int64_t N, int d, int64_t n_p, int64_t n_q,
                               uint64_t num, const uint64_t *num_dev, int model, void *scratch,
                               int rows, uint32_t *flags, double *S, hipStream_t s);

// res->ge = #{b : nums[b] >= res->num}.
hipError_t launch_count_ge(const unsigned long long *nums, int B, ResultDev *res, hipStream_t s);

}  // namespace ddks
