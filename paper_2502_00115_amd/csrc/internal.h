// Internal declarations shared by the DSES device kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dses.h"

namespace dses {

constexpr int kBlock = 1024;            // threads per sweep workgroup (16 wave64s)
constexpr int kWaves = kBlock / 64;
constexpr int kLdsWords = 40960;        // 160 KB of LDS per workgroup on gfx950
// LDS words after the vote array: per-wave partials of the slab scans (8..39),
// the scorer's sums (64..111), the sort's prefix (112..127), the unit counter and
// the occupied source-bucket range (128..130), two words at the very end for the
// batched kernels.  Kept small so that four 101 x 101 planes of 32-bit counters
// fit in one slab.
constexpr int kScratchWords = 136;
constexpr int kHistWordsMax = kLdsWords - kScratchWords;

// Per-registration constants of the sweep.
struct Geom {
    double S16, S15;       // (1/delta) 2^16 and (1/delta) 2^15: fixed-point lattice scales
    int32_t n, m;          // source / reference sizes
    float delta;           // lattice pitch
    float eps, tau;        // inlier threshold, truncation
    float r;               // max(eps, tau): the only neighbourhood that matters
    int32_t klo[3];        // lattice index of bin 0 per axis
    int32_t size[3];       // bins per axis
    int32_t metric;        // dses_metric
    float lp;              // exponent of DSES_TRUNC_LP
    int32_t counter_bits;  // 16: two counters per LDS word (z rows padded to even), 32: one
    int32_t row_words;     // LDS words per z row: (size_z + 1) / 2 or size_z
    int32_t pps;           // x-planes per LDS slab
    int32_t nslabs;        // slabs covering size[0]
    int32_t slab_words;    // LDS words of one full slab (<= kHistWordsMax)
    int32_t wide;          // 1: the x stride in bytes (4 size_y row_words) exceeds 16 bits
};

// Uniform cell grid over the reference for the exact GRID scorer.
struct CellGrid {
    const float *pts;      // reference points in cell order, x y z and a pad per point (4 * m floats)
    const int32_t *start;  // cell start offsets, ncell + 1 entries
    float lo[3];           // grid origin
    float inv;             // 1 / cell pitch
    int32_t dim[3];        // cells per axis
};

// Voxel distance field for the DF scorer.
struct Field {
    const float *val;      // res^3 values, x slowest
    float lo[3];
    float inv[3];          // 1 / voxel pitch per axis
    int32_t res;
    float r;               // value outside the grid
    int32_t lookup;        // dses_df_lookup: nearest voxel or trilinear
};

// Per-rotation source sort: sb_n buckets (a multiple of the block size, at most
// kSrcBuckets) over the fixed-point x coordinate, 2^(16 - sb_shift) buckets per
// bin (16 when the reachable range fits).
constexpr int kSrcBuckets = 8192;
constexpr int kSortMax = 16384;         // largest source cloud that is bucket-sorted
// Vote work units per 64-point lane group when not fixed by the caller: enough
// units for every wave to take several (at most 8 per group).
__host__ __device__ inline int vote_parts_auto(int groups)
{
    const int g = 64 / (groups > 0 ? groups : 1);
    return g < 1 ? 1 : (g > 8 ? 8 : g);
}
// Lane groups of the sorted-source vote: 2^(lg+1) reference points (64, 32 or
// 16), two per lane on 2^lg lanes, repeated on the wave's 64 >> lg lane
// sub-groups, which take alternate 4-source pieces of the same stream window, so
// a wave step covers 2^(lg+1) points x (64 >> lg) sources.  Smaller groups span
// less x, so their windows carry less slack (about 2^(lg+1) * X source-bins per
// slab over all groups, X the reference's x extent in bins), but there are more
// work units, each costing about kUnitSteps wave steps of set-up, padding and
// slab-end imbalance (fitted); rho = n / (X + size_x) sources per bin turns a step
// into 64 / rho source-bins.  The size with the least modelled cost wins (ties:
// the larger group).  It picks 16 points for a 717-point source against a
// 1,024-point reference with eps 0.03 and 64 for 64 / 256 points and for 4,096 /
// 16,384 points.
constexpr float kUnitSteps = 4.9f;
__host__ __device__ inline int lane_group_log2(int m, int n, int size_x, float x_extent,
                                               int vote_parts)
{
    const float per_unit = kUnitSteps * 64.0f * (x_extent + (float)size_x) /
                           (float)(n > 0 ? n : 1);
    int best = 5;
    float best_cost = 0.0f;
    for (int lg = 5; lg >= 3; --lg) {
        const int gref = 2 << lg;
        const int groups = (m + gref - 1) / gref;
        const int parts = vote_parts > 0 ? vote_parts : vote_parts_auto(groups);
        const float cost = (float)gref * x_extent + per_unit * (float)(groups * parts);
        if (lg == 5 || cost < best_cost) {
            best_cost = cost;
            best = lg;
        }
    }
    return best;
}
constexpr int kUnitCounter = 128;       // LDS scratch word: next vote work unit
constexpr int kSrcBmin = 129;           // LDS scratch words: lowest and highest occupied
constexpr int kSrcBmax = 130;           // source bucket of the current rotation
// Kernel scorer value for a vote-only sweep (records unscored: error +inf,
// 0 inliers); the public scorers are DSES_SCORER_BRUTE / GRID / DF.
constexpr int kScoreNone = 0;
// Kernel scorer value of DSES_VOTES: no scoring, records carry error 0 and
// inliers = the mode count, so the selection ranks candidates by it.
constexpr int kScoreVotes = 4;
// Largest source of the exhaustive search (rotated sources held in LDS).
constexpr int kExhaustiveMaxSrc = 12288;

struct SweepArgs {
    const float *src;      // n x 3 AoS
    const float *rot;      // K x 9
    const int32_t *yq;     // fixed-point reference (lattice offset folded in), sorted by x:
                           // four arrays of m, x, y, z at 2^-16 bins and z at 2^-15 bins
    const float *yt;       // reference, SoA (3 * m), same order
    int32_t *scratch;      // per workgroup slot: the rotation's sources sorted by x (below)
    int64_t scratch_stride;   // sources a slot holds (>= n)
    int32_t sb_lo, sb_shift;  // source bucket of P: (P - sb_lo) >> sb_shift, clamped
    int32_t sb_n;             // to [0, sb_n)
    Geom g;
    CellGrid grid;
    Field field;
    dses_record *rec;      // one record per rotation index
    int32_t k;             // rotations
    int32_t vote_parts;    // stream-window parts per lane group (0: vote_parts_auto)
    int32_t lane_group;    // reference points per lane group: 16, 32, 64 (0: lane_group_log2)
    float ref_x_extent;    // x extent of the scaled reference in bins (lane-group choice)
};

// Scratch slot of one workgroup (int32 words): rotated fixed-point sources sorted
// by x as three arrays x, y, z of src_stride(cap) entries each (entries n ..
// stride-1 hold padding that never votes, so windows can be padded to a multiple
// of 4), then the bucket table T[0 .. kSrcBuckets] (T[b] = sources in buckets
// below b).
__host__ __device__ inline int64_t src_stride(int64_t cap) { return (cap + 15) & ~int64_t(15); }
__host__ __device__ inline int64_t slot_words(int64_t cap)
{
    return (3 * src_stride(cap) + kSrcBuckets + 1 + 3) & ~int64_t(3);
}

// Batched registration.
struct DevResult;

struct BatchItem {
    int32_t inst;          // instance index
    int32_t k0, k1;        // rotation range [k0, k1)
    int32_t pad;
};

struct BatchArgs {
    const SweepArgs *inst;     // per-instance sweep arguments (device)
    const BatchItem *items;    // work list, most expensive first
    const int32_t *header;     // header[0] = items, header[1] = instances
    uint32_t *cursor;          // work-list cursor, cleared before each launch
    int32_t *scratch;          // if set: this launch's source-sort scratch (overrides
                               // the instances' own, so concurrent launches never share),
    int64_t scratch_slot;      // slot_words() of each workgroup's part of it
    // In-kernel completion (serving; unused when done_rot is null).  The cursor is
    // then never cleared: a launch fetches exactly items + grid times, so the host
    // passes the value it holds at launch.  done_rot counts each instance's swept
    // rotations (zero at rest); the workgroup whose tile completes an instance
    // selects its result into res, returns the count to zero and sets the flag.
    uint32_t cursor_base;
    uint32_t *done_rot;        // per instance (device memory)
    DevResult *res;            // per instance (host memory mapped for the device)
    uint32_t *done_flag;       // per instance, set to 1 after res (host memory)
};

struct StageDesc {
    const float *tgt;
    const int32_t *perm;
    int32_t m;
    double S16, S15;
    int32_t klo[3];
    int32_t *yq;
    float *yt;
};

struct SelectDesc {
    const dses_record *rec;
    int32_t k;
    float delta;
    const float *rot;
    DevResult *res;
    const uint32_t *status;
};

// Result written on the device by the select kernel.
struct DevResult {
    int32_t rot_index;
    uint32_t votes;
    int32_t inliers;
    float error;
    float t[3];
    float R[9];
    int32_t n_valid;
    uint32_t bad_input;
};

struct CheckArgs {
    const float *src; int32_t n;
    const float *tgt; int32_t m;
    const float *rot; int32_t k;
    float src_limit;       // max |source coordinate| accepted
    float ref_limit;       // max |reference coordinate| accepted
    uint32_t *bad;         // set to non-zero on invalid input
};

// Launchers (defined in kernels.hip); all enqueue on `stream`.
hipError_t launch_check(const CheckArgs &a, hipStream_t stream);
hipError_t launch_stage(const float *tgt, const int32_t *perm, int32_t m, double S16, double S15,
                        const int32_t *klo, int32_t *yq, float *yt, hipStream_t stream);
hipError_t launch_sweep(const SweepArgs &a, int scorer, int grid, hipStream_t stream);
hipError_t launch_select(const dses_record *rec, int32_t k, const float *rot, float delta,
                         DevResult *res, const uint32_t *status, hipStream_t stream);
// Top-k candidates of K records in selection order (k <= DSES_TOPK_MAX): passes of
// workgroup sorts reduce 2048 entries to k each until one workgroup remains; the
// scratch buffers hold ceil(K / 2048) * k entries of 12 bytes each.
size_t topk_scratch_bytes(int32_t K, int32_t k);
hipError_t launch_topk(const dses_record *rec, int32_t K, int32_t k, float delta, void *scr_a,
                       void *scr_b, dses_candidate *out, hipStream_t stream);
// q-pruned scoring after a kScoreNone sweep: M* into *mstar, then score the
// rotations with M_k >= q M* (both device words, the cursor cleared here).
hipError_t launch_score_pruned(const SweepArgs &a, int scorer, float q, uint32_t *mstar,
                               uint32_t *cursor, int grid, hipStream_t stream);
// Alg. 1 (every lattice translation of the box per rotation, scored with the
// BRUTE or GRID scorer): one record per rotation with its best translation.
hipError_t launch_exhaustive(const SweepArgs &a, int scorer, int grid, hipStream_t stream);
hipError_t launch_clear(uint32_t *p, int32_t words, hipStream_t stream);
hipError_t launch_sweep_batch(const BatchArgs &b, int scorer, int grid, hipStream_t stream);
// which = 0: batched staging, 1: batched selection
hipError_t launch_batch_aux(const StageDesc *stage, const SelectDesc *sel, const int32_t *header,
                            int max_count, int which, hipStream_t stream);

}  // namespace dses
