// Host-side internals of the DSES library: device context, workspace, argument
// resolution and the registration driver shared by the plain, resident, batched
// and serving entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <deque>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "dses.h"
#include "internal.h"

namespace dses {

void set_error(const std::string &msg);

#define DSES_HIP(expr)                                                                      \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) {                                                             \
            ::dses::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));           \
            return DSES_E_DEVICE;                                                           \
        }                                                                                   \
    } while (0)

// Every device and pinned-host allocation of the library goes through these,
// so that dses_debug_fail_allocs() can make chosen ones fail (tests of the
// error paths).  On failure *p is null.
hipError_t dev_alloc_raw(void **p, size_t bytes);
hipError_t host_alloc_raw(void **p, size_t bytes, unsigned int flags);
template <class T>
inline hipError_t dev_alloc(T **p, size_t bytes)
{
    void *v = nullptr;
    const hipError_t e = dev_alloc_raw(&v, bytes);
    *p = static_cast<T *>(v);
    return e;
}
template <class T>
inline hipError_t host_alloc(T **p, size_t bytes, unsigned int flags)
{
    void *v = nullptr;
    const hipError_t e = host_alloc_raw(&v, bytes, flags);
    *p = static_cast<T *>(v);
    return e;
}

// A roctx range on the calling thread (rocprofv3 --marker-trace records it)
// around a host-side phase of an entry point; end() closes it early.
struct TraceRange {
    bool open = true;
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    void end()
    {
        if (open) roctxRangePop();
        open = false;
    }
    ~TraceRange() { end(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// A device allocation that grows on demand (never shrinks while in use).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    dses_status ensure(size_t want);
    void release();
    ~DevBuf() { release(); }
};

// Pinned host buffer (hipHostMalloc), grown on demand.
struct PinnedBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    dses_status ensure(size_t want);
    void release();
    ~PinnedBuf() { release(); }
};

struct Context {
    int device = -1;
    int n_cu = 0;
    int lds_max = 0;
    std::string arch;
    hipStream_t stream = nullptr;
    std::mutex mu;                       // serialises the plain entry points
    // workspace of the plain path
    DevBuf in_src, in_tgt, in_rot, yq, yt, rec, res, status, grid_pts, grid_start, perm, scratch;
    DevBuf topk_a, topk_b, topk_out;     // top-k passes and output staging
    DevBuf prune;                        // q-pruning: M* and the work cursor
    DevResult *host_res = nullptr;       // pinned
    PinnedBuf host_stage;                // staging of host-built uploads (cell grid)
    // timing
    bool timing_enabled = false;
    std::mutex stats_mu;
    dses_kstats stats{};
};

// Returns the initialised context or nullptr (error set).
Context *ctx();

// Resolved numeric parameters of one registration.
struct Params {
    float eps, delta, tau, r;
    int32_t klo[3], size[3];
    int metric;
    int scorer;
    float lp = 0.5f;         // exponent of DSES_TRUNC_LP
    int32_t df_lookup = DSES_DF_NEAREST;   // how the DF scorer reads the field
};

// Applies the plain-path options that resolve_params does not see (the Lp
// exponent; q has no meaning with DSES_VOTES; lane_group is 0, 16, 32 or 64;
// the distance-field lookup).
// Host-side check, no device use.
dses_status apply_metric_options(const dses_options &o, Params *p);

dses_status resolve_params(float eps, int metric, float delta_t, float tau, const float *t_min,
                           const float *t_max, int scorer, Params *p);
// Largest |coordinate| accepted for a registration with these parameters.
// Largest accepted |coordinate|: reference points must keep the fixed-point
// lattice values in range (ref_coord_limit); a source point of any magnitude up
// to kSrcCoordLimit is accepted (its lattice value saturates where it can no
// longer vote).
float ref_coord_limit(const Params &p);
constexpr float kSrcCoordLimit = 1.0e4f;

// Counter width of the vote: 32 bits when some bin could reach 2^16 votes (the
// proven bound), and also when every 32-bit slab would still carry at least
// 2^20 pairs, where the two VALU of the 16-bit increment cost more than the
// doubled per-slab work (4,096 x 16,384 points, box 101^3, 2.0M pairs per 32-bit
// slab: 3.4% faster; 717 x 1,024 points, box 69^3, 82K pairs: 25% slower).
int counter_bits_for(int64_t bound, int32_t n, int32_t m, const Params &p);
dses_status plan_geom(const Context *c, const Params &p, int32_t n, int32_t m, int counter_bits,
                      Geom *g);
// Upper bound on any bin's vote count (decides 16- vs 32-bit LDS counters):
// n x the largest reference population of a 2 x 2 x 2 block of cells of pitch
// slightly above delta (for a fixed source point, the pairs sharing a bin have
// their references in one delta-cube).
int64_t ref_block_population(const float *tgt_aos, int32_t m, const Params &p);
int64_t counter_bound(const float *tgt_aos, int32_t m, int32_t n, const Params &p);

// Fixed-point lattice scales (1/delta) 2^16 and (1/delta) 2^15, in double.
void lattice_scales(float delta, double *S16, double *S15);

// Reference order sorted by x; the staged fixed-point x coordinates (2^-16 bins,
// lattice offset folded in, the staging arithmetic) of the first and last point
// of that order (false if the sorted sweep cannot be used); the source bucket
// origin, shift and count of a box of size_x x-planes.
void sort_by_x(const float *tgt_aos, int32_t m, std::vector<int32_t> *perm);
bool ref_x_range(const float *tgt_aos, const std::vector<int32_t> &perm, float delta,
                 int32_t klo_x, int32_t *ylo, int32_t *yhi);
void source_buckets(int32_t ylo, int32_t yhi, int32_t size_x, int32_t *sb_lo, int32_t *sb_shift,
                    int32_t *sb_n);
// x extent in bins of the staged reference (lane-group choice).
inline float ref_x_extent(int32_t ylo, int32_t yhi)
{
    return (float)((double)(yhi - ylo) / 65536.0) + 1.0f;
}

// Exact cell grid for the GRID scorer, built on the host from reference points.
struct HostGrid {
    std::vector<float> pts;      // x y z and a pad per point (16 B), cell order
    std::vector<int32_t> start;  // ncell + 1
    float lo[3];
    float inv;
    int32_t dim[3];
};
dses_status build_grid(const float *tgt_aos, int32_t m, float r, HostGrid *out);

// Resident reference cloud.
struct TargetRes {
    int32_t m = 0;
    float *aos = nullptr;            // m x 3 device copy
    float *yt = nullptr;             // SoA device copy
    std::vector<float> host_aos;     // host copy (grid builds)
    float max_abs = 0.0f;            // largest |coordinate| (lattice range check)
    // distance field
    float *df = nullptr;
    int32_t df_res = 0;
    float df_r = 0.0f;
    float df_lo[3] = {0, 0, 0}, df_h[3] = {0, 0, 0}, df_inv[3] = {0, 0, 0};
    // Caches, guarded by grid_mu.  Entries are never freed before the target is
    // destroyed: kernels of the serving loop may still read an older entry.
    std::mutex grid_mu;
    std::vector<int32_t> perm_x;             // reference order sorted by x
    int32_t *d_perm = nullptr;
    struct Stage {                           // staged copy for one (delta, box)
        float delta;
        int32_t klo[3];
        int32_t *yq;                         // fixed-point copy (4 m int32)
        float *yt;
        bool sorted;                         // ref_x_range succeeded
        int32_t ylo = 0, yhi = 0;            // its result
    };
    std::deque<Stage> stages;                // deque: references survive push_back
    struct Population {                      // ref_block_population for (delta, box)
        float delta;
        int32_t klo[3], size[3];
        int64_t pop;
    };
    std::vector<Population> pops;
    struct Grid {                            // cell grid for one radius
        float r;
        float *pts;
        int32_t *start;
        HostGrid meta;
    };
    std::deque<Grid> grids;
};

struct RotRes {
    int64_t k = 0;
    float *rot = nullptr;            // k x 9 device copy
};

// Everything the driver needs about one registration, with device pointers.
struct Job {
    const float *src = nullptr;      // n x 3, device
    int32_t n = 0;
    const float *tgt = nullptr;      // m x 3, device (AoS)
    int32_t m = 0;
    const float *rot = nullptr;      // k x 9, device
    int32_t k = 0;
    Params p{};
    const TargetRes *target = nullptr;   // resident reference (grid / field source)
    const float *host_tgt = nullptr;     // host AoS copy of the reference, if known
    bool exhaustive = false;             // Alg. 1: every lattice translation per rotation
};

// The option struct a caller passed, checked against its declared size (0: the
// full current size) and copied; missing trailing fields stay 0 (defaults).
dses_status copy_options(const dses_options *opt, dses_options *o);

// Device memory handed out from a fixed region instead of allocated: takes of
// 256-byte-aligned blocks from [base, base + cap); null when the region is spent.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    void *take(size_t bytes)
    {
        const size_t at = (used + 255) & ~size_t(255);
        if (at > cap || bytes > cap - at) return nullptr;
        used = at + bytes;
        return base + at;
    }
};

// Run one registration on `stream` using the context workspace (caller holds c->mu).
// With an arena every device buffer of the call comes from it and nothing is
// allocated (no timing events, no pinned staging, no top-k or pruning buffers).
dses_status run_plain(Context *c, const Job &job, hipStream_t stream, bool check_inputs,
                      dses_result *out, const dses_options &o, Arena *arena = nullptr);

void add_stats(Context *c, double vote_ms, double score_ms, double select_ms, double stage_ms,
               int64_t launches, int64_t pairs_voted, int64_t pairs_scored, int64_t cands);

// Stage a resident target for lattice pitch p.delta / box p.klo (cached; holds
// tm->grid_mu while building; synchronous on `stream`).
// ref_block_population of a resident target, cached per (delta, box).
int64_t target_block_population(TargetRes *tm, const Params &p);
dses_status ensure_target_stage(TargetRes *tm, const Params &p, hipStream_t stream,
                                const TargetRes::Stage **out);
// Build (or reuse) the resident target's cell grid for radius r; fills cg.
dses_status ensure_target_grid(TargetRes *tm, float r, CellGrid *cg);

// Distance field build (device), defined in field.hip.
hipError_t launch_df_build(const float *pts_soa, const int32_t *start, const HostGrid &grid,
                           int32_t res, const float *lo, const float *h, float r, float *out,
                           hipStream_t stream);

}  // namespace dses

struct dses_target {
    dses::TargetRes res;
};

struct dses_rotset {
    dses::RotRes res;
};
