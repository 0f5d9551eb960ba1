// DSES C ABI: context, argument checking and the plain registration driver.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "host.h"

namespace dses {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

namespace {
std::mutex g_fault_mu;
int64_t g_fault_skip = 0, g_fault_count = 0;   // dses_debug_fail_allocs

// true if this allocation is one the injection makes fail
bool injected_failure()
{
    std::lock_guard<std::mutex> lk(g_fault_mu);
    if (g_fault_count <= 0) return false;
    if (g_fault_skip > 0) {
        --g_fault_skip;
        return false;
    }
    --g_fault_count;
    return true;
}
}  // namespace

hipError_t dev_alloc_raw(void **p, size_t bytes)
{
    *p = nullptr;
    if (injected_failure()) return hipErrorOutOfMemory;
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) *p = nullptr;
    return e;
}

hipError_t host_alloc_raw(void **p, size_t bytes, unsigned int flags)
{
    *p = nullptr;
    if (injected_failure()) return hipErrorOutOfMemory;
    const hipError_t e = hipHostMalloc(p, bytes, flags);
    if (e != hipSuccess) *p = nullptr;
    return e;
}

dses_status DevBuf::ensure(size_t want)
{
    if (want <= bytes && ptr) return DSES_OK;
    release();
    size_t b = std::max<size_t>(want, 256);
    b = (b + 4095) & ~size_t(4095);
    if (dev_alloc(&ptr, b) != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        set_error("device allocation of " + std::to_string(b) + " bytes failed");
        return DSES_E_NOMEM;
    }
    bytes = b;
    return DSES_OK;
}

void DevBuf::release()
{
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

dses_status PinnedBuf::ensure(size_t want)
{
    if (want <= bytes && ptr) return DSES_OK;
    release();
    const size_t b = (std::max<size_t>(want, 4096) + 4095) & ~size_t(4095);
    if (host_alloc(&ptr, b, hipHostMallocDefault) != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        set_error("pinned host allocation of " + std::to_string(b) + " bytes failed");
        return DSES_E_NOMEM;
    }
    bytes = b;
    return DSES_OK;
}

void PinnedBuf::release()
{
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

static std::mutex g_init_mu;
static Context *g_ctx = nullptr;

static dses_status init_device(int device)
{
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (g_ctx) {
        if (device >= 0 && device != g_ctx->device) {
            set_error("library already initialised on another device");
            return DSES_E_STATE;
        }
        return DSES_OK;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        set_error("no HIP device available");
        return DSES_E_DEVICE;
    }
    if (device < 0) device = 0;
    if (device >= count) {
        set_error("device index out of range");
        return DSES_E_DEVICE;
    }
    hipDeviceProp_t prop;
    DSES_HIP(hipGetDeviceProperties(&prop, device));
    std::string arch = prop.gcnArchName;
    if (arch.rfind("gfx950", 0) != 0) {
        set_error("unsupported GPU architecture " + arch + " (gfx950 required)");
        return DSES_E_DEVICE;
    }
    DSES_HIP(hipSetDevice(device));
    auto *c = new Context();
    c->device = device;
    c->arch = arch;
    c->n_cu = prop.multiProcessorCount;
    int lds = 0;
    DSES_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    c->lds_max = std::min(lds, 160 * 1024);
    void *hr = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = host_alloc(&hr, sizeof(DevResult), hipHostMallocDefault);
    if (e != hipSuccess) {
        if (c->stream) (void)hipStreamDestroy(c->stream);
        delete c;
        DSES_HIP(e);
    }
    c->host_res = static_cast<DevResult *>(hr);
    g_ctx = c;
    return DSES_OK;
}

Context *ctx()
{
    if (!g_ctx && init_device(-1) != DSES_OK) return nullptr;
    if (g_ctx) (void)hipSetDevice(g_ctx->device);
    return g_ctx;
}

dses_status resolve_params(float eps, int metric, float delta_t, float tau, const float *t_min,
                           const float *t_max, int scorer, Params *p)
{
    if (!(eps > 0.0f) || !std::isfinite(eps)) {
        set_error("eps must be positive and finite");
        return DSES_E_INVAL;
    }
    if (metric < DSES_TRUNC_L2 || metric > DSES_VOTES) {
        set_error("unknown metric");
        return DSES_E_INVAL;
    }
    if (scorer < DSES_SCORER_AUTO || scorer > DSES_SCORER_DF) {
        set_error("unknown scorer");
        return DSES_E_INVAL;
    }
    p->eps = eps;
    p->delta = delta_t == 0.0f ? eps : delta_t;
    p->tau = tau == 0.0f ? eps : tau;
    if (!(p->delta > 0.0f) || !std::isfinite(p->delta) || !(p->tau > 0.0f) ||
        !std::isfinite(p->tau)) {
        set_error("delta_t and tau must be positive and finite");
        return DSES_E_INVAL;
    }
    p->r = std::max(p->eps, p->tau);
    p->metric = metric;
    p->scorer = scorer;
    float lo[3] = {-1.0f, -1.0f, -1.0f}, hi[3] = {1.0f, 1.0f, 1.0f};
    bool zero = true;
    if (t_min && t_max)
        for (int a = 0; a < 3; ++a) zero = zero && t_min[a] == 0.0f && t_max[a] == 0.0f;
    if (!zero)
        for (int a = 0; a < 3; ++a) { lo[a] = t_min[a]; hi[a] = t_max[a]; }
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(lo[a]) || !std::isfinite(hi[a])) {
            set_error("translation box must be finite");
            return DSES_E_INVAL;
        }
        const double kl = std::ceil((double)lo[a] / (double)p->delta - 1e-4);
        const double kh = std::floor((double)hi[a] / (double)p->delta + 1e-4);
        if (!(kh >= kl) || kh - kl + 1 > 4096 || std::fabs(kl) > 1e6 || std::fabs(kh) > 1e6) {
            set_error("translation box is empty or has more than 4096 bins per axis");
            return DSES_E_INVAL;
        }
        p->klo[a] = (int32_t)kl;
        p->size[a] = (int32_t)(kh - kl + 1);
    }
    return DSES_OK;
}

int counter_bits_for(int64_t bound, int32_t n, int32_t m, const Params &p)
{
    if (bound > 65535) return 32;
    const int64_t plane_words = (int64_t)p.size[1] * p.size[2];
    const int64_t pps = std::max<int64_t>(1, std::min<int64_t>((kHistWordsMax & ~3) / plane_words,
                                                               p.size[0]));
    const int64_t nslabs32 = (p.size[0] + pps - 1) / pps;
    return (int64_t)n * m >= (int64_t)nslabs32 << 20 ? 32 : 16;
}

dses_status plan_geom(const Context *c, const Params &p, int32_t n, int32_t m, int counter_bits,
                      Geom *g)
{
    (void)c;
    g->n = n;
    g->m = m;
    g->delta = p.delta;
    lattice_scales(p.delta, &g->S16, &g->S15);
    g->eps = p.eps;
    g->tau = p.tau;
    g->r = p.r;
    g->metric = p.metric;
    g->lp = p.lp;
    for (int a = 0; a < 3; ++a) { g->klo[a] = p.klo[a]; g->size[a] = p.size[a]; }
    g->counter_bits = counter_bits;
    g->row_words = counter_bits == 16 ? (p.size[2] + 1) / 2 : p.size[2];
    const int64_t plane_words = (int64_t)p.size[1] * g->row_words;
    const int64_t avail = kHistWordsMax & ~int64_t(3);
    int64_t pps = avail / plane_words;
    if (pps < 1) {
        set_error("translation box plane (size_y * size_z bins) does not fit in LDS");
        return DSES_E_INVAL;
    }
    pps = std::min<int64_t>(pps, p.size[0]);
    const int64_t nslabs = (p.size[0] + pps - 1) / pps;
    pps = (p.size[0] + nslabs - 1) / nslabs;
    g->pps = (int32_t)pps;
    g->nslabs = (int32_t)nslabs;
    g->slab_words = (int32_t)(pps * plane_words);
    g->wide = 4 * plane_words > 0xFFFF ? 1 : 0;
    return DSES_OK;
}

// Largest vote count any bin can reach: for a fixed source point the pairs that
// share a bin have reference points inside one cube of side delta (widened by the
// float rounding of the bin decision), and such a cube meets at most 2 cells per
// axis of a grid of pitch slightly above delta.  So every count is at most
// n * (largest reference population of a 2x2x2 block of cells).
int64_t ref_block_population(const float *tgt, int32_t m, const Params &p)
{
    double maxabs = 0.0;
    for (int64_t e = 0; e < 3 * (int64_t)m; ++e) maxabs = std::max(maxabs, (double)std::fabs(tgt[e]));
    int32_t kmax = 0;
    for (int a = 0; a < 3; ++a) kmax = std::max(kmax, std::abs(p.klo[a]) + p.size[a]);
    const double s = 1.0 / (double)p.delta;
    const double slack = 16.0 * 5.97e-8 * (4.0 * maxabs * s + kmax + 2.0);   // bin units
    const double h = (double)p.delta * (1.0 + std::max(1e-3, 4.0 * slack));
    auto key = [](int64_t x, int64_t y, int64_t z) {
        return ((x + (1 << 20)) << 42) | ((y + (1 << 20)) << 21) | (z + (1 << 20));
    };
    // points per cell of pitch h; the bound is the largest total of a block of
    // 2 x 2 x 2 cells.  When the cells span a modest box, counts go to a dense
    // array with a one-cell margin and each point's 8 blocks are summed there;
    // otherwise a hash map of cells and blocks gives the same number.
    std::vector<int64_t> ci(3 * (size_t)m);
    int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, hi[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
    for (int32_t j = 0; j < m; ++j)
        for (int a = 0; a < 3; ++a) {
            const int64_t c = (int64_t)std::floor((double)tgt[3 * j + a] / h);
            ci[3 * (size_t)j + a] = c;
            lo[a] = std::min(lo[a], c);
            hi[a] = std::max(hi[a], c);
        }
    if (m > 0 && hi[0] - lo[0] < (1 << 12) && hi[1] - lo[1] < (1 << 12) &&
        hi[2] - lo[2] < (1 << 12)) {
        const int64_t D1 = hi[1] - lo[1] + 3, D2 = hi[2] - lo[2] + 3;
        const int64_t cells = (hi[0] - lo[0] + 3) * D1 * D2;
        if (cells <= ((int64_t)1 << 21)) {
            thread_local std::vector<int32_t> cnt;       // all zero between calls
            if ((int64_t)cnt.size() < cells) cnt.assign((size_t)cells, 0);
            auto at = [&](int32_t j) {
                return ((ci[3 * (size_t)j] - lo[0] + 1) * D1 + (ci[3 * (size_t)j + 1] - lo[1] + 1)) * D2 +
                       (ci[3 * (size_t)j + 2] - lo[2] + 1);
            };
            for (int32_t j = 0; j < m; ++j) cnt[(size_t)at(j)] += 1;
            int64_t best = 0;
            for (int32_t j = 0; j < m; ++j) {
                const int64_t c = at(j);
                for (int ox = -1; ox <= 0; ++ox)
                    for (int oy = -1; oy <= 0; ++oy)
                        for (int oz = -1; oz <= 0; ++oz) {
                            const int64_t o = c + (ox * D1 + oy) * D2 + oz;    // block origin
                            int64_t sum = 0;
                            for (int dx = 0; dx <= 1; ++dx)
                                for (int dy = 0; dy <= 1; ++dy)
                                    for (int dz = 0; dz <= 1; ++dz)
                                        sum += cnt[(size_t)(o + (dx * D1 + dy) * D2 + dz)];
                            best = std::max(best, sum);
                        }
            }
            for (int32_t j = 0; j < m; ++j) cnt[(size_t)at(j)] = 0;
            return best;
        }
    }
    std::unordered_map<int64_t, int32_t> cell;
    cell.reserve((size_t)m * 2);
    for (int32_t j = 0; j < m; ++j)
        cell[key(ci[3 * (size_t)j], ci[3 * (size_t)j + 1], ci[3 * (size_t)j + 2])] += 1;
    std::unordered_map<int64_t, int64_t> block;
    block.reserve(cell.size() * 16);
    for (const auto &kv : cell) {
        const int64_t z = (kv.first & ((1 << 21) - 1)) - (1 << 20);
        const int64_t y = ((kv.first >> 21) & ((1 << 21) - 1)) - (1 << 20);
        const int64_t x = (kv.first >> 42) - (1 << 20);
        for (int ox = -1; ox <= 0; ++ox)
            for (int oy = -1; oy <= 0; ++oy)
                for (int oz = -1; oz <= 0; ++oz) block[key(x + ox, y + oy, z + oz)] += kv.second;
    }
    int64_t best = 0;
    for (const auto &kv : block) best = std::max(best, kv.second);
    return best;
}

int64_t counter_bound(const float *tgt, int32_t m, int32_t n, const Params &p)
{
    return ref_block_population(tgt, m, p) * (int64_t)n;
}

// ---------------------------------------------------------------------------
// exact cell grid (host build)
// ---------------------------------------------------------------------------
dses_status build_grid(const float *tgt, int32_t m, float r, HostGrid *out)
{
    // Cell pitch slightly above r so that, despite float rounding of the cell
    // index, every reference point within r of a query is in the 27 cells around
    // the query's cell.
    const float h = r * 1.001f;
    out->inv = 1.0f / h;
    float mn[3] = {tgt[0], tgt[1], tgt[2]}, mx[3] = {tgt[0], tgt[1], tgt[2]};
    for (int32_t j = 1; j < m; ++j)
        for (int a = 0; a < 3; ++a) {
            mn[a] = std::min(mn[a], tgt[3 * j + a]);
            mx[a] = std::max(mx[a], tgt[3 * j + a]);
        }
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        out->lo[a] = mn[a];
        const double span = ((double)mx[a] - (double)mn[a]) * (double)out->inv;
        out->dim[a] = (int32_t)std::floor(span) + 2;
        ncell *= out->dim[a];
    }
    if (ncell > (int64_t)64 << 20) {
        set_error("reference extent too large for the cell grid at this eps/tau");
        return DSES_E_INVAL;
    }
    std::vector<int32_t> cell(m);
    out->start.assign((size_t)ncell + 1, 0);
    for (int32_t j = 0; j < m; ++j) {
        int32_t id[3];
        for (int a = 0; a < 3; ++a) {
            const float u = (tgt[3 * j + a] - out->lo[a]) * out->inv;
            id[a] = std::min(std::max((int32_t)std::floor(u), 0), out->dim[a] - 1);
        }
        cell[j] = (id[0] * out->dim[1] + id[1]) * out->dim[2] + id[2];
        out->start[cell[j] + 1]++;
    }
    for (int64_t q = 0; q < ncell; ++q) out->start[q + 1] += out->start[q];
    std::vector<int32_t> cur(out->start.begin(), out->start.end() - 1);
    out->pts.assign((size_t)4 * m, 0.0f);
    for (int32_t j = 0; j < m; ++j) {
        const int32_t at = cur[cell[j]]++;
        for (int a = 0; a < 3; ++a) out->pts[(size_t)4 * at + a] = tgt[3 * j + a];
    }
    return DSES_OK;
}

// ---------------------------------------------------------------------------
// host-side input checks
// ---------------------------------------------------------------------------
// The fixed-point vote needs every staged reference value |y s + 1/2 - k_lo|
// below 2^13 bins, so that every pair difference and the padding values stay
// apart in 32 bits (a rotated source value is saturated at 2^14 bins instead:
// beyond it no pair with such a reference can land in the box).
float ref_coord_limit(const Params &p)
{
    int32_t kmax = 0;
    for (int a = 0; a < 3; ++a)
        kmax = std::max(kmax, std::max(std::abs(p.klo[a]), std::abs(p.klo[a] + p.size[a])));
    const double lim = ((double)(1 << 13) - kmax - 8.0) * (double)p.delta;
    return (float)std::min(std::max(lim, 0.0), 1.0e4);
}

static dses_status check_host_inputs(const float *src, int64_t n, const float *tgt, int64_t m,
                                     const float *rot, int64_t k, float limit)
{
    for (int64_t e = 0; e < 3 * n; ++e)
        if (!(std::fabs(src[e]) <= kSrcCoordLimit)) {
            set_error("source coordinate is non-finite or too large for the lattice");
            return DSES_E_INVAL;
        }
    if (tgt)
        for (int64_t e = 0; e < 3 * m; ++e)
            if (!(std::fabs(tgt[e]) <= limit)) {
                set_error("reference coordinate is non-finite or too large for the lattice");
                return DSES_E_INVAL;
            }
    if (rot)
        for (int64_t q = 0; q < k; ++q) {
            const float *R = rot + 9 * q;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    float d = R[i] * R[j] + R[3 + i] * R[3 + j] + R[6 + i] * R[6 + j];
                    d -= (i == j) ? 1.0f : 0.0f;
                    if (!(std::fabs(d) <= 1e-4f)) {
                        set_error("rotation " + std::to_string(q) +
                                  " is not orthonormal (|R^T R - I| > 1e-4) or not finite");
                        return DSES_E_INVAL;
                    }
                }
        }
    return DSES_OK;
}

void add_stats(Context *c, double vote_ms, double score_ms, double select_ms, double stage_ms,
               int64_t launches, int64_t pairs_voted, int64_t pairs_scored, int64_t cands)
{
    std::lock_guard<std::mutex> lk(c->stats_mu);
    c->stats.vote_score_ms += vote_ms;
    c->stats.score_ms += score_ms;
    c->stats.select_ms += select_ms;
    c->stats.stage_ms += stage_ms;
    c->stats.vote_score_launches += launches;
    c->stats.pairs_voted += pairs_voted;
    c->stats.pairs_scored += pairs_scored;
    c->stats.candidates += cands;
}

void sort_by_x(const float *tgt, int32_t m, std::vector<int32_t> *perm)
{
    // (x, index) pairs: ascending x, equal x in index order (a stable sort by x)
    std::vector<std::pair<float, int32_t>> kv((size_t)m);
    for (int32_t j = 0; j < m; ++j) kv[j] = {tgt[3 * (size_t)j], j};
    std::sort(kv.begin(), kv.end());
    perm->resize(m);
    for (int32_t j = 0; j < m; ++j) (*perm)[j] = kv[j].second;
}

void lattice_scales(float delta, double *S16, double *S15)
{
    const double s = 1.0 / (double)delta;
    *S16 = s * 65536.0;
    *S15 = s * 32768.0;
}

// The staging arithmetic of one reference x coordinate (two rounded double
// operations, then to the nearest integer, halves to even).
static int32_t stage_x(float y, double S16, int32_t klo_x)
{
    double v = (double)y * S16;
    v = v + (0.5 - (double)klo_x) * 65536.0;
    return (int32_t)std::nearbyint(v);
}

bool ref_x_range(const float *tgt, const std::vector<int32_t> &perm, float delta, int32_t klo_x,
                 int32_t *ylo, int32_t *yhi)
{
    if (perm.empty()) return false;
    double S16, S15;
    lattice_scales(delta, &S16, &S15);
    *ylo = stage_x(tgt[3 * (size_t)perm.front()], S16, klo_x);
    *yhi = stage_x(tgt[3 * (size_t)perm.back()], S16, klo_x);
    return *yhi >= *ylo;
}

void source_buckets(int32_t ylo, int32_t yhi, int32_t size_x, int32_t *sb_lo, int32_t *sb_shift,
                    int32_t *sb_n)
{
    // a source votes only if some Y - P lies in [0, size_x 2^16): P in
    // (ylo - size_x 2^16, yhi]
    const int64_t lo = (int64_t)ylo - ((int64_t)size_x << 16) + 1;
    const int64_t range = (int64_t)yhi - lo + 1;
    // 16 buckets per bin when the range fits: window ends are rounded to a bucket,
    // and finer buckets measured faster up to 16 (4,096-point sources against
    // 16,384 points: 2.4% against 4 per bin; 717 against 1,024: 0.3%; 32 per bin
    // no better, 64 slower)
    int shift = 12;
    while ((range >> shift) + 1 > kSrcBuckets && shift < 31) ++shift;
    *sb_lo = (int32_t)lo;
    *sb_shift = shift;
    // only as many buckets as the range needs (the sort clears and scans them all)
    const int64_t need = (range >> shift) + 2;
    *sb_n = (int32_t)std::min<int64_t>(kSrcBuckets, (need + kBlock - 1) / kBlock * kBlock);
}

dses_status apply_metric_options(const dses_options &o, Params *p)
{
    if (!(o.p >= 0.0f && o.p <= 1.0f)) {
        set_error("the Lp exponent p must be in (0, 1] (0: default 0.5)");
        return DSES_E_INVAL;
    }
    p->lp = o.p > 0.0f ? o.p : 0.5f;
    if (p->metric == DSES_VOTES && o.q > 0.0f) {
        set_error("q-pruning has no effect with DSES_VOTES");
        return DSES_E_INVAL;
    }
    if (o.lane_group != 0 && o.lane_group != 16 && o.lane_group != 32 && o.lane_group != 64) {
        set_error("lane_group must be 0 (automatic), 16, 32 or 64");
        return DSES_E_INVAL;
    }
    if (o.df_lookup != DSES_DF_NEAREST && o.df_lookup != DSES_DF_TRILINEAR) {
        set_error("df_lookup must be DSES_DF_NEAREST or DSES_DF_TRILINEAR");
        return DSES_E_INVAL;
    }
    p->df_lookup = o.df_lookup;
    return DSES_OK;
}

dses_status copy_options(const dses_options *opt, dses_options *o)
{
    *o = dses_options{};
    if (!opt) return DSES_OK;
    const size_t given = opt->struct_size ? opt->struct_size : sizeof(dses_options);
    // the first field that existed in every version ends at lane_group
    if (given < offsetof(dses_options, df_lookup) || given > sizeof(dses_options)) {
        set_error("dses_options.struct_size is not a size of this structure");
        return DSES_E_INVAL;
    }
    std::memcpy(o, opt, given);
    return DSES_OK;
}

static int effective_scorer(const Job &job)
{
    if (job.p.metric == DSES_VOTES) return kScoreVotes;
    int s = job.p.scorer;
    if (s == DSES_SCORER_AUTO)
        s = (job.target && job.target->df && job.target->df_r == job.p.r &&
             job.p.metric != DSES_TRUNC_L1)
                ? DSES_SCORER_DF
                : DSES_SCORER_GRID;
    return s;
}

// ---------------------------------------------------------------------------
// the plain driver
// ---------------------------------------------------------------------------
dses_status run_plain(Context *c, const Job &job, hipStream_t stream, bool check_inputs,
                      dses_result *out, const dses_options &o, Arena *arena)
{
    TraceRange whole("dses.registration");
    TraceRange prepare("dses.prepare");        // host work and staging before the launches
    // a device buffer of the call: from the arena when given, else the context's
    auto dbuf = [&](DevBuf &b, size_t bytes, void **ptr) -> dses_status {
        if (arena) {
            *ptr = arena->take(bytes);
            if (*ptr) return DSES_OK;
            set_error("the call needs more than the " + std::to_string(arena->cap >> 20) +
                      " MiB scratch array of the no-allocation entry point");
            return DSES_E_NOMEM;
        }
        const dses_status s = b.ensure(bytes);
        *ptr = b.ptr;
        return s;
    };
    if (arena && (o.q > 0.0f || o.top_k > 0 || c->timing_enabled || job.exhaustive)) {
        set_error("the no-allocation path takes no pruning, top-k, timing or Alg. 1");
        return DSES_E_INVAL;
    }
    const Params &p = job.p;
    void *records = o.records;
    const bool on_device = (o.flags & DSES_DEVICE_PTRS) != 0;
    if (o.top_k < 0 || o.top_k > DSES_TOPK_MAX || (o.top_k > 0 && !o.topk) ||
        !(o.q >= 0.0f && o.q <= 1.0f)) {
        set_error("top_k must be in 0..DSES_TOPK_MAX with a topk buffer, q in [0, 1]");
        return DSES_E_INVAL;
    }
    const int scorer = effective_scorer(job);
    if (scorer == DSES_SCORER_DF) {
        if (!job.target || !job.target->df) {
            set_error("DF scorer needs a resident target created with a distance field");
            return DSES_E_INVAL;
        }
        if (job.target->df_r != p.r) {
            set_error("distance field truncation must equal max(eps, tau)");
            return DSES_E_INVAL;
        }
        if (p.metric == DSES_TRUNC_L1) {
            set_error("the DF scorer does not support DSES_TRUNC_L1");
            return DSES_E_INVAL;
        }
    }
    const size_t m = (size_t)job.m;
    dses_status st;
    // host copy of the reference: needed for the counter bound and the cell grid
    std::vector<float> host_copy;
    const float *ht = job.target ? job.target->host_aos.data() : job.host_tgt;
    if (!ht) {
        host_copy.resize(3 * m);
        DSES_HIP(hipMemcpyAsync(host_copy.data(), job.tgt, 3 * m * sizeof(float),
                                hipMemcpyDeviceToHost, stream));
        DSES_HIP(hipStreamSynchronize(stream));
        for (float v : host_copy)
            if (!(std::fabs(v) <= ref_coord_limit(p))) {
                set_error("reference coordinate is non-finite or too large for the lattice");
                return DSES_E_INVAL;
            }
        ht = host_copy.data();
    }
    const int64_t bound =
        job.target ? target_block_population(const_cast<TargetRes *>(job.target), p) * job.n
                   : counter_bound(ht, job.m, job.n, p);
    const int counter_bits = counter_bits_for(bound, job.n, job.m, p);
    Geom g;
    if ((st = plan_geom(c, p, job.n, job.m, counter_bits, &g)) != DSES_OK) return st;

    // Reference sorted by x, and the range of its staged fixed-point x coordinate
    // (the same arithmetic as the staging kernel) for the source buckets, so each
    // wave can restrict its vote loop to reachable points.
    std::vector<int32_t> perm_local;
    const std::vector<int32_t> *perm = nullptr;
    if (job.target) {
        auto *tm = const_cast<TargetRes *>(job.target);
        std::lock_guard<std::mutex> lk(tm->grid_mu);
        if (tm->perm_x.empty()) sort_by_x(ht, job.m, &tm->perm_x);
        perm = &tm->perm_x;
    } else {
        sort_by_x(ht, job.m, &perm_local);
        perm = &perm_local;
    }
    int32_t ylo = 0, yhi = 0;
    const bool sorted = job.n <= kSortMax && ref_x_range(ht, *perm, p.delta, p.klo[0], &ylo, &yhi);
    const int grid = std::max(1, std::min(job.k, c->n_cu));
    void *d_perm = nullptr, *d_scratch = nullptr, *d_yq = nullptr, *d_yt = nullptr;
    void *d_rec = nullptr, *d_res = nullptr, *d_status = nullptr;
    if ((st = dbuf(c->perm, m * sizeof(int32_t), &d_perm)) != DSES_OK) return st;
    DSES_HIP(hipMemcpyAsync(d_perm, perm->data(), m * sizeof(int32_t), hipMemcpyHostToDevice,
                            stream));
    if (sorted && (st = dbuf(c->scratch, (size_t)grid * slot_words(job.n) * sizeof(int32_t),
                             &d_scratch)) != DSES_OK)
        return st;

    if ((st = dbuf(c->yq, 4 * m * sizeof(int32_t), &d_yq)) != DSES_OK) return st;
    if ((st = dbuf(c->yt, 3 * m * sizeof(float), &d_yt)) != DSES_OK) return st;
    // with an arena the records go straight to the caller's buffer when it gives one
    if (arena && records)
        d_rec = records;
    else if ((st = dbuf(c->rec, (size_t)job.k * sizeof(dses_record), &d_rec)) != DSES_OK)
        return st;
    if ((st = dbuf(c->res, sizeof(DevResult), &d_res)) != DSES_OK) return st;
    if ((st = dbuf(c->status, 64, &d_status)) != DSES_OK) return st;
    uint32_t *bad = static_cast<uint32_t *>(d_status);

    SweepArgs a{};
    a.src = job.src;
    a.rot = job.rot;
    a.yq = static_cast<int32_t *>(d_yq);
    a.yt = static_cast<float *>(d_yt);
    a.rec = static_cast<dses_record *>(d_rec);
    a.k = job.k;
    a.g = g;
    a.scratch = sorted ? static_cast<int32_t *>(d_scratch) : nullptr;
    a.scratch_stride = job.n;
    source_buckets(ylo, yhi, g.size[0], &a.sb_lo, &a.sb_shift, &a.sb_n);
    a.lane_group = o.lane_group;
    a.ref_x_extent = ref_x_extent(ylo, yhi);

    if (scorer == DSES_SCORER_GRID) {
        const TargetRes *t = job.target;
        if (t) {
            if ((st = ensure_target_grid(const_cast<TargetRes *>(t), p.r, &a.grid)) != DSES_OK)
                return st;
        } else {
            HostGrid hg;
            if ((st = build_grid(ht, job.m, p.r, &hg)) != DSES_OK) return st;
            const size_t pb = hg.pts.size() * sizeof(float), sb = hg.start.size() * sizeof(int32_t);
            void *d_pts = nullptr, *d_start = nullptr;
            if ((st = dbuf(c->grid_pts, pb, &d_pts)) != DSES_OK) return st;
            if ((st = dbuf(c->grid_start, sb, &d_start)) != DSES_OK) return st;
            if (arena) {
                // no pinned staging: the copies read the host vectors, which live
                // until this call's final synchronisation
                DSES_HIP(hipMemcpyAsync(d_pts, hg.pts.data(), pb, hipMemcpyHostToDevice, stream));
                DSES_HIP(hipMemcpyAsync(d_start, hg.start.data(), sb, hipMemcpyHostToDevice,
                                        stream));
                DSES_HIP(hipStreamSynchronize(stream));
            } else {
                // through pinned staging: the copies stay asynchronous (the buffer is
                // reused by the next call only after this call's final synchronisation)
                if ((st = c->host_stage.ensure(pb + sb)) != DSES_OK) return st;
                char *hs = static_cast<char *>(c->host_stage.ptr);
                std::memcpy(hs, hg.pts.data(), pb);
                std::memcpy(hs + pb, hg.start.data(), sb);
                DSES_HIP(hipMemcpyAsync(d_pts, hs, pb, hipMemcpyHostToDevice, stream));
                DSES_HIP(hipMemcpyAsync(d_start, hs + pb, sb, hipMemcpyHostToDevice, stream));
            }
            a.grid.pts = static_cast<float *>(d_pts);
            a.grid.start = static_cast<int32_t *>(d_start);
            for (int q = 0; q < 3; ++q) { a.grid.lo[q] = hg.lo[q]; a.grid.dim[q] = hg.dim[q]; }
            a.grid.inv = hg.inv;
        }
    } else if (scorer == DSES_SCORER_DF) {
        const TargetRes *t = job.target;
        a.field.val = t->df;
        a.field.res = t->df_res;
        a.field.r = t->df_r;
        a.field.lookup = job.p.df_lookup;
        for (int q = 0; q < 3; ++q) { a.field.lo[q] = t->df_lo[q]; a.field.inv[q] = t->df_inv[q]; }
    }

    const bool timing = c->timing_enabled;
    hipEvent_t ev[4] = {};
    if (timing)
        for (auto &e : ev) DSES_HIP(hipEventCreate(&e));
    auto rec_ev = [&](int i) { if (timing) (void)hipEventRecord(ev[i], stream); };

    prepare.end();
    TraceRange device("dses.sweep_select");    // launches to the result on the host
    rec_ev(0);
    DSES_HIP(launch_clear(bad, 16, stream));
    if (check_inputs) {
        CheckArgs ca{job.src,  job.n, job.tgt, job.m, job.rot, job.k, kSrcCoordLimit,
                     ref_coord_limit(p), bad};
        DSES_HIP(launch_check(ca, stream));
    }
    DSES_HIP(launch_stage(job.tgt, static_cast<int32_t *>(d_perm), job.m, g.S16, g.S15, p.klo,
                          static_cast<int32_t *>(d_yq), static_cast<float *>(d_yt), stream));
    rec_ev(1);
    if (job.exhaustive) {
        DSES_HIP(launch_exhaustive(a, scorer, grid, stream));
    } else if (o.q > 0.0f) {
        if ((st = c->prune.ensure(64)) != DSES_OK) return st;
        uint32_t *pw = static_cast<uint32_t *>(c->prune.ptr);
        DSES_HIP(launch_sweep(a, kScoreNone, grid, stream));
        DSES_HIP(launch_score_pruned(a, scorer, o.q, pw, pw + 1, grid, stream));
    } else {
        DSES_HIP(launch_sweep(a, scorer, grid, stream));
    }
    rec_ev(2);
    DSES_HIP(launch_select(a.rec, job.k, job.rot, p.delta, static_cast<DevResult *>(d_res), bad,
                           stream));
    rec_ev(3);
    DSES_HIP(hipMemcpyAsync(c->host_res, d_res, sizeof(DevResult), hipMemcpyDeviceToHost, stream));
    DSES_HIP(hipStreamSynchronize(stream));
    device.end();
    const DevResult r = *c->host_res;
    if (timing) {
        float t01 = 0, t12 = 0, t23 = 0;
        (void)hipEventElapsedTime(&t01, ev[0], ev[1]);
        (void)hipEventElapsedTime(&t12, ev[1], ev[2]);
        (void)hipEventElapsedTime(&t23, ev[2], ev[3]);
        for (auto &e : ev) (void)hipEventDestroy(e);
        const int64_t pairs = (int64_t)job.n * job.m * job.k;
        add_stats(c, t12, 0.0, t23, t01, 1, pairs, scorer == DSES_SCORER_BRUTE ? pairs : 0, job.k);
    }
    if (r.bad_input) {
        set_error("non-finite or out-of-range coordinate, or non-orthonormal rotation");
        return DSES_E_INVAL;
    }
    if (r.rot_index < 0) {
        set_error("no rotation received a vote inside the translation box");
        return DSES_E_NOCANDIDATE;
    }
    if (records && records != (void *)a.rec) {
        DSES_HIP(hipMemcpyAsync(records, a.rec, (size_t)job.k * sizeof(dses_record),
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                stream));
    }
    if (o.top_k > 0) {
        const size_t sb = topk_scratch_bytes(job.k, o.top_k);
        if ((st = c->topk_a.ensure(sb)) != DSES_OK) return st;
        if ((st = c->topk_b.ensure(sb)) != DSES_OK) return st;
        if ((st = c->topk_out.ensure(DSES_TOPK_MAX * sizeof(dses_candidate))) != DSES_OK) return st;
        auto *dst = on_device ? static_cast<dses_candidate *>(o.topk)
                              : static_cast<dses_candidate *>(c->topk_out.ptr);
        DSES_HIP(launch_topk(a.rec, job.k, o.top_k, p.delta, c->topk_a.ptr, c->topk_b.ptr, dst,
                             stream));
        if (!on_device)
            DSES_HIP(hipMemcpyAsync(o.topk, dst, (size_t)o.top_k * sizeof(dses_candidate),
                                    hipMemcpyDeviceToHost, stream));
    }
    if (records || o.top_k > 0) DSES_HIP(hipStreamSynchronize(stream));
    if (out) {
        std::memcpy(out->R, r.R, sizeof(out->R));
        std::memcpy(out->t, r.t, sizeof(out->t));
        out->rot_index = r.rot_index;
        out->inliers = r.inliers;
        out->error = r.error;
        out->votes = r.votes;
        out->n_valid = r.n_valid;
    }
    return DSES_OK;
}

}  // namespace dses

using namespace dses;

extern "C" {

const char *dses_last_error(void) { return g_err.c_str(); }

const char *dses_version(void) { return "dses-mi355x 0.1"; }

dses_status dses_init(int32_t device) { return init_device(device); }

dses_status dses_debug_fail_allocs(int32_t skip, int32_t count)
{
    if (skip < 0 || count < 0) {
        set_error("dses_debug_fail_allocs: negative argument");
        return DSES_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(g_fault_mu);
    g_fault_skip = count > 0 ? skip : 0;
    g_fault_count = count;
    return DSES_OK;
}

dses_status dses_kernel_stats(dses_kstats *out, int32_t reset)
{
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    std::lock_guard<std::mutex> lk(c->stats_mu);
    if (out) *out = c->stats;
    if (reset) c->stats = dses_kstats{};
    return DSES_OK;
}

dses_status dses_register(const float *src, int64_t n, const float *tgt, int64_t m,
                          const float *rotations, int64_t k, float eps, dses_metric metric,
                          const dses_options *opt, dses_result *out)
{
    set_error("");
    if (!src || !tgt || !rotations || !out) {
        set_error("NULL pointer argument");
        return DSES_E_INVAL;
    }
    if (n <= 0 || m <= 0 || k <= 0 || k > INT32_MAX || n * m >= ((int64_t)1 << 31)) {
        set_error("n, m, k must be positive with n*m < 2^31 and k < 2^31");
        return DSES_E_INVAL;
    }
    dses_options o;
    if (copy_options(opt, &o) != DSES_OK) return DSES_E_INVAL;
    if (o.top_k < 0 || o.top_k > DSES_TOPK_MAX || (o.top_k > 0 && !o.topk) ||
        !(o.q >= 0.0f && o.q <= 1.0f)) {
        set_error("top_k must be in 0..DSES_TOPK_MAX with a topk buffer, q in [0, 1]");
        return DSES_E_INVAL;
    }
    Params p;
    dses_status st = resolve_params(eps, metric, o.delta_t, o.tau, o.t_min, o.t_max, o.scorer, &p);
    if (st != DSES_OK) return st;
    if ((st = apply_metric_options(o, &p)) != DSES_OK) return st;
    if (p.scorer == DSES_SCORER_DF && p.metric != DSES_VOTES) {
        set_error("the DF scorer needs a resident target (dses_register_resident)");
        return DSES_E_INVAL;
    }
    const bool dev = (o.flags & DSES_DEVICE_PTRS) != 0;
    if (!dev) {
        st = check_host_inputs(src, n, tgt, m, rotations, k, ref_coord_limit(p));
        if (st != DSES_OK) return st;
    }
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    std::lock_guard<std::mutex> lk(c->mu);
    c->timing_enabled = (o.flags & DSES_TIMING) != 0;
    hipStream_t stream = o.stream ? static_cast<hipStream_t>(o.stream) : c->stream;
    Job job;
    job.n = (int32_t)n;
    job.m = (int32_t)m;
    job.k = (int32_t)k;
    job.p = p;
    if (dev) {
        job.src = src;
        job.tgt = tgt;
        job.rot = rotations;
    } else {
        if ((st = c->in_src.ensure(3 * n * sizeof(float))) != DSES_OK) return st;
        if ((st = c->in_tgt.ensure(3 * m * sizeof(float))) != DSES_OK) return st;
        if ((st = c->in_rot.ensure(9 * k * sizeof(float))) != DSES_OK) return st;
        DSES_HIP(hipMemcpyAsync(c->in_src.ptr, src, 3 * n * sizeof(float), hipMemcpyHostToDevice,
                                stream));
        DSES_HIP(hipMemcpyAsync(c->in_tgt.ptr, tgt, 3 * m * sizeof(float), hipMemcpyHostToDevice,
                                stream));
        DSES_HIP(hipMemcpyAsync(c->in_rot.ptr, rotations, 9 * k * sizeof(float),
                                hipMemcpyHostToDevice, stream));
        job.src = static_cast<float *>(c->in_src.ptr);
        job.tgt = static_cast<float *>(c->in_tgt.ptr);
        job.rot = static_cast<float *>(c->in_rot.ptr);
        job.host_tgt = tgt;
    }
    return run_plain(c, job, stream, dev, out, o);
}

dses_status dses_register_exhaustive(const float *src, int64_t n, const float *tgt, int64_t m,
                                     const float *rotations, int64_t k, float eps,
                                     dses_metric metric, const dses_options *opt,
                                     dses_result *out)
{
    set_error("");
    if (!src || !tgt || !rotations || !out) {
        set_error("NULL pointer argument");
        return DSES_E_INVAL;
    }
    if (n <= 0 || m <= 0 || k <= 0 || k > INT32_MAX || n * m >= ((int64_t)1 << 31) ||
        n > kExhaustiveMaxSrc) {
        set_error("n, m, k must be positive with n*m < 2^31 and n <= 12288");
        return DSES_E_INVAL;
    }
    dses_options o;
    if (copy_options(opt, &o) != DSES_OK) return DSES_E_INVAL;
    if (o.top_k != 0 || o.q != 0.0f) {
        set_error("top_k and q are not options of the exhaustive search");
        return DSES_E_INVAL;
    }
    Params p;
    dses_status st = resolve_params(eps, metric, o.delta_t, o.tau, o.t_min, o.t_max, o.scorer, &p);
    if (st != DSES_OK) return st;
    if ((st = apply_metric_options(o, &p)) != DSES_OK) return st;
    if (p.metric == DSES_VOTES || p.scorer == DSES_SCORER_DF) {
        set_error("the exhaustive search scores with BRUTE or GRID and a robust metric");
        return DSES_E_INVAL;
    }
    if ((int64_t)p.size[0] * p.size[1] * p.size[2] > INT32_MAX) {
        set_error("the exhaustive search takes at most 2^31 - 1 translations per rotation");
        return DSES_E_INVAL;
    }
    const bool dev = (o.flags & DSES_DEVICE_PTRS) != 0;
    if (!dev) {
        st = check_host_inputs(src, n, tgt, m, rotations, k, ref_coord_limit(p));
        if (st != DSES_OK) return st;
    }
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    std::lock_guard<std::mutex> lk(c->mu);
    c->timing_enabled = (o.flags & DSES_TIMING) != 0;
    hipStream_t stream = o.stream ? static_cast<hipStream_t>(o.stream) : c->stream;
    Job job;
    job.n = (int32_t)n;
    job.m = (int32_t)m;
    job.k = (int32_t)k;
    job.p = p;
    job.exhaustive = true;
    if (dev) {
        job.src = src;
        job.tgt = tgt;
        job.rot = rotations;
    } else {
        if ((st = c->in_src.ensure(3 * n * sizeof(float))) != DSES_OK) return st;
        if ((st = c->in_tgt.ensure(3 * m * sizeof(float))) != DSES_OK) return st;
        if ((st = c->in_rot.ensure(9 * k * sizeof(float))) != DSES_OK) return st;
        DSES_HIP(hipMemcpyAsync(c->in_src.ptr, src, 3 * n * sizeof(float), hipMemcpyHostToDevice,
                                stream));
        DSES_HIP(hipMemcpyAsync(c->in_tgt.ptr, tgt, 3 * m * sizeof(float), hipMemcpyHostToDevice,
                                stream));
        DSES_HIP(hipMemcpyAsync(c->in_rot.ptr, rotations, 9 * k * sizeof(float),
                                hipMemcpyHostToDevice, stream));
        job.src = static_cast<float *>(c->in_src.ptr);
        job.tgt = static_cast<float *>(c->in_tgt.ptr);
        job.rot = static_cast<float *>(c->in_rot.ptr);
        job.host_tgt = tgt;
    }
    return run_plain(c, job, stream, dev, out, o);
}

}  // extern "C"
