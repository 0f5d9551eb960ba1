// Batched registration: many independent registrations in one persistent launch
// over a shared work list, captured once in a HIP graph and replayed.
//
// The host prepares every instance exactly as the single-registration path does
// (same counter width, slab plan, x order and window table, same scorer data),
// writes one SweepArgs per instance and a work list of (instance, rotation tile)
// items sorted most expensive first, and launches
//   clear -> batched stage -> persistent k_sweep_batch -> batched select -> D2H
// The graph's kernel arguments only point at fixed device buffers whose contents
// are rewritten before each replay, so one captured graph serves any batch that
// fits the buffers' capacity.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <map>
#include <numeric>
#include <tuple>
#include <thread>
#include <vector>

#include "host.h"

namespace dses {

namespace {

struct Prepared {
    dses_status status = DSES_OK;
    Params p{};
    Geom g{};
    int scorer = DSES_SCORER_GRID;
    int32_t n = 0, m = 0, k = 0;
    const float *src = nullptr, *tgt = nullptr, *rot = nullptr;   // device pointers
    const float *host_src = nullptr, *host_tgt = nullptr, *host_rot = nullptr;
    std::vector<float> tgt_copy;           // host copy when the caller gave device memory
    const TargetRes *target = nullptr;
    std::vector<int32_t> perm_local;
    const std::vector<int32_t> *perm = nullptr;
    int32_t ylo = 0, yhi = 0;              // ref_x_range of the sorted reference
    bool sorted = false;
    HostGrid grid;                          // GRID scorer (non-resident targets)
    const float *grid_pts = nullptr;        // device (resident cache)
    const int32_t *grid_start = nullptr;
    // offsets into the arena (bytes)
    size_t off_src = 0, off_tgt = 0, off_rot = 0, off_yq = 0, off_yt = 0, off_perm = 0,
           off_rec = 0, off_gpts = 0, off_gstart = 0;
    void *records = nullptr;
    bool ready = false;
};

size_t bump(size_t &cursor, size_t bytes)
{
    const size_t at = cursor;
    cursor += (bytes + 255) & ~size_t(255);
    return at;
}

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    int scorer = -1;
    int cap_count = 0, cap_items = 0, grid = 0;
    hipStream_t stream = nullptr;
};

struct BatchState {
    DevBuf arena, inst, items, stage, sel, header, status, results, scratch;
    DevResult *host_res = nullptr;
    int cap_count = 0, cap_items = 0;
    size_t cap_scratch = 0;
    GraphCache graph[4];
};

BatchState *g_batch = nullptr;

// Launch layout of a batch: work-list granularity and vote window parts.
struct Layout {
    int items_per_cu = 24;
    int vote_parts = 0;                // 0: vote_parts_auto
};

// Tuned layouts by batch class (count, scorer, log2 buckets of total pairs, mean
// source size and mean rotation count), guarded by the context mutex.
struct ClassKey {
    int count, scorer, pairs_b, n_b, k_b;
    bool operator<(const ClassKey &o) const
    {
        return std::tie(count, scorer, pairs_b, n_b, k_b) <
               std::tie(o.count, o.scorer, o.pairs_b, o.n_b, o.k_b);
    }
};
std::map<ClassKey, std::pair<Layout, float>> g_tuned;

thread_local dses_batch_config t_last_config{};
thread_local bool t_have_config = false;

}  // namespace

static dses_status ensure_capacity(BatchState *b, int count, int n_items, size_t scratch_bytes)
{
    dses_status st;
    bool grew = false;
    if (count > b->cap_count) {
        const int cap = std::max(count, 64);
        // until every buffer below is in place the capacity reads 0, so a failed
        // allocation (which releases the old buffer) is retried by the next call
        b->cap_count = 0;
        if ((st = b->inst.ensure(cap * sizeof(SweepArgs))) != DSES_OK) return st;
        if ((st = b->stage.ensure(cap * sizeof(StageDesc))) != DSES_OK) return st;
        if ((st = b->sel.ensure(cap * sizeof(SelectDesc))) != DSES_OK) return st;
        if ((st = b->results.ensure(cap * sizeof(DevResult))) != DSES_OK) return st;
        if ((st = b->status.ensure(cap * sizeof(uint32_t) + 64)) != DSES_OK) return st;
        if (b->host_res) (void)hipHostFree(b->host_res);
        b->host_res = nullptr;
        void *hr = nullptr;
        DSES_HIP(host_alloc(&hr, cap * sizeof(DevResult), hipHostMallocDefault));
        b->host_res = static_cast<DevResult *>(hr);
        b->cap_count = cap;
        grew = true;
    }
    if (n_items > b->cap_items) {
        const int cap = std::max(n_items, 4096);
        b->cap_items = 0;
        if ((st = b->items.ensure(cap * sizeof(BatchItem))) != DSES_OK) return st;
        b->cap_items = cap;
        grew = true;
    }
    if ((st = b->header.ensure(64)) != DSES_OK) return st;
    if (scratch_bytes > b->cap_scratch) {
        b->cap_scratch = 0;
        if ((st = b->scratch.ensure(scratch_bytes)) != DSES_OK) return st;
        b->cap_scratch = b->scratch.bytes;
        grew = true;
    }
    if (grew)
        for (auto &gc : b->graph) {
            if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
            gc.exec = nullptr;
        }
    return DSES_OK;
}

// Enqueue (or capture) clear -> stage -> sweep -> select -> copy back.
static dses_status enqueue_batch(BatchState *b, int scorer, int grid, hipStream_t stream)
{
    uint32_t *status = static_cast<uint32_t *>(b->status.ptr);
    uint32_t *cursor = status + b->cap_count;      // one word after the per-instance flags
    const int32_t *header = static_cast<int32_t *>(b->header.ptr);
    DSES_HIP(launch_clear(cursor, 1, stream));
    DSES_HIP(launch_batch_aux(static_cast<StageDesc *>(b->stage.ptr), nullptr, header,
                              b->cap_count, 0, stream));
    BatchArgs ba{static_cast<SweepArgs *>(b->inst.ptr), static_cast<BatchItem *>(b->items.ptr),
                 header, cursor, nullptr};
    DSES_HIP(launch_sweep_batch(ba, scorer, grid, stream));
    DSES_HIP(launch_batch_aux(nullptr, static_cast<SelectDesc *>(b->sel.ptr), header,
                              b->cap_count, 1, stream));
    DSES_HIP(hipMemcpyAsync(b->host_res, b->results.ptr, b->cap_count * sizeof(DevResult),
                            hipMemcpyDeviceToHost, stream));
    return DSES_OK;
}

static dses_status run_graph(BatchState *b, int scorer, int grid, hipStream_t stream)
{
    GraphCache &gc = b->graph[scorer];
    if (!gc.exec || gc.cap_count != b->cap_count || gc.cap_items != b->cap_items ||
        gc.grid != grid || gc.stream != stream) {
        if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
        gc.exec = nullptr;
        hipGraph_t graph = nullptr;
        DSES_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        dses_status st = enqueue_batch(b, scorer, grid, stream);
        hipError_t e = hipStreamEndCapture(stream, &graph);
        if (st != DSES_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        DSES_HIP(e);
        e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        DSES_HIP(e);
        gc.scorer = scorer;
        gc.cap_count = b->cap_count;
        gc.cap_items = b->cap_items;
        gc.grid = grid;
        gc.stream = stream;
    }
    DSES_HIP(hipGraphLaunch(gc.exec, stream));
    return DSES_OK;
}

static int scorer_for(const Params &p, const TargetRes *t)
{
    int s = p.scorer;
    if (s == DSES_SCORER_AUTO)
        s = (t && t->df && t->df_r == p.r && p.metric != DSES_TRUNC_L1) ? DSES_SCORER_DF
                                                                           : DSES_SCORER_GRID;
    return s;
}

}  // namespace dses

using namespace dses;

extern "C" dses_status dses_register_batch(const dses_problem *probs, int32_t count,
                                           const dses_batch_opts *opt, dses_result *out,
                                           dses_status *status_out)
{
    set_error("");
    TraceRange range("dses.batch");
    if (!probs || !out || !status_out || count <= 0) {
        set_error("invalid batch arguments");
        return DSES_E_INVAL;
    }
    dses_batch_opts o{};
    if (opt) {
        const size_t given = opt->struct_size ? opt->struct_size : sizeof(dses_batch_opts);
        if (given < offsetof(dses_batch_opts, df_lookup) || given > sizeof(dses_batch_opts)) {
            set_error("dses_batch_opts.struct_size is not a size of this structure");
            return DSES_E_INVAL;
        }
        std::memcpy(&o, opt, given);
    }
    if (o.scorer < DSES_SCORER_AUTO || o.scorer > DSES_SCORER_DF || o.tile_rot < 0 ||
        o.vote_parts < 0 || o.vote_parts > 16 ||
        (o.df_lookup != DSES_DF_NEAREST && o.df_lookup != DSES_DF_TRILINEAR)) {
        set_error("invalid batch options");
        return DSES_E_INVAL;
    }
    const bool dev = (o.flags & DSES_DEVICE_PTRS) != 0;
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!g_batch) g_batch = new BatchState();
    BatchState *b = g_batch;
    hipStream_t stream = o.stream ? static_cast<hipStream_t>(o.stream) : c->stream;

    // ---------------- host preparation, instance by instance ----------------
    std::vector<Prepared> P(count);
    int batch_scorer = -1;
    int32_t max_n = 1;
    size_t arena_bytes = 0;
    auto prepare_one = [&](int i) {
        const dses_problem &q = probs[i];
        Prepared &x = P[i];
        auto fail = [&](dses_status s, const char *msg) {
            x.status = s;
            set_error(msg);
        };
        const TargetRes *T = q.target ? &q.target->res : nullptr;
        const int64_t m = T ? T->m : q.m;
        const int64_t k = q.rotset ? q.rotset->res.k : q.k;
        if (!q.src || q.n <= 0 || m <= 0 || k <= 0 || (!T && !q.tgt) ||
            (!q.rotset && !q.rotations) || q.n * m >= ((int64_t)1 << 31) || k > INT32_MAX) {
            fail(DSES_E_INVAL, "invalid problem sizes or pointers");
            return;
        }
        dses_status st = resolve_params(q.eps, q.metric, q.delta_t, q.tau, q.t_min, q.t_max,
                                        o.scorer, &x.p);
        if (st != DSES_OK) { x.status = st; return; }
        if (q.metric == DSES_TRUNC_LP || q.metric == DSES_VOTES) {
            fail(DSES_E_INVAL, "DSES_TRUNC_LP and DSES_VOTES are plain-path metrics");
            return;
        }
        x.n = (int32_t)q.n;
        x.m = (int32_t)m;
        x.k = (int32_t)k;
        x.target = T;
        x.scorer = scorer_for(x.p, T);
        if (x.scorer == DSES_SCORER_DF &&
            (!T || !T->df || T->df_r != x.p.r || x.p.metric == DSES_TRUNC_L1)) {
            fail(DSES_E_INVAL, "DF scorer needs a resident target with a matching field");
            return;
        }
        // host view of the reference
        const float *ht = nullptr;
        if (T) {
            ht = T->host_aos.data();
        } else if (!dev) {
            ht = q.tgt;
        } else {
            x.tgt_copy.resize(3 * (size_t)m);
            if (hipMemcpy(x.tgt_copy.data(), q.tgt, 3 * m * sizeof(float),
                          hipMemcpyDeviceToHost) != hipSuccess) {
                (void)hipGetLastError();
                fail(DSES_E_DEVICE, "reading the reference back failed");
                return;
            }
            ht = x.tgt_copy.data();
        }
        const float lim = ref_coord_limit(x.p);
        bool ok = true;
        for (int64_t e = 0; e < 3 * m && ok; ++e) ok = std::fabs(ht[e]) <= lim;
        if (!dev)
            for (int64_t e = 0; e < 3 * q.n && ok; ++e) ok = std::fabs(q.src[e]) <= kSrcCoordLimit;
        if (!dev && !q.rotset)
            for (int64_t r = 0; r < k && ok; ++r) {
                const float *R = q.rotations + 9 * r;
                for (int a = 0; a < 3 && ok; ++a)
                    for (int bb = 0; bb < 3 && ok; ++bb) {
                        float d = R[a] * R[bb] + R[3 + a] * R[3 + bb] + R[6 + a] * R[6 + bb];
                        d -= (a == bb) ? 1.0f : 0.0f;
                        ok = std::fabs(d) <= 1e-4f;
                    }
            }
        if (!ok) {
            fail(DSES_E_INVAL, "non-finite or out-of-range coordinate, or non-orthonormal rotation");
            return;
        }
        x.host_tgt = ht;
        const int64_t bound = T ? target_block_population(const_cast<TargetRes *>(T), x.p) * x.n
                                : counter_bound(ht, x.m, x.n, x.p);
        const int bits = counter_bits_for(bound, x.n, x.m, x.p);
        if ((st = plan_geom(c, x.p, x.n, x.m, bits, &x.g)) != DSES_OK) { x.status = st; return; }
        if (T) {
            auto *tm = const_cast<TargetRes *>(T);
            std::lock_guard<std::mutex> gl(tm->grid_mu);
            if (tm->perm_x.empty()) sort_by_x(ht, x.m, &tm->perm_x);
            x.perm = &tm->perm_x;
        } else {
            sort_by_x(ht, x.m, &x.perm_local);
            x.perm = &x.perm_local;
        }
        x.sorted = x.n <= kSortMax && ref_x_range(ht, *x.perm, x.p.delta, x.p.klo[0], &x.ylo, &x.yhi);
        if (x.scorer == DSES_SCORER_GRID) {
            if (T) {
                CellGrid cg{};
                if ((st = ensure_target_grid(const_cast<TargetRes *>(T), x.p.r, &cg)) != DSES_OK) {
                    x.status = st;
                    return;
                }
                x.grid_pts = cg.pts;
                x.grid_start = cg.start;
                for (int q = 0; q < 3; ++q) { x.grid.lo[q] = cg.lo[q]; x.grid.dim[q] = cg.dim[q]; }
                x.grid.inv = cg.inv;
            } else if ((st = build_grid(ht, x.m, x.p.r, &x.grid)) != DSES_OK) {
                x.status = st;
                return;
            }
        }
        x.ready = true;
    };
    {
        const int nt = std::max(1, std::min<int>(count, std::min<int>(16,
                                 (int)std::thread::hardware_concurrency())));
        std::vector<std::thread> pool;
        std::atomic<int> next{0};
        for (int w = 0; w < nt; ++w)
            pool.emplace_back([&] {
                (void)hipSetDevice(c->device);
                for (int i = next++; i < count; i = next++) prepare_one(i);
            });
        for (auto &t : pool) t.join();
    }
    for (int i = 0; i < count; ++i) {
        const dses_problem &q = probs[i];
        Prepared &x = P[i];
        if (x.status != DSES_OK) continue;
        if (batch_scorer >= 0 && x.scorer != batch_scorer) {
            x.status = DSES_E_INVAL;
            set_error("all problems of a batch must use the same scorer");
            continue;
        }
        const TargetRes *T = x.target;
        batch_scorer = x.scorer;
        max_n = std::max(max_n, x.n);
        // arena layout
        if (!dev) {
            x.off_src = bump(arena_bytes, 3 * (size_t)x.n * sizeof(float));
            if (!T) x.off_tgt = bump(arena_bytes, 3 * (size_t)x.m * sizeof(float));
            if (!q.rotset) x.off_rot = bump(arena_bytes, 9 * (size_t)x.k * sizeof(float));
        }
        x.off_yq = bump(arena_bytes, 4 * (size_t)x.m * sizeof(int32_t));
        x.off_yt = bump(arena_bytes, 3 * (size_t)x.m * sizeof(float));
        x.off_perm = bump(arena_bytes, (size_t)x.m * sizeof(int32_t));
        x.off_rec = bump(arena_bytes, (size_t)x.k * sizeof(dses_record));
        if (x.scorer == DSES_SCORER_GRID && !T) {
            x.off_gpts = bump(arena_bytes, x.grid.pts.size() * sizeof(float));
            x.off_gstart = bump(arena_bytes, x.grid.start.size() * sizeof(int32_t));
        }
        x.src = dev ? q.src : nullptr;
        x.tgt = T ? T->aos : (dev ? q.tgt : nullptr);
        x.rot = q.rotset ? q.rotset->res.rot : (dev ? q.rotations : nullptr);
        x.host_src = dev ? nullptr : q.src;
        x.host_rot = (dev || q.rotset) ? nullptr : q.rotations;
        x.records = q.records;
    }
    for (int i = 0; i < count; ++i) status_out[i] = P[i].status;
    if (batch_scorer < 0) return P[0].status;          // nothing valid to run

    // ---------------- device buffers and uploads ----------------
    const int grid = std::max(1, c->n_cu);
    dses_status st = b->arena.ensure(arena_bytes);
    if (st != DSES_OK) return st;
    char *arena = static_cast<char *>(b->arena.ptr);

    // work list: rotation tiles, most expensive first; the tile is sized so the list
    // holds about items_per_cu items per compute unit (or fixed by tile_rot)
    double total = 0.0, sum_n = 0.0, sum_k = 0.0;
    int n_ok = 0;
    for (auto &x : P)
        if (x.status == DSES_OK) {
            total += (double)x.n * x.m * x.k;
            sum_n += x.n;
            sum_k += x.k;
            ++n_ok;
        }
    auto build_items = [&](int items_per_cu, std::vector<BatchItem> *list) {
        const double target_cost = std::max(1.0, total / ((double)grid * items_per_cu));
        struct Tile { double cost; BatchItem it; };
        std::vector<Tile> tiles;
        for (int i = 0; i < count; ++i) {
            const Prepared &x = P[i];
            if (x.status != DSES_OK) continue;
            const double per_rot = (double)x.n * x.m + 1.0;
            const int tile = o.tile_rot > 0
                                 ? o.tile_rot
                                 : (int)std::max(1.0, std::min((double)x.k, target_cost / per_rot));
            for (int32_t k0 = 0; k0 < x.k; k0 += tile) {
                const int32_t k1 = std::min<int32_t>(x.k, k0 + tile);
                tiles.push_back({per_rot * (k1 - k0), BatchItem{i, k0, k1, 0}});
            }
        }
        std::stable_sort(tiles.begin(), tiles.end(),
                         [](const Tile &a, const Tile &bb) { return a.cost > bb.cost; });
        list->resize(tiles.size());
        for (size_t t = 0; t < tiles.size(); ++t) (*list)[t] = tiles[t].it;
    };
    static const int kItemsPerCu[] = {6, 12, 24, 48, 96};
    static const int kVoteParts[] = {1, 2, 4, 8};
    const bool tune = (o.flags & DSES_BATCH_TUNE) != 0;
    const bool caller_layout = o.tile_rot > 0 || o.vote_parts > 0;
    auto lg = [](double v) { return v >= 1.0 ? (int)std::floor(std::log2(v)) : 0; };
    const ClassKey key{count, batch_scorer, lg(total), lg(sum_n / std::max(1, n_ok)),
                       lg(sum_k / std::max(1, n_ok))};
    Layout lay;
    dses_batch_config cfg{};
    cfg.source = 0;
    if (!tune) {
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            lay = it->second.first;
            cfg.source = 2;
            cfg.sweep_ms = it->second.second;
        }
    }
    if (o.vote_parts > 0) lay.vote_parts = o.vote_parts;
    if (caller_layout && !tune) cfg.source = 3;
    std::vector<BatchItem> items;
    int max_items = 0;
    for (int f : kItemsPerCu) {
        if (!tune && f != lay.items_per_cu) continue;
        build_items(f, &items);
        max_items = std::max(max_items, (int)items.size());
    }
    build_items(lay.items_per_cu, &items);
    int n_items = (int)items.size();
    if ((st = ensure_capacity(b, count, max_items,
                              (size_t)grid * slot_words(max_n) * sizeof(int32_t))) != DSES_OK)
        return st;

    std::vector<SweepArgs> inst(b->cap_count);
    std::vector<StageDesc> stage(b->cap_count);
    std::vector<SelectDesc> sel(b->cap_count);
    uint32_t *status_dev = static_cast<uint32_t *>(b->status.ptr);
    DevResult *res_dev = static_cast<DevResult *>(b->results.ptr);
    for (int i = 0; i < count; ++i) {
        Prepared &x = P[i];
        StageDesc &sd = stage[i];
        SelectDesc &sl = sel[i];
        if (x.status != DSES_OK) {       // empty stage/select entries
            sd = StageDesc{nullptr, nullptr, 0, 1.0, 1.0, {0, 0, 0}, nullptr, nullptr};
            sl = SelectDesc{nullptr, 0, 1.0f, nullptr, res_dev + i, nullptr};
            continue;
        }
        if (x.host_src) {
            x.src = reinterpret_cast<float *>(arena + x.off_src);
            DSES_HIP(hipMemcpyAsync(const_cast<float *>(x.src), x.host_src,
                                    3 * (size_t)x.n * sizeof(float), hipMemcpyHostToDevice, stream));
        }
        if (!x.tgt) {
            x.tgt = reinterpret_cast<float *>(arena + x.off_tgt);
            DSES_HIP(hipMemcpyAsync(const_cast<float *>(x.tgt), x.host_tgt,
                                    3 * (size_t)x.m * sizeof(float), hipMemcpyHostToDevice, stream));
        }
        if (!x.rot) {
            x.rot = reinterpret_cast<float *>(arena + x.off_rot);
            DSES_HIP(hipMemcpyAsync(const_cast<float *>(x.rot), x.host_rot,
                                    9 * (size_t)x.k * sizeof(float), hipMemcpyHostToDevice, stream));
        }
        int32_t *perm_dev = reinterpret_cast<int32_t *>(arena + x.off_perm);
        DSES_HIP(hipMemcpyAsync(perm_dev, x.perm->data(), (size_t)x.m * sizeof(int32_t),
                                hipMemcpyHostToDevice, stream));
        SweepArgs &a = inst[i];
        a = SweepArgs{};
        a.src = x.src;
        a.rot = x.rot;
        a.yq = reinterpret_cast<int32_t *>(arena + x.off_yq);
        a.yt = reinterpret_cast<float *>(arena + x.off_yt);
        a.scratch = x.sorted ? static_cast<int32_t *>(b->scratch.ptr) : nullptr;
        a.scratch_stride = max_n;
        source_buckets(x.ylo, x.yhi, x.g.size[0], &a.sb_lo, &a.sb_shift, &a.sb_n);
        a.ref_x_extent = ref_x_extent(x.ylo, x.yhi);
        a.g = x.g;
        a.rec = reinterpret_cast<dses_record *>(arena + x.off_rec);
        a.k = x.k;
        a.vote_parts = lay.vote_parts;
        if (x.scorer == DSES_SCORER_GRID) {
            if (x.target) {
                a.grid.pts = x.grid_pts;
                a.grid.start = x.grid_start;
            } else {
                float *gp = reinterpret_cast<float *>(arena + x.off_gpts);
                int32_t *gs = reinterpret_cast<int32_t *>(arena + x.off_gstart);
                DSES_HIP(hipMemcpyAsync(gp, x.grid.pts.data(), x.grid.pts.size() * sizeof(float),
                                        hipMemcpyHostToDevice, stream));
                DSES_HIP(hipMemcpyAsync(gs, x.grid.start.data(),
                                        x.grid.start.size() * sizeof(int32_t),
                                        hipMemcpyHostToDevice, stream));
                a.grid.pts = gp;
                a.grid.start = gs;
            }
            for (int q = 0; q < 3; ++q) { a.grid.lo[q] = x.grid.lo[q]; a.grid.dim[q] = x.grid.dim[q]; }
            a.grid.inv = x.grid.inv;
        } else if (x.scorer == DSES_SCORER_DF) {
            a.field.val = x.target->df;
            a.field.res = x.target->df_res;
            a.field.r = x.target->df_r;
            a.field.lookup = o.df_lookup;
            for (int q = 0; q < 3; ++q) {
                a.field.lo[q] = x.target->df_lo[q];
                a.field.inv[q] = x.target->df_inv[q];
            }
        }
        sd = StageDesc{x.tgt, perm_dev, x.m, x.g.S16, x.g.S15,
                       {x.p.klo[0], x.p.klo[1], x.p.klo[2]}, const_cast<int32_t *>(a.yq),
                       const_cast<float *>(a.yt)};
        sl = SelectDesc{a.rec, x.k, x.p.delta, x.rot, res_dev + i, status_dev + i};
    }
    int32_t header[2] = {n_items, count};
    DSES_HIP(hipMemcpyAsync(b->inst.ptr, inst.data(), inst.size() * sizeof(SweepArgs),
                            hipMemcpyHostToDevice, stream));
    DSES_HIP(hipMemcpyAsync(b->stage.ptr, stage.data(), stage.size() * sizeof(StageDesc),
                            hipMemcpyHostToDevice, stream));
    DSES_HIP(hipMemcpyAsync(b->sel.ptr, sel.data(), sel.size() * sizeof(SelectDesc),
                            hipMemcpyHostToDevice, stream));
    DSES_HIP(hipMemcpyAsync(b->items.ptr, items.data(), items.size() * sizeof(BatchItem),
                            hipMemcpyHostToDevice, stream));
    DSES_HIP(hipMemcpyAsync(b->header.ptr, header, sizeof(header), hipMemcpyHostToDevice, stream));
    DSES_HIP(launch_clear(status_dev, b->cap_count, stream));
    if (dev)       // device-memory inputs are checked on the device, per instance
        for (int i = 0; i < count; ++i) {
            const Prepared &x = P[i];
            if (x.status != DSES_OK) continue;
            CheckArgs ca{x.src,          x.n, x.tgt, x.m, x.rot, x.k, kSrcCoordLimit,
                         ref_coord_limit(x.p), status_dev + i};
            DSES_HIP(launch_check(ca, stream));
        }
    // everything above must land before a captured graph is replayed
    DSES_HIP(hipStreamSynchronize(stream));

    if (tune) {
        // time the sweep alone for each candidate layout (stage once, then clear the
        // work cursor and sweep); one coordinate at a time: granularity with the
        // default vote split, then the vote split with the best granularity
        uint32_t *cursor = status_dev + b->cap_count;
        const int32_t *hdr_dev = static_cast<int32_t *>(b->header.ptr);
        DSES_HIP(launch_batch_aux(static_cast<StageDesc *>(b->stage.ptr), nullptr, hdr_dev,
                                  b->cap_count, 0, stream));
        hipEvent_t t0 = nullptr, t1 = nullptr;
        DSES_HIP(hipEventCreate(&t0));
        DSES_HIP(hipEventCreate(&t1));
        auto time_layout = [&](const Layout &L, float *ms) -> dses_status {
            build_items(L.items_per_cu, &items);
            header[0] = (int32_t)items.size();
            for (int i = 0; i < count; ++i) inst[i].vote_parts = L.vote_parts;
            DSES_HIP(hipMemcpyAsync(b->items.ptr, items.data(), items.size() * sizeof(BatchItem),
                                    hipMemcpyHostToDevice, stream));
            DSES_HIP(hipMemcpyAsync(b->header.ptr, header, sizeof(header), hipMemcpyHostToDevice,
                                    stream));
            DSES_HIP(hipMemcpyAsync(b->inst.ptr, inst.data(), count * sizeof(SweepArgs),
                                    hipMemcpyHostToDevice, stream));
            DSES_HIP(launch_clear(cursor, 1, stream));
            DSES_HIP(hipEventRecord(t0, stream));
            BatchArgs ba{static_cast<SweepArgs *>(b->inst.ptr),
                         static_cast<BatchItem *>(b->items.ptr), hdr_dev, cursor, nullptr};
            DSES_HIP(launch_sweep_batch(ba, batch_scorer, grid, stream));
            DSES_HIP(hipEventRecord(t1, stream));
            DSES_HIP(hipStreamSynchronize(stream));
            DSES_HIP(hipEventElapsedTime(ms, t0, t1));
            ++cfg.candidates;
            return DSES_OK;
        };
        Layout best = lay;
        float best_ms = INFINITY;
        dses_status tst = DSES_OK;
        if (o.tile_rot <= 0)
            for (int f : kItemsPerCu) {
                Layout L{f, best.vote_parts};
                float ms = 0.0f;
                if ((tst = time_layout(L, &ms)) != DSES_OK) break;
                if (ms < best_ms) { best_ms = ms; best = L; }
            }
        if (tst == DSES_OK && o.vote_parts <= 0)
            for (int gm : kVoteParts) {
                if (gm == best.vote_parts && best_ms < INFINITY) continue;
                Layout L{best.items_per_cu, gm};
                float ms = 0.0f;
                if ((tst = time_layout(L, &ms)) != DSES_OK) break;
                if (ms < best_ms) { best_ms = ms; best = L; }
            }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        if (tst != DSES_OK) return tst;
        lay = best;
        if (!caller_layout) g_tuned[key] = {best, best_ms};
        cfg.source = cfg.candidates > 0 ? 1 : 3;
        cfg.sweep_ms = cfg.candidates > 0 ? best_ms : 0.0f;
        // restore the chosen layout for the run below
        build_items(lay.items_per_cu, &items);
        n_items = (int)items.size();
        header[0] = n_items;
        for (int i = 0; i < count; ++i) inst[i].vote_parts = lay.vote_parts;
        DSES_HIP(hipMemcpyAsync(b->items.ptr, items.data(), items.size() * sizeof(BatchItem),
                                hipMemcpyHostToDevice, stream));
        DSES_HIP(hipMemcpyAsync(b->header.ptr, header, sizeof(header), hipMemcpyHostToDevice,
                                stream));
        DSES_HIP(hipMemcpyAsync(b->inst.ptr, inst.data(), count * sizeof(SweepArgs),
                                hipMemcpyHostToDevice, stream));
        DSES_HIP(hipStreamSynchronize(stream));
    }
    cfg.items_per_cu = o.tile_rot > 0 ? 0 : lay.items_per_cu;
    cfg.vote_parts = lay.vote_parts;
    cfg.n_items = n_items;

    const bool timing = (o.flags & DSES_TIMING) != 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing) {
        DSES_HIP(hipEventCreate(&e0));
        DSES_HIP(hipEventCreate(&e1));
        DSES_HIP(hipEventRecord(e0, stream));
    }
    if (o.use_graph) {
        if ((st = run_graph(b, batch_scorer, grid, stream)) != DSES_OK) return st;
    } else if ((st = enqueue_batch(b, batch_scorer, grid, stream)) != DSES_OK) {
        return st;
    }
    if (timing) DSES_HIP(hipEventRecord(e1, stream));
    DSES_HIP(hipStreamSynchronize(stream));
    if (timing) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        int64_t pairs = 0, cands = 0;
        for (auto &x : P)
            if (x.status == DSES_OK) {
                pairs += (int64_t)x.n * x.m * x.k;
                cands += x.k;
            }
        add_stats(c, ms, 0.0, 0.0, 0.0, 1, pairs, 0, cands);
    }

    // ---------------- results ----------------
    bool any_records = false;
    for (int i = 0; i < count; ++i) {
        Prepared &x = P[i];
        if (x.status != DSES_OK) continue;
        const DevResult &r = b->host_res[i];
        if (r.bad_input) {
            status_out[i] = DSES_E_INVAL;
            continue;
        }
        if (r.rot_index < 0) {
            status_out[i] = DSES_E_NOCANDIDATE;
            continue;
        }
        dses_result &o2 = out[i];
        std::memcpy(o2.R, r.R, sizeof(o2.R));
        std::memcpy(o2.t, r.t, sizeof(o2.t));
        o2.rot_index = r.rot_index;
        o2.inliers = r.inliers;
        o2.error = r.error;
        o2.votes = r.votes;
        o2.n_valid = r.n_valid;
        if (x.records) {
            DSES_HIP(hipMemcpyAsync(x.records, arena + x.off_rec,
                                    (size_t)x.k * sizeof(dses_record),
                                    dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, stream));
            any_records = true;
        }
    }
    if (any_records) DSES_HIP(hipStreamSynchronize(stream));
    t_last_config = cfg;
    t_have_config = true;
    for (int i = 0; i < count; ++i)
        if (status_out[i] != DSES_OK) return DSES_OK;     // per-problem statuses carry the detail
    return DSES_OK;
}

extern "C" dses_status dses_batch_last_config(dses_batch_config *out)
{
    set_error("");
    if (!out) {
        set_error("NULL output");
        return DSES_E_INVAL;
    }
    if (!t_have_config) {
        set_error("no batch has completed on this thread");
        return DSES_E_STATE;
    }
    *out = t_last_config;
    return DSES_OK;
}
