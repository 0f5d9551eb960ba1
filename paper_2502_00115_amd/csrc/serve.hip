// Serving: a request loop with memory-based admission and continuous batching.
//
// Clients submit registrations against resident reference clouds and rotation
// lists.  A scheduler thread owns all device work of the server:
//  * admission: FIFO, a request enters the device when its buffers fit the
//    memory budget (a first-fit pool carved from one allocation made at create
//    time, so admission never calls hipMalloc/hipFree) and an instance slot is
//    free;
//  * continuous batching: the GPU runs a sequence of short persistent launches
//    ("slices") of the batched sweep kernel, alternating between two streams so
//    one slice's tail overlaps the next slice's start.  Each slice's work list
//    takes rotation tiles from the requests on the device in priority order
//    (estimated remaining GPU time minus `aging` x time since submission), so
//    requests that arrive while others run join the next slice and their
//    rotations overlap on the device with the older requests';
//  * a request completes inside the sweep: the workgroup whose tile finishes
//    its last rotations selects its result into host memory and raises a flag
//    the scheduler polls; its memory then returns to the pool.
// Each rotation runs the same sweep_one() as a lone registration, so a request's
// result does not depend on what it was served with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <thread>
#include <vector>

#include "host.h"

namespace dses {
namespace {

using Clock = std::chrono::steady_clock;

constexpr int kSliceSets = 3;               // slices in flight + one being filled
constexpr int kMaxSliceItems = 8192;
constexpr int32_t kServeMaxSrc = 16384;     // largest source a request may carry
// pinned staging per slot: the source, then its SweepArgs
constexpr size_t kSlotStageBytes = ((12 * (size_t)kServeMaxSrc + sizeof(SweepArgs)) + 255) & ~size_t(255);

// First-fit allocator over one device allocation (offsets in bytes).
struct Pool {
    size_t size = 0;
    std::map<size_t, size_t> free_;         // offset -> length
    void init(size_t n) { size = n; free_.clear(); free_[0] = n; }
    bool alloc(size_t n, size_t *off)
    {
        n = (n + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + 255) & ~size_t(255);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Request {
    uint64_t id = 0;
    const TargetRes *target = nullptr;
    const RotRes *rots = nullptr;
    std::vector<float> src;
    int32_t n = 0, m = 0, k = 0;
    Params p{};
    int scorer = DSES_SCORER_GRID;
    // lifecycle
    enum State { QUEUED, ADMITTED, DONE } state = QUEUED;
    dses_status status = DSES_OK;
    dses_result out{};
    Clock::time_point t_submit, t_admit, t_done;
    // device residency
    size_t off = 0, bytes = 0;
    int slot = -1;
    bool ready = false;                      // its uploads are complete
    bool copying = false;                    // top-k / record copies enqueued on `down`
    int32_t next_k = 0;                      // rotations handed to slices so far
    double pair_cost = 0.0;                  // n * m per rotation
    dses_record *d_rec = nullptr;            // records inside the request's pool range
    // optional outputs (caller-owned host buffers, filled before DONE)
    dses_record *host_rec = nullptr;
    dses_candidate *host_topk = nullptr;
    int32_t top_k = 0;
    void *d_topk_a = nullptr, *d_topk_b = nullptr;   // top-k passes, in the pool range
    dses_candidate *d_topk = nullptr;
};

struct SliceSet {
    BatchItem *h_items = nullptr;            // host memory the slice's kernel reads in place
    int32_t *h_header = nullptr;             // host memory: items in the slice
    const BatchItem *dv_items = nullptr;     // their device addresses
    const int32_t *dv_header = nullptr;
    uint32_t *d_cursor = nullptr;            // work-list cursor, never cleared
    uint32_t cursor = 0;                     // its value when the next launch starts
    int32_t *d_scratch = nullptr;            // source-sort scratch of this slice's launch
    hipEvent_t swept = nullptr;              // the slice's sweep is complete
    hipStream_t stream = nullptr;            // stream the slice ran on
    bool busy = false;
    double pairs = 0.0;
    int n_last = 0;                          // requests whose last tile is in the slice
    Clock::time_point t_launch;
    std::vector<uint64_t> carried;           // ids of the requests with tiles in the slice (trace)
};

}  // namespace

struct ServerImpl {
    Context *c = nullptr;
    dses_server_opts opt{};
    // Streams.  A sweep workgroup holds a whole CU (all of its LDS and registers),
    // so any other kernel -- the runtime's copy kernels included -- waits for a
    // sweep workgroup to finish.  Nothing a slice needs is therefore ordered
    // behind such a kernel: a request joins slices only once its uploads are seen
    // complete, and top-k passes and copies to caller buffers are polled.
    hipStream_t up = nullptr;                // admission uploads and staging
    hipStream_t down = nullptr;              // top-k passes and copies to caller buffers
    hipEvent_t up_done = nullptr;            // recorded after every admission's uploads
    std::vector<Request *> uploading;        // admitted, uploads not yet seen complete
    hipStream_t stream = nullptr;            // even slices
    hipStream_t stream2 = nullptr;           // odd slices
    uint64_t n_slices = 0;
    double rate = 5.0e11;                    // estimated sweep rate, pairs per second
    void *pool_mem = nullptr;
    Pool pool;
    int max_slots = 0;
    SweepArgs *d_args = nullptr;             // one per slot
    uint32_t *d_done = nullptr;              // per slot: rotations swept (kernel-owned)
    DevResult *h_res = nullptr;              // per slot, host memory written by the kernel
    uint32_t *h_flag = nullptr;              // per slot, raised by the kernel after h_res
    DevResult *dv_res = nullptr;             // device addresses of h_res and h_flag
    uint32_t *dv_flag = nullptr;
    std::vector<hipEvent_t> slot_event;      // per slot: end of a request's copies
    float *h_stage = nullptr;                // pinned per-slot source staging
    SliceSet sets[kSliceSets];
    int grid = 0;
    double slice_pairs = 0.0;
    // shared state
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::vector<Request *> active;           // admitted, not finished
    std::map<uint64_t, Request *> all;
    std::vector<int> free_slots;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    std::string fatal;
    // optional trace (environment DSES_SERVE_TRACE=<file>): one line per finished
    // slice and per finished request, times in seconds since the server started
    FILE *trace = nullptr;
    Clock::time_point t0 = Clock::now();
    double since(Clock::time_point t) const { return std::chrono::duration<double>(t - t0).count(); }

    dses_status init(Context *ctx, const dses_server_opts &o);
    void run();
    bool admit_locked();
    bool launch_slice();
    void poll_slices();
    bool finish(Request *r);
    size_t need_bytes(const Request &r) const;
    dses_status prepare(Request *r);
    ~ServerImpl();
};

size_t ServerImpl::need_bytes(const Request &r) const
{
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    size_t b = al(12 * (size_t)r.n) + al(24 * (size_t)r.k);
    if (r.top_k > 0)
        b += 2 * al(topk_scratch_bytes(r.k, r.top_k)) + al(sizeof(dses_candidate) * r.top_k);
    return b;
}

dses_status ServerImpl::init(Context *ctx, const dses_server_opts &o)
{
    c = ctx;
    opt = o;
    if (opt.memory_budget <= 0) opt.memory_budget = (int64_t)1 << 30;
    if (opt.max_inflight <= 0) opt.max_inflight = 64;
    if (opt.aging == 0.0f) opt.aging = 3.0f;
    if (opt.aging < 0.0f) opt.aging = 0.0f;
    max_slots = opt.max_inflight;
    slice_pairs = 1.0e6 * (opt.slice_mpairs > 0 ? opt.slice_mpairs : 48000);
    // The slice streams must sit on two different hardware queues: kernels of one
    // queue never overlap, and streams created the ordinary way share a small
    // pool of queues (two of them can land on the same one).  A stream created
    // with a CU mask gets a queue of its own; the mask here covers every CU.
    grid = std::max(1, c->n_cu);
    std::vector<uint32_t> slice_mask((size_t)(grid + 31) / 32, 0u);
    for (int cu = 0; cu < grid; ++cu) slice_mask[(size_t)cu / 32] |= 1u << (cu % 32);
    DSES_HIP(hipExtStreamCreateWithCUMask(&stream, (uint32_t)slice_mask.size(), slice_mask.data()));
    DSES_HIP(hipExtStreamCreateWithCUMask(&stream2, (uint32_t)slice_mask.size(), slice_mask.data()));
    DSES_HIP(hipStreamCreateWithFlags(&up, hipStreamNonBlocking));
    DSES_HIP(hipStreamCreateWithFlags(&down, hipStreamNonBlocking));
    DSES_HIP(hipEventCreateWithFlags(&up_done, hipEventDisableTiming));
    DSES_HIP(hipEventRecord(up_done, up));
    if (dev_alloc(&pool_mem, (size_t)opt.memory_budget) != hipSuccess) {
        (void)hipGetLastError();
        set_error("cannot reserve the serving memory budget on the device");
        return DSES_E_NOMEM;
    }
    pool.init((size_t)opt.memory_budget);
    DSES_HIP(dev_alloc(&d_args, max_slots * sizeof(SweepArgs)));
    DSES_HIP(dev_alloc(&d_done, max_slots * sizeof(uint32_t)));
    DSES_HIP(hipMemset(d_done, 0, max_slots * sizeof(uint32_t)));
    // host memory the kernels read or write in place: coherent (not cached by
    // the device), mapped into the device's address space
    void *p = nullptr;
    auto host_mapped = [&](size_t bytes, void **h, void **dv) {
        DSES_HIP(host_alloc(h, bytes, hipHostMallocCoherent | hipHostMallocMapped));
        std::memset(*h, 0, bytes);
        const hipError_t e = hipHostGetDevicePointer(dv, *h, 0);
        if (e != hipSuccess) {
            (void)hipHostFree(*h);
            *h = nullptr;
        }
        DSES_HIP(e);
        return DSES_OK;
    };
    void *dv = nullptr;
    if (host_mapped(max_slots * sizeof(DevResult), &p, &dv) != DSES_OK) return DSES_E_DEVICE;
    h_res = static_cast<DevResult *>(p);
    dv_res = static_cast<DevResult *>(dv);
    if (host_mapped(max_slots * sizeof(uint32_t), &p, &dv) != DSES_OK) return DSES_E_DEVICE;
    h_flag = static_cast<uint32_t *>(p);
    dv_flag = static_cast<uint32_t *>(dv);
    DSES_HIP(host_alloc(&p, (size_t)max_slots * kSlotStageBytes, hipHostMallocDefault));
    h_stage = static_cast<float *>(p);
    for (auto &s : sets) {
        if (host_mapped(kMaxSliceItems * sizeof(BatchItem), &p, &dv) != DSES_OK) return DSES_E_DEVICE;
        s.h_items = static_cast<BatchItem *>(p);
        s.dv_items = static_cast<const BatchItem *>(dv);
        if (host_mapped(64, &p, &dv) != DSES_OK) return DSES_E_DEVICE;
        s.h_header = static_cast<int32_t *>(p);
        s.dv_header = static_cast<const int32_t *>(dv);
        DSES_HIP(dev_alloc(&s.d_cursor, 64));
        DSES_HIP(hipMemset(s.d_cursor, 0, 64));
        DSES_HIP(dev_alloc(&s.d_scratch, (size_t)grid * slot_words(kServeMaxSrc) * sizeof(int32_t)));
        DSES_HIP(hipEventCreateWithFlags(&s.swept, hipEventDisableTiming));
    }
    DSES_HIP(hipDeviceSynchronize());
    slot_event.assign(max_slots, nullptr);
    for (auto &e : slot_event) DSES_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (int i = max_slots - 1; i >= 0; --i) free_slots.push_back(i);
    if (const char *tp = std::getenv("DSES_SERVE_TRACE")) trace = std::fopen(tp, "w");
    t0 = Clock::now();
    worker = std::thread([this] { run(); });
    return DSES_OK;
}

ServerImpl::~ServerImpl()
{
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv_work.notify_all();
    if (worker.joinable()) worker.join();
    if (up) (void)hipStreamSynchronize(up);
    if (down) (void)hipStreamSynchronize(down);
    if (stream) (void)hipStreamSynchronize(stream);
    if (stream2) (void)hipStreamSynchronize(stream2);
    if (up_done) (void)hipEventDestroy(up_done);
    for (auto &s : sets) {
        if (s.d_scratch) (void)hipFree(s.d_scratch);
        if (s.h_items) (void)hipHostFree(s.h_items);
        if (s.h_header) (void)hipHostFree(s.h_header);
        if (s.d_cursor) (void)hipFree(s.d_cursor);
        if (s.swept) (void)hipEventDestroy(s.swept);
    }
    for (auto e : slot_event)
        if (e) (void)hipEventDestroy(e);
    if (h_res) (void)hipHostFree(h_res);
    if (h_flag) (void)hipHostFree(h_flag);
    if (h_stage) (void)hipHostFree(h_stage);
    if (d_args) (void)hipFree(d_args);
    if (d_done) (void)hipFree(d_done);
    if (pool_mem) (void)hipFree(pool_mem);
    if (up) (void)hipStreamDestroy(up);
    if (down) (void)hipStreamDestroy(down);
    if (stream) (void)hipStreamDestroy(stream);
    if (stream2) (void)hipStreamDestroy(stream2);
    for (auto &kv : all) delete kv.second;
    if (trace) std::fclose(trace);
}

// Device preparation of an admitted request (scheduler thread; the request owns
// its pool range and slot): the reference is staged once per target and pitch
// (cached), so a request only uploads its source and its sweep arguments, both
// from the slot's pinned staging area, asynchronously on the upload stream; its
// tiles join slices once those uploads are seen complete.
dses_status ServerImpl::prepare(Request *r)
{
    auto *tm = const_cast<TargetRes *>(r->target);
    const int bits = counter_bits_for(target_block_population(tm, r->p) * r->n, r->n, r->m, r->p);
    Geom g;
    dses_status st = plan_geom(c, r->p, r->n, r->m, bits, &g);
    if (st != DSES_OK) return st;
    const TargetRes::Stage *stg = nullptr;
    if ((st = ensure_target_stage(tm, r->p, up, &stg)) != DSES_OK) return st;
    CellGrid cg{};
    if (r->scorer == DSES_SCORER_GRID && (st = ensure_target_grid(tm, r->p.r, &cg)) != DSES_OK)
        return st;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    char *base = static_cast<char *>(pool_mem) + r->off;
    float *d_src = reinterpret_cast<float *>(base);
    r->d_rec = reinterpret_cast<dses_record *>(base + al(12 * (size_t)r->n));
    if (r->top_k > 0) {
        char *tk = base + al(12 * (size_t)r->n) + al(24 * (size_t)r->k);
        const size_t sb = al(topk_scratch_bytes(r->k, r->top_k));
        r->d_topk_a = tk;
        r->d_topk_b = tk + sb;
        r->d_topk = reinterpret_cast<dses_candidate *>(tk + 2 * sb);
    }
    char *stage = reinterpret_cast<char *>(h_stage) + (size_t)r->slot * kSlotStageBytes;
    std::memcpy(stage, r->src.data(), 12 * (size_t)r->n);
    SweepArgs &a = *reinterpret_cast<SweepArgs *>(stage + 12 * (size_t)kServeMaxSrc);
    a = SweepArgs{};
    a.src = d_src;
    a.rot = r->rots->rot;
    a.yq = stg->yq;
    a.yt = stg->yt;
    const bool sorted = r->n <= kSortMax && stg->sorted;
    a.scratch = sorted ? reinterpret_cast<int32_t *>(4) : nullptr;   // per-slice scratch at launch
    a.scratch_stride = r->n;                 // arrays inside the slice's fixed-size slots
    source_buckets(stg->ylo, stg->yhi, g.size[0], &a.sb_lo, &a.sb_shift, &a.sb_n);
    a.ref_x_extent = ref_x_extent(stg->ylo, stg->yhi);
    a.g = g;
    a.grid = cg;
    if (r->scorer == DSES_SCORER_DF) {
        a.field.val = tm->df;
        a.field.res = tm->df_res;
        a.field.r = tm->df_r;
        a.field.lookup = r->p.df_lookup;
        for (int q = 0; q < 3; ++q) { a.field.lo[q] = tm->df_lo[q]; a.field.inv[q] = tm->df_inv[q]; }
    }
    a.rec = r->d_rec;
    a.k = r->k;
    DSES_HIP(hipMemcpyAsync(d_src, stage, 12 * (size_t)r->n, hipMemcpyHostToDevice, up));
    DSES_HIP(hipMemcpyAsync(d_args + r->slot, &a, sizeof(SweepArgs), hipMemcpyHostToDevice, up));
    DSES_HIP(hipEventRecord(up_done, up));
    return DSES_OK;
}

bool ServerImpl::admit_locked()
{
    bool any = false;
    while (!queue.empty()) {
        Request *r = queue.front();
        if (free_slots.empty()) break;
        size_t off = 0;
        if (!pool.alloc(r->bytes, &off)) break;      // wait for memory to be returned
        queue.pop_front();
        r->off = off;
        r->slot = free_slots.back();
        free_slots.pop_back();
        r->t_admit = Clock::now();
        __atomic_store_n(h_flag + r->slot, 0u, __ATOMIC_RELEASE);
        mu.unlock();
        dses_status st = prepare(r);
        mu.lock();
        if (st != DSES_OK) {
            r->status = st;
            r->state = Request::DONE;
            r->t_done = Clock::now();
            pool.release(r->off, r->bytes);
            free_slots.push_back(r->slot);
            cv_done.notify_all();
            continue;
        }
        r->state = Request::ADMITTED;
        active.push_back(r);
        uploading.push_back(r);
        any = true;
    }
    return any;
}

// Fill and launch one slice from the active requests (scheduler thread, mu held).
bool ServerImpl::launch_slice()
{
    SliceSet *s = nullptr;
    for (auto &cand : sets)
        if (!cand.busy) { s = &cand; break; }
    if (!s) return false;
    std::vector<Request *> order;
    for (Request *r : active)
        if (r->ready && r->next_k < r->k) order.push_back(r);
    if (order.empty()) return false;
    const auto now = Clock::now();
    const double aging = opt.aging;
    auto prio = [&](const Request *r) {
        const double remaining = (r->k - r->next_k) * r->pair_cost / rate;
        const double age = std::chrono::duration<double>(now - r->t_submit).count();
        return remaining - aging * age;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](const Request *a, const Request *b) { return prio(a) < prio(b); });
    const int scorer = order.front()->scorer;      // one kernel instantiation per slice
    int n_items = 0;
    double budget = slice_pairs;
    s->n_last = 0;
    s->carried.clear();
    for (Request *r : order) {
        if (budget <= 0.0 || n_items >= kMaxSliceItems) break;
        if (r->scorer != scorer) continue;
        const double per_tile_target = std::max(1.0, slice_pairs / (4.0 * grid));
        const int32_t tile =
            (int32_t)std::max(1.0, std::min((double)r->k, per_tile_target / r->pair_cost));
        if (trace && r->next_k < r->k && budget > 0.0 && n_items < kMaxSliceItems)
            s->carried.push_back(r->id);
        while (r->next_k < r->k && budget > 0.0 && n_items < kMaxSliceItems) {
            const int32_t k0 = r->next_k, k1 = std::min(r->k, k0 + tile);
            s->h_items[n_items++] = BatchItem{r->slot, k0, k1, 0};
            r->next_k = k1;
            budget -= (k1 - k0) * r->pair_cost;
        }
        if (r->next_k == r->k) ++s->n_last;
    }
    s->h_header[0] = n_items;
    s->h_header[1] = 0;
    s->pairs = slice_pairs - budget;
    s->t_launch = Clock::now();
    mu.unlock();
    bool ok = true;
    auto chk = [&](hipError_t e) { if (e != hipSuccess) { ok = false; fatal = hipGetErrorString(e); } };
    // slices alternate between two streams so one slice's tail overlaps the next;
    // the kernel reads the work list from host memory, so a launch is the only
    // device work a slice enqueues
    hipStream_t st = (n_slices & 1) ? stream2 : stream;
    roctxMarkA("dses.slice_launch");
    BatchArgs ba{d_args, s->dv_items, s->dv_header, s->d_cursor, s->d_scratch,
                 slot_words(kServeMaxSrc), s->cursor, d_done, dv_res, dv_flag};
    chk(launch_sweep_batch(ba, scorer, grid, st));
    chk(hipEventRecord(s->swept, st));
    s->cursor += (uint32_t)(n_items + grid);   // every workgroup fetches once past the end
    ++n_slices;
    mu.lock();
    s->stream = st;
    s->busy = true;
    return ok;
}

// A request whose result the kernel has published (scheduler thread, mu held).
// Top-k passes and copies to the caller's buffers are enqueued on `down` and
// polled (they may wait for a sweep workgroup to free a CU); returns true once
// the request is complete, its memory and slot returned.
bool ServerImpl::finish(Request *r)
{
    const DevResult &d = h_res[r->slot];
    if (!r->copying && (r->host_rec || (r->top_k > 0 && d.rot_index >= 0))) {
        bool ok = true;
        auto chk = [&](hipError_t e) { if (e != hipSuccess) ok = false; };
        if (r->top_k > 0 && d.rot_index >= 0) {
            chk(launch_topk(r->d_rec, r->k, r->top_k, r->p.delta, r->d_topk_a, r->d_topk_b,
                            r->d_topk, down));
            chk(hipMemcpyAsync(r->host_topk, r->d_topk, sizeof(dses_candidate) * r->top_k,
                               hipMemcpyDeviceToHost, down));
        }
        if (r->host_rec)
            chk(hipMemcpyAsync(r->host_rec, r->d_rec, sizeof(dses_record) * r->k,
                               hipMemcpyDeviceToHost, down));
        chk(hipEventRecord(slot_event[r->slot], down));
        r->copying = true;
        if (!ok) {
            (void)hipGetLastError();
            fatal = "enqueueing the copies of a finished request failed";
            return false;
        }
    }
    if (r->copying) {
        const hipError_t e = hipEventQuery(slot_event[r->slot]);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fatal = hipGetErrorString(e);
            return false;
        }
    }
    if (d.rot_index < 0) {
        r->status = DSES_E_NOCANDIDATE;
    } else {
        std::memcpy(r->out.R, d.R, sizeof(r->out.R));
        std::memcpy(r->out.t, d.t, sizeof(r->out.t));
        r->out.rot_index = d.rot_index;
        r->out.inliers = d.inliers;
        r->out.error = d.error;
        r->out.votes = d.votes;
        r->out.n_valid = d.n_valid;
    }
    r->state = Request::DONE;
    r->t_done = Clock::now();
    roctxMarkA("dses.request_done");
    if (trace)
        std::fprintf(trace, "R %llu %d %d %d %.6f %.6f %.6f\n", (unsigned long long)r->id, r->n,
                     r->m, r->k, since(r->t_submit), since(r->t_admit), since(r->t_done));
    pool.release(r->off, r->bytes);
    free_slots.push_back(r->slot);
    r->src.clear();
    r->src.shrink_to_fit();
    return true;
}

void ServerImpl::poll_slices()
{
    // admission uploads: one event, recorded after each admission's, covers all
    if (!uploading.empty() && hipEventQuery(up_done) == hipSuccess) {
        for (Request *r : uploading) r->ready = true;
        uploading.clear();
    }
    // requests with every tile handed out whose result flag is up
    bool any = false;
    for (size_t i = 0; i < active.size();) {
        Request *r = active[i];
        if (r->next_k < r->k || __atomic_load_n(h_flag + r->slot, __ATOMIC_ACQUIRE) == 0u) {
            ++i;
            continue;
        }
        if (!finish(r)) {
            ++i;
            continue;
        }
        active.erase(active.begin() + (long)i);
        any = true;
    }
    // slices whose sweep is complete free their work-list buffers
    for (auto &s : sets) {
        if (!s.busy || hipEventQuery(s.swept) != hipSuccess) continue;
        const auto now = Clock::now();
        if (trace) {
            std::fprintf(trace, "S %d %.6f %.6f %.0f %d", s.stream == stream2 ? 1 : 0,
                         since(s.t_launch), since(now), s.pairs, s.n_last);
            for (uint64_t id : s.carried) std::fprintf(trace, " %llu", (unsigned long long)id);
            std::fprintf(trace, "\n");
        }
        const double dt = std::chrono::duration<double>(now - s.t_launch).count();
        if (dt > 1e-4 && s.pairs > 0.0)
            rate = 0.8 * rate + 0.2 * std::min(4.0e12, std::max(1.0e10, s.pairs / dt));
        s.busy = false;
        any = true;
    }
    if (any) cv_done.notify_all();
}

void ServerImpl::run()
{
    roctxNameOsThread("dses.scheduler");
    (void)hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        poll_slices();
        admit_locked();
        bool launched = false;
        int busy = 0;
        for (auto &s : sets) busy += s.busy ? 1 : 0;
        if (busy < kSliceSets - 1) launched = launch_slice();
        if (!fatal.empty()) {
            // a HIP failure poisons the server: fail everything still pending
            for (auto &kv : all)
                if (kv.second->state != Request::DONE) {
                    kv.second->status = DSES_E_DEVICE;
                    kv.second->state = Request::DONE;
                }
            queue.clear();
            active.clear();
            uploading.clear();
            cv_done.notify_all();
            if (stop) break;
            cv_work.wait_for(lk, std::chrono::milliseconds(50));
            continue;
        }
        busy = 0;
        for (auto &s : sets) busy += s.busy ? 1 : 0;
        if (stop && queue.empty() && active.empty() && busy == 0) break;
        if (!launched) {
            if (busy > 0 || !uploading.empty() || !active.empty())
                cv_work.wait_for(lk, std::chrono::microseconds(100));
            else
                cv_work.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
}

}  // namespace dses

struct dses_server {
    dses::ServerImpl impl;
};

using namespace dses;

extern "C" {

dses_status dses_server_create(const dses_server_opts *opt, dses_server **out)
{
    set_error("");
    if (!out) {
        set_error("NULL output handle");
        return DSES_E_INVAL;
    }
    dses_server_opts o{};
    if (opt) o = *opt;
    if (o.memory_budget < 0 || o.max_inflight < 0 || o.max_inflight > 4096 ||
        o.scorer < DSES_SCORER_AUTO || o.scorer > DSES_SCORER_DF || o.slice_mpairs < 0) {
        set_error("invalid server options");
        return DSES_E_INVAL;
    }
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    auto *s = new dses_server();
    dses_status st = s->impl.init(c, o);
    if (st != DSES_OK) {
        delete s;
        return st;
    }
    *out = s;
    return DSES_OK;
}

dses_status dses_server_submit(dses_server *srv, const dses_target *tgt, const dses_rotset *rots,
                               const float *src, int64_t n, float eps, dses_metric metric,
                               const dses_options *opt, uint64_t *req_id)
{
    set_error("");
    if (!srv || !tgt || !rots || !src || !req_id || n <= 0 || n > kServeMaxSrc ||
        n * (int64_t)tgt->res.m >= ((int64_t)1 << 31)) {
        set_error("invalid request");
        return DSES_E_INVAL;
    }
    dses_options o;
    if (copy_options(opt, &o) != DSES_OK) return DSES_E_INVAL;
    if (o.flags != 0 || o.stream || o.q != 0.0f || o.p != 0.0f || o.lane_group != 0 ||
        o.top_k < 0 || o.top_k > DSES_TOPK_MAX || (o.top_k > 0 && !o.topk)) {
        set_error("served requests take delta_t, tau, the box, scorer, df_lookup, records "
                  "and top_k (with a topk buffer) only");
        return DSES_E_INVAL;
    }
    ServerImpl &S = srv->impl;
    auto *r = new Request();
    dses_status st = resolve_params(eps, metric, o.delta_t, o.tau, o.t_min, o.t_max,
                                    o.scorer ? o.scorer : S.opt.scorer, &r->p);
    if (st == DSES_OK) st = apply_metric_options(o, &r->p);
    if (st == DSES_OK && (metric == DSES_TRUNC_LP || metric == DSES_VOTES)) {
        set_error("DSES_TRUNC_LP and DSES_VOTES are plain-path metrics");
        st = DSES_E_INVAL;
    }
    if (st == DSES_OK && !(tgt->res.max_abs <= ref_coord_limit(r->p))) {
        set_error("reference coordinate too large for the lattice of this delta and box");
        st = DSES_E_INVAL;
    }
    if (st != DSES_OK) {
        delete r;
        return st;
    }
    for (int64_t e = 0; e < 3 * n; ++e)
        if (!(std::fabs(src[e]) <= kSrcCoordLimit)) {
            delete r;
            set_error("source coordinate is non-finite or too large for the lattice");
            return DSES_E_INVAL;
        }
    r->target = &tgt->res;
    r->rots = &rots->res;
    r->n = (int32_t)n;
    r->m = tgt->res.m;
    r->k = (int32_t)rots->res.k;
    r->host_rec = static_cast<dses_record *>(o.records);
    r->host_topk = static_cast<dses_candidate *>(o.topk);
    r->top_k = o.top_k;
    r->scorer = r->p.scorer;
    if (r->scorer == DSES_SCORER_AUTO)
        r->scorer = (tgt->res.df && tgt->res.df_r == r->p.r && metric != DSES_TRUNC_L1)
                        ? DSES_SCORER_DF
                        : DSES_SCORER_GRID;
    if (r->scorer == DSES_SCORER_DF &&
        (!tgt->res.df || tgt->res.df_r != r->p.r || metric == DSES_TRUNC_L1)) {
        delete r;
        set_error("DF scorer needs a target field truncated at max(eps, tau)");
        return DSES_E_INVAL;
    }
    r->src.assign(src, src + 3 * n);
    r->pair_cost = (double)r->n * r->m + 1.0;
    r->bytes = S.need_bytes(*r);
    if (r->bytes > (size_t)S.opt.memory_budget) {
        delete r;
        set_error("request needs more device memory than the whole serving budget");
        return DSES_E_NOMEM;
    }
    {
        std::lock_guard<std::mutex> lk(S.mu);
        if (!S.fatal.empty()) {
            delete r;
            set_error("server failed: " + S.fatal);
            return DSES_E_DEVICE;
        }
        r->id = S.next_id++;
        r->t_submit = Clock::now();
        S.all[r->id] = r;
        S.queue.push_back(r);
        *req_id = r->id;
    }
    S.cv_work.notify_all();
    return DSES_OK;
}

dses_status dses_server_wait(dses_server *srv, uint64_t req_id, int32_t timeout_ms,
                             dses_result *out, dses_status *req_status, double *queue_s,
                             double *total_s)
{
    if (!srv || !out || !req_status) return DSES_E_INVAL;
    ServerImpl &S = srv->impl;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.all.find(req_id);
    if (it == S.all.end()) {
        set_error("unknown or already consumed request id");
        return DSES_E_STATE;
    }
    // the request is looked up afresh at every wake-up: another thread's wait may
    // consume (and free) it meanwhile
    auto done = [&] {
        auto f = S.all.find(req_id);
        return f == S.all.end() || f->second->state == Request::DONE;
    };
    if (timeout_ms < 0)
        S.cv_done.wait(lk, done);
    else if (!S.cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
        set_error("request not finished within the timeout");
        return DSES_E_TIMEOUT;
    }
    it = S.all.find(req_id);
    if (it == S.all.end()) {
        set_error("request consumed by another wait");
        return DSES_E_STATE;
    }
    Request *r = it->second;
    *out = r->out;
    *req_status = r->status;
    if (queue_s) *queue_s = std::chrono::duration<double>(r->t_admit - r->t_submit).count();
    if (total_s) *total_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    S.all.erase(it);
    delete r;
    return DSES_OK;
}

dses_status dses_server_cancel(dses_server *srv, uint64_t req_id)
{
    if (!srv) return DSES_E_INVAL;
    ServerImpl &S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(req_id);
    if (it == S.all.end() || it->second->state != Request::QUEUED) {
        set_error("request unknown, consumed, already on the device or finished");
        return DSES_E_STATE;
    }
    Request *r = it->second;
    auto q = std::find(S.queue.begin(), S.queue.end(), r);
    if (q == S.queue.end()) {
        // taken by the scheduler for admission (memory is being prepared)
        set_error("request is being admitted to the device");
        return DSES_E_STATE;
    }
    S.queue.erase(q);
    S.all.erase(it);
    delete r;
    return DSES_OK;
}

int32_t dses_server_poll(dses_server *srv, uint64_t req_id)
{
    if (!srv) return DSES_E_INVAL;
    ServerImpl &S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(req_id);
    if (it == S.all.end()) return DSES_E_STATE;
    return it->second->state == Request::DONE ? 1 : 0;
}

dses_status dses_server_timing(dses_server *srv, uint64_t req_id, double *queue_s,
                               double *total_s)
{
    if (!srv) return DSES_E_INVAL;
    ServerImpl &S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(req_id);
    if (it == S.all.end() || it->second->state != Request::DONE) {
        set_error("request unknown or not finished");
        return DSES_E_STATE;
    }
    Request *r = it->second;
    if (queue_s)
        *queue_s = std::chrono::duration<double>(r->t_admit - r->t_submit).count();
    if (total_s)
        *total_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    return DSES_OK;
}

dses_status dses_server_destroy(dses_server *srv)
{
    if (!srv) return DSES_E_INVAL;
    delete srv;
    return DSES_OK;
}

}  // extern "C"
