// dses_register_noalloc: dses_register for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Every device buffer of the call -- the staged reference, the cell
// grid, the per-workgroup source-sort slots, the records, the result and the
// status words -- is carved out of one statically allocated device array of
// kNoAllocScratchBytes per GPU; the call makes no hipMalloc, hipFree or pinned
// host allocation.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host.h"

namespace dses {
namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;   // 64 MiB per GPU
constexpr int kMaxDevices = 64;

// The scratch array.  In host code its name is a host-side stand-in, never a
// device address: kernels and copies only ever see the address that
// hipGetSymbolAddress returns for the current device (scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of this GPU's copy of the scratch array, looked up once
// per device with that device current.
dses_status scratch_ptr(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) {
        set_error("device index out of range for the no-allocation scratch array");
        return DSES_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error(std::string("hipGetSymbolAddress of the scratch array failed: ") +
                      hipGetErrorString(e));
            return DSES_E_DEVICE;
        }
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return DSES_OK;
}

}  // namespace
}  // namespace dses

using namespace dses;

extern "C" {

size_t dses_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

dses_status dses_register_noalloc(const float *src, int64_t n, const float *tgt, int64_t m,
                                  const float *rotations, int64_t k, float eps,
                                  dses_metric metric, const dses_options *opt, dses_result *out)
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
    if ((o.flags & ~(uint32_t)DSES_DEVICE_PTRS) != 0 || !(o.flags & DSES_DEVICE_PTRS)) {
        set_error("dses_register_noalloc takes device pointers (DSES_DEVICE_PTRS) and no "
                  "other flag");
        return DSES_E_INVAL;
    }
    if (o.top_k != 0 || o.q != 0.0f) {
        set_error("dses_register_noalloc takes no top-k and no pruning");
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
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    void *base = nullptr;
    if ((st = scratch_ptr(c->device, &base)) != DSES_OK) return st;
    std::lock_guard<std::mutex> lk(c->mu);
    c->timing_enabled = false;
    hipStream_t stream = o.stream ? static_cast<hipStream_t>(o.stream) : c->stream;
    Job job;
    job.n = (int32_t)n;
    job.m = (int32_t)m;
    job.k = (int32_t)k;
    job.p = p;
    job.src = src;
    job.tgt = tgt;
    job.rot = rotations;
    Arena arena;
    arena.base = static_cast<char *>(base);
    arena.cap = kNoAllocScratchBytes;
    return run_plain(c, job, stream, true, out, o, &arena);
}

}  // extern "C"
