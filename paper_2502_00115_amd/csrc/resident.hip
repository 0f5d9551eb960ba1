// Resident reference clouds (with optional distance field) and rotation lists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "host.h"

namespace dses {

static dses_status copy_to_host(const float *p, size_t count, bool dev, std::vector<float> *out)
{
    out->resize(count);
    if (dev) {
        DSES_HIP(hipMemcpy(out->data(), p, count * sizeof(float), hipMemcpyDeviceToHost));
    } else {
        std::memcpy(out->data(), p, count * sizeof(float));
    }
    return DSES_OK;
}

dses_status ensure_target_grid(TargetRes *tm, float r, CellGrid *cg)
{
    std::lock_guard<std::mutex> gl(tm->grid_mu);
    const TargetRes::Grid *hit = nullptr;
    for (const auto &g : tm->grids)
        if (g.r == r) hit = &g;
    if (!hit) {
        TargetRes::Grid g{r, nullptr, nullptr, HostGrid{}};
        dses_status st = build_grid(tm->host_aos.data(), tm->m, r, &g.meta);
        if (st != DSES_OK) return st;
        if (dev_alloc(&g.pts, g.meta.pts.size() * sizeof(float)) != hipSuccess ||
            dev_alloc(&g.start, g.meta.start.size() * sizeof(int32_t)) != hipSuccess ||
            hipMemcpy(g.pts, g.meta.pts.data(), g.meta.pts.size() * sizeof(float),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g.start, g.meta.start.data(), g.meta.start.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            if (g.pts) (void)hipFree(g.pts);
            if (g.start) (void)hipFree(g.start);
            set_error("cell grid upload failed");
            return DSES_E_NOMEM;
        }
        g.meta.pts.clear();
        g.meta.pts.shrink_to_fit();
        g.meta.start.clear();
        g.meta.start.shrink_to_fit();
        tm->grids.push_back(g);
        hit = &tm->grids.back();
    }
    if (cg) {
        cg->pts = hit->pts;
        cg->start = hit->start;
        for (int q = 0; q < 3; ++q) {
            cg->lo[q] = hit->meta.lo[q];
            cg->dim[q] = hit->meta.dim[q];
        }
        cg->inv = hit->meta.inv;
    }
    return DSES_OK;
}

int64_t target_block_population(TargetRes *tm, const Params &p)
{
    std::lock_guard<std::mutex> gl(tm->grid_mu);
    for (const auto &e : tm->pops)
        if (e.delta == p.delta && std::equal(e.klo, e.klo + 3, p.klo) &&
            std::equal(e.size, e.size + 3, p.size))
            return e.pop;
    TargetRes::Population e{p.delta, {p.klo[0], p.klo[1], p.klo[2]},
                            {p.size[0], p.size[1], p.size[2]},
                            ref_block_population(tm->host_aos.data(), tm->m, p)};
    tm->pops.push_back(e);
    return e.pop;
}

dses_status ensure_target_stage(TargetRes *tm, const Params &p, hipStream_t stream,
                                const TargetRes::Stage **out)
{
    std::lock_guard<std::mutex> gl(tm->grid_mu);
    for (const auto &st : tm->stages)
        if (st.delta == p.delta && st.klo[0] == p.klo[0] && st.klo[1] == p.klo[1] &&
            st.klo[2] == p.klo[2]) {
            *out = &st;
            return DSES_OK;
        }
    const size_t m = (size_t)tm->m;
    if (tm->perm_x.empty()) sort_by_x(tm->host_aos.data(), tm->m, &tm->perm_x);
    if (!tm->d_perm) {
        int32_t *perm = nullptr;
        DSES_HIP(dev_alloc(&perm, 4 * m));
        const hipError_t e = hipMemcpy(perm, tm->perm_x.data(), 4 * m, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(perm);
            DSES_HIP(e);
        }
        tm->d_perm = perm;
    }
    double S16, S15;
    lattice_scales(p.delta, &S16, &S15);
    TargetRes::Stage st{p.delta, {p.klo[0], p.klo[1], p.klo[2]}, nullptr, nullptr, false, 0, 0};
    st.sorted = ref_x_range(tm->host_aos.data(), tm->perm_x, p.delta, p.klo[0], &st.ylo, &st.yhi);
    hipError_t e = dev_alloc(&st.yq, 16 * m);
    if (e == hipSuccess) e = dev_alloc(&st.yt, 12 * m);
    if (e == hipSuccess)
        e = launch_stage(tm->aos, tm->d_perm, tm->m, S16, S15, p.klo, st.yq, st.yt, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        if (st.yq) (void)hipFree(st.yq);
        if (st.yt) (void)hipFree(st.yt);
        DSES_HIP(e);
    }
    tm->stages.push_back(st);
    *out = &tm->stages.back();
    return DSES_OK;
}

}  // namespace dses

using namespace dses;

extern "C" {

dses_status dses_target_create(const float *tgt, int64_t m, const dses_target_opts *opt,
                               dses_target **out)
{
    set_error("");
    TraceRange range("dses.target_create");
    if (!tgt || !out || m <= 0 || m >= ((int64_t)1 << 31)) {
        set_error("invalid reference cloud");
        return DSES_E_INVAL;
    }
    dses_target_opts o{};
    if (opt) o = *opt;
    if (!(o.df_trunc >= 0.0f) || !std::isfinite(o.df_trunc) || o.df_res < 0 || o.df_res > 1024) {
        set_error("invalid distance-field options");
        return DSES_E_INVAL;
    }
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    auto *t = new dses_target();
    TargetRes &T = t->res;
    T.m = (int32_t)m;
    dses_status st = copy_to_host(tgt, 3 * (size_t)m, (o.flags & DSES_DEVICE_PTRS) != 0,
                                  &T.host_aos);
    if (st != DSES_OK) { delete t; return st; }
    for (float v : T.host_aos) {
        if (!std::isfinite(v) || std::fabs(v) > 1e4f) {
            delete t;
            set_error("reference coordinate is non-finite or larger than 1e4");
            return DSES_E_INVAL;
        }
        T.max_abs = std::max(T.max_abs, std::fabs(v));
    }
    auto fail = [&](dses_status s) {
        dses_target_destroy(t);
        return s;
    };
    if (dev_alloc(&T.aos, 3 * (size_t)m * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation failed");
        return fail(DSES_E_NOMEM);
    }
    if (hipMemcpy(T.aos, T.host_aos.data(), 3 * (size_t)m * sizeof(float),
                  hipMemcpyHostToDevice) != hipSuccess) {
        set_error("upload of the reference failed");
        return fail(DSES_E_DEVICE);
    }
    if (o.df_trunc > 0.0f) {
        const int32_t res = o.df_res ? o.df_res : 128;
        const float r = o.df_trunc;
        // field box: reference AABB padded by r (float arithmetic, see dses.h)
        for (int a = 0; a < 3; ++a) {
            float mn = T.host_aos[a], mx = T.host_aos[a];
            for (int64_t j = 1; j < m; ++j) {
                const float v = T.host_aos[3 * j + a];
                if (v < mn) mn = v;
                if (v > mx) mx = v;
            }
            const float l = mn - r, u = mx + r;
            const float ext = u - l;
            T.df_lo[a] = l;
            T.df_h[a] = ext / (float)res;
            T.df_inv[a] = 1.0f / T.df_h[a];
        }
        HostGrid hg;
        if ((st = build_grid(T.host_aos.data(), T.m, r, &hg)) != DSES_OK) return fail(st);
        float *gp = nullptr;
        int32_t *gs = nullptr;
        const size_t nvox = (size_t)res * res * res;
        if (dev_alloc(&gp, hg.pts.size() * sizeof(float)) != hipSuccess ||
            dev_alloc(&gs, hg.start.size() * sizeof(int32_t)) != hipSuccess ||
            dev_alloc(&T.df, nvox * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            if (gp) (void)hipFree(gp);
            if (gs) (void)hipFree(gs);
            set_error("device allocation for the distance field failed");
            return fail(DSES_E_NOMEM);
        }
        hipError_t e = hipMemcpy(gp, hg.pts.data(), hg.pts.size() * sizeof(float),
                                 hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(gs, hg.start.data(), hg.start.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_df_build(gp, gs, hg, res, T.df_lo, T.df_h, r, T.df, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        (void)hipFree(gp);
        (void)hipFree(gs);
        if (e != hipSuccess) {
            set_error(std::string("distance field build failed: ") + hipGetErrorString(e));
            return fail(DSES_E_DEVICE);
        }
        T.df_res = res;
        T.df_r = r;
    }
    *out = t;
    return DSES_OK;
}

dses_status dses_target_destroy(dses_target *t)
{
    if (!t) return DSES_E_INVAL;
    TargetRes &T = t->res;
    for (auto &st : T.stages)
        for (void *q : {(void *)st.yq, (void *)st.yt})
            if (q) (void)hipFree(q);
    for (auto &g : T.grids) {
        if (g.pts) (void)hipFree(g.pts);
        if (g.start) (void)hipFree(g.start);
    }
    if (T.d_perm) (void)hipFree(T.d_perm);
    if (T.aos) (void)hipFree(T.aos);
    if (T.yt) (void)hipFree(T.yt);
    if (T.df) (void)hipFree(T.df);
    delete t;
    return DSES_OK;
}

dses_status dses_target_field(const dses_target *t, float *field, float *lo, float *h)
{
    if (!t) return DSES_E_INVAL;
    const TargetRes &T = t->res;
    if (!T.df) {
        set_error("target has no distance field");
        return DSES_E_STATE;
    }
    if (field) {
        const size_t nvox = (size_t)T.df_res * T.df_res * T.df_res;
        DSES_HIP(hipMemcpy(field, T.df, nvox * sizeof(float), hipMemcpyDeviceToHost));
    }
    if (lo) std::memcpy(lo, T.df_lo, sizeof(T.df_lo));
    if (h) std::memcpy(h, T.df_h, sizeof(T.df_h));
    return DSES_OK;
}

dses_status dses_rotations_create(const float *rotations, int64_t k, uint32_t flags,
                                  dses_rotset **out)
{
    set_error("");
    if (!rotations || !out || k <= 0 || k > INT32_MAX) {
        set_error("invalid rotation list");
        return DSES_E_INVAL;
    }
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    std::vector<float> host;
    dses_status st = copy_to_host(rotations, 9 * (size_t)k, (flags & DSES_DEVICE_PTRS) != 0, &host);
    if (st != DSES_OK) return st;
    for (int64_t q = 0; q < k; ++q) {
        const float *R = host.data() + 9 * q;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                float d = R[i] * R[j] + R[3 + i] * R[3 + j] + R[6 + i] * R[6 + j];
                d -= (i == j) ? 1.0f : 0.0f;
                if (!(std::fabs(d) <= 1e-4f)) {
                    set_error("rotation " + std::to_string(q) + " is not orthonormal");
                    return DSES_E_INVAL;
                }
            }
    }
    auto *r = new dses_rotset();
    r->res.k = k;
    if (dev_alloc(&r->res.rot, 9 * (size_t)k * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        delete r;
        set_error("device allocation failed");
        return DSES_E_NOMEM;
    }
    if (hipMemcpy(r->res.rot, host.data(), 9 * (size_t)k * sizeof(float),
                  hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(r->res.rot);
        delete r;
        set_error("upload of the rotation list failed");
        return DSES_E_DEVICE;
    }
    *out = r;
    return DSES_OK;
}

dses_status dses_rotations_destroy(dses_rotset *r)
{
    if (!r) return DSES_E_INVAL;
    if (r->res.rot) (void)hipFree(r->res.rot);
    delete r;
    return DSES_OK;
}

dses_status dses_register_resident(const dses_target *tgt, const dses_rotset *rots,
                                   const float *src, int64_t n, float eps, dses_metric metric,
                                   const dses_options *opt, dses_result *out)
{
    set_error("");
    if (!tgt || !rots || !src || !out || n <= 0 || n * (int64_t)tgt->res.m >= ((int64_t)1 << 31)) {
        set_error("invalid arguments");
        return DSES_E_INVAL;
    }
    dses_options o;
    if (copy_options(opt, &o) != DSES_OK) return DSES_E_INVAL;
    Params p;
    dses_status st = resolve_params(eps, metric, o.delta_t, o.tau, o.t_min, o.t_max, o.scorer, &p);
    if (st != DSES_OK) return st;
    if ((st = apply_metric_options(o, &p)) != DSES_OK) return st;
    const bool dev = (o.flags & DSES_DEVICE_PTRS) != 0;
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    std::lock_guard<std::mutex> lk(c->mu);
    c->timing_enabled = (o.flags & DSES_TIMING) != 0;
    hipStream_t stream = o.stream ? static_cast<hipStream_t>(o.stream) : c->stream;
    Job job;
    job.n = (int32_t)n;
    job.m = tgt->res.m;
    job.k = (int32_t)rots->res.k;
    job.p = p;
    job.tgt = tgt->res.aos;
    job.rot = rots->res.rot;
    job.target = &tgt->res;
    job.host_tgt = tgt->res.host_aos.data();
    if (!(tgt->res.max_abs <= ref_coord_limit(p))) {
        set_error("reference coordinate too large for the lattice of this delta and box");
        return DSES_E_INVAL;
    }
    if (dev) {
        job.src = src;
    } else {
        for (int64_t e = 0; e < 3 * n; ++e)
            if (!(std::fabs(src[e]) <= kSrcCoordLimit)) {
                set_error("source coordinate is non-finite or too large for the lattice");
                return DSES_E_INVAL;
            }
        if ((st = c->in_src.ensure(3 * n * sizeof(float))) != DSES_OK) return st;
        DSES_HIP(hipMemcpyAsync(c->in_src.ptr, src, 3 * n * sizeof(float), hipMemcpyHostToDevice,
                                stream));
        job.src = static_cast<float *>(c->in_src.ptr);
    }
    return run_plain(c, job, stream, dev, out, o);
}

}  // extern "C"
