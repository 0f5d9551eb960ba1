// Voxel distance field of a reference cloud, built once per resident target.
//
// Value at voxel centre c (float32, c_a = lo_a + (idx_a + 1/2) h_a):
//   D = min(min_j ||c - y_j||, r)
// Only reference points within r matter, and the cell grid (pitch >= r) holds
// all of them in the 27 cells around c's cell, so each voxel visits a handful
// of points instead of all m.  One thread per voxel, z fastest so neighbouring
// lanes share cells (coalesced gathers through L2).
#include <hip/hip_runtime.h>
#include <math.h>

#include "host.h"

namespace dses {

__device__ __forceinline__ int flr_i(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

struct DfArgs {
    const float *pts;        // x y z and a pad per point (16 B), cell order
    const int32_t *start;    // ncell + 1
    float glo[3];
    float ginv;
    int32_t gdim[3];
    int32_t res;
    float lo[3], h[3];
    float r2, r;
    float *out;
};

__global__ void __launch_bounds__(256) k_df_build(DfArgs a)
{
    const int64_t total = (int64_t)a.res * a.res * a.res;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < total;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int iz = (int)(v % a.res);
        const int iy = (int)((v / a.res) % a.res);
        const int ix = (int)(v / ((int64_t)a.res * a.res));
        const float cx = fmaf((float)ix + 0.5f, a.h[0], a.lo[0]);
        const float cy = fmaf((float)iy + 0.5f, a.h[1], a.lo[1]);
        const float cz = fmaf((float)iz + 0.5f, a.h[2], a.lo[2]);
        const int gx = flr_i(__fmul_rn(cx - a.glo[0], a.ginv));
        const int gy = flr_i(__fmul_rn(cy - a.glo[1], a.ginv));
        const int gz = flr_i(__fmul_rn(cz - a.glo[2], a.ginv));
        const float4 *pt = reinterpret_cast<const float4 *>(a.pts);
        float best = a.r2;
        const int zlo = max(gz - 1, 0), zhi = min(gz + 1, a.gdim[2] - 1);
        if (zlo <= zhi)
            for (int x = max(gx - 1, 0); x <= min(gx + 1, a.gdim[0] - 1); ++x)
                for (int y = max(gy - 1, 0); y <= min(gy + 1, a.gdim[1] - 1); ++y) {
                    const int row = (x * a.gdim[1] + y) * a.gdim[2];
                    const int b = a.start[row + zlo], e = a.start[row + zhi + 1];
                    for (int j = b; j < e; ++j) {
                        const float4 y = pt[j];
                        const float dx = cx - y.x, dy = cy - y.y, dz = cz - y.z;
                        best = fminf(best, fmaf(dz, dz, fmaf(dy, dy, __fmul_rn(dx, dx))));
                    }
                }
        a.out[v] = fminf(sqrtf(best), a.r);
    }
}

hipError_t launch_df_build(const float *pts_soa, const int32_t *start, const HostGrid &grid,
                           int32_t res, const float *lo, const float *h, float r, float *out,
                           hipStream_t stream)
{
    DfArgs a{};
    a.pts = pts_soa;
    a.start = start;
    for (int q = 0; q < 3; ++q) {
        a.glo[q] = grid.lo[q];
        a.gdim[q] = grid.dim[q];
        a.lo[q] = lo[q];
        a.h[q] = h[q];
    }
    a.ginv = grid.inv;
    a.res = res;
    a.r = r;
    a.r2 = r * r;
    a.out = out;
    const int64_t total = (int64_t)res * res * res;
    int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_df_build, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace dses
