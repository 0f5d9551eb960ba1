// DSES device kernels for CDNA4 (gfx950): input staging, the fused per-rotation
// sweep (vote -> mode -> score), candidate selection and top-k.
//
// Sweep design (one workgroup of 16 wave64s per rotation, one workgroup per CU):
//  * Source points are rotated once per rotation, quantised to the fixed-point
//    lattice (2^-16 bins, the lattice offset folded into the reference) and
//    bucket-sorted by x into a per-workgroup scratch slot (an x array, a 64-bit
//    (y, z) array and a bucket table).
//  * In the vote each lane holds two points of the x-sorted reference (a work
//    unit's lane group: 64, 32 or 16 consecutive points, the smaller groups
//    repeated on the wave's lane sub-groups) and streams the sources of the
//    window whose pairs can land in the current slab; the sub-groups take
//    alternate 4-source pieces of it.  Sources arrive through 16-byte buffer
//    loads (one address per sub-group), two blocks in flight.  A pair's bin is
//    exact integer arithmetic: one 64-bit add for the y and z differences, one
//    subtraction for x, the bin being the high 16 bits of each.
//  * The vote array of Alg. 2 lives in LDS, in x-slabs that each fit it, as
//    16-bit counters packed two per 32-bit word (incremented with ds_add_u32 of
//    1 or 1<<16) or as 32-bit counters.  16-bit counters are used only when the
//    host has proven that no bin can reach 2^16 votes (counter_bound in
//    api.hip), and 32-bit ones also when every slab carries at least 2^20 pairs
//    (counter_bits_for), where the cheaper pairs outweigh the extra slabs.
//  * The mode per slab: the largest count by a packed 16-bit max over the slab,
//    then, only when it beats the earlier slabs, its lowest linear index.
//  * Scoring rotates the sources again, in input order; the error sum is a
//    fixed-order tree, so a rotation's record does not depend on what else runs
//    on the GPU.
#include <hip/hip_runtime.h>

#include <utility>
#include <math.h>
#include <stdint.h>

#include "internal.h"

namespace dses {

// floor to int32 in one VALU op (v_cvt_flr_i32_f32: D = (int)floor(S0)).
__device__ __forceinline__ int cvt_flr(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// 24-bit multiply-add (v_mad_u32_u24: D = a[23:0] * b[23:0] + c, 32-bit wrap);
// written as asm so the compiler keeps one instruction instead of mul + add3.
__device__ __forceinline__ uint32_t mad24(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// (a << 2) + b in one instruction (v_lshl_add_u32); b is wave-uniform.
__device__ __forceinline__ uint32_t lshl2_add(uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_lshl_add_u32 %0, %1, 2, %2" : "=v"(r) : "v"(a), "s"(b));
    return r;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// p = R x with the header's FMA chain (float).
__device__ __forceinline__ void rotate(const float *R, float x, float y, float z, float &px,
                                       float &py, float &pz)
{
    px = fmaf(R[2], z, fmaf(R[1], y, __fmul_rn(R[0], x)));
    py = fmaf(R[5], z, fmaf(R[4], y, __fmul_rn(R[3], x)));
    pz = fmaf(R[8], z, fmaf(R[7], y, __fmul_rn(R[6], x)));
}

__device__ __forceinline__ float wave_sum(float v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_isum(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// --------------------------------------------------------------------------
// input checks (device-pointer inputs): finiteness, coordinate range, rotations
// --------------------------------------------------------------------------
__global__ void k_check(CheckArgs a)
{
    const int64_t total = (int64_t)a.n * 3 + (int64_t)a.m * 3 + a.k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        bool bad = false;
        if (e < (int64_t)a.n * 3) {
            float v = a.src[e];
            bad = !(fabsf(v) <= a.src_limit);
        } else if (e < (int64_t)a.n * 3 + (int64_t)a.m * 3) {
            float v = a.tgt[e - (int64_t)a.n * 3];
            bad = !(fabsf(v) <= a.ref_limit);
        } else {
            const float *R = a.rot + 9 * (e - (int64_t)a.n * 3 - (int64_t)a.m * 3);
            float worst = 0.0f;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    float d = R[i] * R[j] + R[3 + i] * R[3 + j] + R[6 + i] * R[6 + j];
                    d -= (i == j) ? 1.0f : 0.0f;
                    worst = fmaxf(worst, fabsf(d));
                }
            bad = !(worst <= 1e-4f);
        }
        if (bad) atomicOr(a.bad, 1u);
    }
}

hipError_t launch_check(const CheckArgs &a, hipStream_t stream)
{
    const int64_t total = (int64_t)a.n * 3 + (int64_t)a.m * 3 + a.k;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_check, dim3(blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Fixed-point lattice coordinates.  A coordinate v (a reference coordinate, or a
// rotated source coordinate) becomes an integer in units of 2^-F bins:
//     q(v) = rint(v * S_F [+ (1/2 - k_lo) 2^F])     S_F = (1/delta) 2^F,
// every product and sum a separately rounded double operation (the products of
// two floats are exact in double), rint rounding halves to even.  The pair
// difference D = Y - P of a reference value Y and a source value P is then exact
// integer arithmetic, and floor(D / 2^F) is the box-relative bin of Alg. 2's
// ROUND up to the two roundings of q, at most 2^-F bins together: F = 16 on x and
// y, and on z 15 with 16-bit counters (the two counters of a word are z
// neighbours, so D >> 16 is the word and bit 15 the half), 16 with 32-bit ones.
// --------------------------------------------------------------------------
__device__ __forceinline__ int32_t quant(double v) { return __double2int_rn(v); }

// A rotated source value saturates at +-2^30 units (2^14 bins): every reference
// value is below 2^29 units and a voting difference below 2^28, so no pair with a
// source value beyond 2^30 can vote, before or after the saturation.
__device__ __forceinline__ int32_t quant_src(double v)
{
    return quant(fmin(fmax(v, -1073741824.0), 1073741824.0));
}

__device__ __forceinline__ int32_t quant_ref(float y, double S, double ofs)
{
    return quant(__dadd_rn(__dmul_rn((double)y, S), ofs));
}

// p_a = (R_a0 x + R_a1 y) + R_a2 z in double, then q(p_a) with S16 on x and y and
// Sz (S15 or S16) on z, saturated.
__device__ __forceinline__ void rotate_quant(const float *R, float x, float y, float z, double S16,
                                             double Sz, int32_t &Px, int32_t &Py, int32_t &Pz)
{
    const double dx = (double)x, dy = (double)y, dz = (double)z;
    const double p0 = __dadd_rn(__dadd_rn(__dmul_rn((double)R[0], dx), __dmul_rn((double)R[1], dy)),
                                __dmul_rn((double)R[2], dz));
    const double p1 = __dadd_rn(__dadd_rn(__dmul_rn((double)R[3], dx), __dmul_rn((double)R[4], dy)),
                                __dmul_rn((double)R[5], dz));
    const double p2 = __dadd_rn(__dadd_rn(__dmul_rn((double)R[6], dx), __dmul_rn((double)R[7], dy)),
                                __dmul_rn((double)R[8], dz));
    Px = quant_src(__dmul_rn(p0, S16));
    Py = quant_src(__dmul_rn(p1, S16));
    Pz = quant_src(__dmul_rn(p2, Sz));
}

// --------------------------------------------------------------------------
// staging: reference AoS -> SoA float (scoring) and the fixed-point copy used
// for binning, four arrays of m: x, y, z at 2^-16 bins and z at 2^-15 bins,
//   Y_a = q(y_a) with the offset (1/2 - k_lo_a) 2^F folded in.
// --------------------------------------------------------------------------
__device__ __forceinline__ void stage_point(const float *tgt, int src, int j, int32_t m,
                                            double S16, double S15, const int32_t *klo,
                                            int32_t *yq, float *yt)
{
    for (int a = 0; a < 3; ++a) {
        const float y = tgt[3 * src + a];
        yq[a * m + j] = quant_ref(y, S16, (0.5 - (double)klo[a]) * 65536.0);
        yt[a * m + j] = y;
    }
    yq[3 * m + j] = quant_ref(tgt[3 * src + 2], S15, (0.5 - (double)klo[2]) * 32768.0);
}

__global__ void k_stage(const float *tgt, const int32_t *perm, int32_t m, double S16, double S15,
                        int32_t klo0, int32_t klo1, int32_t klo2, int32_t *yq, float *yt)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int32_t klo[3] = {klo0, klo1, klo2};
    stage_point(tgt, perm ? perm[j] : j, j, m, S16, S15, klo, yq, yt);
}

hipError_t launch_stage(const float *tgt, const int32_t *perm, int32_t m, double S16, double S15,
                        const int32_t *klo, int32_t *yq, float *yt, hipStream_t stream)
{
    hipLaunchKernelGGL(k_stage, dim3((m + 255) / 256), dim3(256), 0, stream, tgt, perm, m, S16,
                       S15, klo[0], klo[1], klo[2], yq, yt);
    return hipGetLastError();
}

__global__ void k_clear(uint32_t *p, int32_t words)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_clear(uint32_t *p, int32_t words, hipStream_t stream)
{
    int blocks = (words + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_clear, dim3(blocks), dim3(256), 0, stream, p, words);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// the fused sweep
// --------------------------------------------------------------------------

// Read-only inputs are read through the constant address space so that
// wave-uniform indices compile to scalar loads (s_load) into SGPRs.
typedef const float __attribute__((address_space(4))) *kfloat;
typedef const int32_t __attribute__((address_space(4))) *kint;
__device__ __forceinline__ kfloat kc(const float *p) { return (kfloat)p; }
__device__ __forceinline__ kint kc(const int32_t *p) { return (kint)p; }

// Copy a wave-uniform struct from device memory through the constant address
// space (scalar loads into SGPRs).
template <class T>
__device__ __forceinline__ T kload(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized structs only");
    T v;
    const kint src = kc(reinterpret_cast<const int32_t *>(p));
    int32_t *dst = reinterpret_cast<int32_t *>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return v;
}

// Lane layout for a chunk of up to 1024 source points: `sw` waves hold the chunk
// (one point per lane) and the reference is split into G partitions, one per
// group of sw waves, when the chunk is small.
struct ChunkLayout {
    int sw, G, part, i;
    bool active;
};

__device__ __forceinline__ ChunkLayout chunk_layout(int c0, int n, int wave, int lane)
{
    ChunkLayout L;
    const int nc = min(kBlock, n - c0);
    L.sw = (nc + 63) >> 6;
    L.G = max(1, kWaves / L.sw);
    L.part = wave / L.sw;
    L.active = L.part < L.G;
    L.i = c0 + (wave % L.sw) * 64 + lane;
    return L;
}

// One pair's vote from its fixed-point differences D_a = Y_a - P_a (x with the
// slab's first plane folded into Y, so every range starts at 0).  The pair votes
// iff D_x < np 2^16, D_y < S_y 2^16 and D_z < S_z 2^Fz as unsigned numbers (a
// negative difference is a huge one); then its counter is at LDS byte address
//     base + (D_x >> 16) sx4 + (D_y >> 16) sy4 + (D_z >> 16) 4
// (16-bit counters: D_z >> 16 is the z bin halved, bit 15 its half, so the
// increment is 1 or 1 << 16; 32-bit counters: D_z >> 16 is the z bin).  The
// upper halves of the differences feed v_mad_u32_u16 directly through op_sel, so
// the address costs three multiply-adds and no extraction; WIDE (x stride in
// bytes above 16 bits) multiplies word strides and scales the sum by 4 at the end.
// Without XT the x test is left out: the caller has proven 0 <= D_x < np 2^16
// for every lane (the interior of a window).
// Each variant is one asm block: the v_cmpx narrow EXEC to the voting lanes,
// the address arithmetic and the ds_add_u32 run on those lanes only, and EXEC is
// restored -- no branch, no VALU -> SALU round trip per pair.
struct VoteConst {
    uint32_t npx, syx, szx;    // range limits: np << 16, S_y << 16, S_z << Fz
    uint32_t sx, sy;           // x and y strides: bytes (sx4, sy4), or words when WIDE
    uint32_t base;             // LDS byte address of the slab's first counter
};

#define DSES_VP_X "v_cmpx_gt_u32 vcc, %[npx], %[dx]\n\t"
#define DSES_VP_YZ                                                                           \
    "v_cmpx_gt_u32 vcc, %[syx], %[dy]\n\t"                                                   \
    "v_cmpx_gt_u32 vcc, %[szx], %[dz]\n\t"
#define DSES_VP_ADDR_BYTES                                                                   \
    "v_mad_u32_u16 %[t1], %[dz], 4, %[base] op_sel:[1,0,0,0]\n\t"                             \
    "v_mad_u32_u16 %[t1], %[dy], %[sy], %[t1] op_sel:[1,0,0,0]\n\t"                           \
    "v_mad_u32_u16 %[t1], %[dx], %[sx], %[t1] op_sel:[1,0,0,0]\n\t"
#define DSES_VP_ADDR_WORDS                                                                   \
    "v_lshrrev_b32 %[t1], 16, %[dz]\n\t"                                                     \
    "v_mad_u32_u16 %[t1], %[dy], %[sy], %[t1] op_sel:[1,0,0,0]\n\t"                           \
    "v_mad_u32_u16 %[t1], %[dx], %[sx], %[t1] op_sel:[1,0,0,0]\n\t"                           \
    "v_lshl_add_u32 %[t1], %[t1], 2, %[base]\n\t"
#define DSES_VP_HALF                                                                         \
    "v_bfe_u32 %[t2], %[dz], 15, 1\n\t"                                                      \
    "v_mad_u32_u24 %[t2], %[t2], %[ffff], 1\n\t"
// 16-bit counters: the increment t2 is computed in the block; 32-bit: it is 1
#define DSES_VP_OPERANDS                                                                     \
    [dx] "v"(dx), [dy] "v"(dy), [dz] "v"(dz), [npx] "s"(v.npx), [syx] "s"(v.syx),            \
        [szx] "s"(v.szx), [sx] "s"(v.sx), [sy] "s"(v.sy), [base] "s"(v.base)
#define DSES_VP_ASM16(TEXT)                                                                  \
    asm volatile("s_mov_b64 %[save], exec\n\t" TEXT "ds_add_u32 %[t1], %[t2]\n\t"            \
                 "s_mov_b64 exec, %[save]"                                                   \
                 : [save] "=&s"(save), [t1] "=&v"(t1), [t2] "=&v"(t2)                          \
                 : DSES_VP_OPERANDS, [ffff] "s"(0xFFFFu)                                      \
                 : "vcc", "memory")
#define DSES_VP_ASM32(TEXT)                                                                  \
    asm volatile("s_mov_b64 %[save], exec\n\t" TEXT "ds_add_u32 %[t1], %[t2]\n\t"            \
                 "s_mov_b64 exec, %[save]"                                                   \
                 : [save] "=&s"(save), [t1] "=&v"(t1)                                         \
                 : DSES_VP_OPERANDS, [t2] "v"(1u)                                            \
                 : "vcc", "memory")

template <int CW, bool WIDE, bool XT = true>
__device__ __forceinline__ void vote_pair(uint32_t dx, uint32_t dy, uint32_t dz, const VoteConst &v)
{
    uint64_t save;
    uint32_t t1, t2;
    if (CW == 16) {
        if (XT && !WIDE) DSES_VP_ASM16(DSES_VP_X DSES_VP_YZ DSES_VP_ADDR_BYTES DSES_VP_HALF);
        if (XT && WIDE) DSES_VP_ASM16(DSES_VP_X DSES_VP_YZ DSES_VP_ADDR_WORDS DSES_VP_HALF);
        if (!XT && !WIDE) DSES_VP_ASM16(DSES_VP_YZ DSES_VP_ADDR_BYTES DSES_VP_HALF);
        if (!XT && WIDE) DSES_VP_ASM16(DSES_VP_YZ DSES_VP_ADDR_WORDS DSES_VP_HALF);
    } else {
        if (XT && !WIDE) DSES_VP_ASM32(DSES_VP_X DSES_VP_YZ DSES_VP_ADDR_BYTES);
        if (XT && WIDE) DSES_VP_ASM32(DSES_VP_X DSES_VP_YZ DSES_VP_ADDR_WORDS);
        if (!XT && !WIDE) DSES_VP_ASM32(DSES_VP_YZ DSES_VP_ADDR_BYTES);
        if (!XT && WIDE) DSES_VP_ASM32(DSES_VP_YZ DSES_VP_ADDR_WORDS);
        (void)t2;
    }
}
#undef DSES_VP_ASM32
#undef DSES_VP_ASM16
#undef DSES_VP_OPERANDS
#undef DSES_VP_HALF
#undef DSES_VP_ADDR_WORDS
#undef DSES_VP_ADDR_BYTES
#undef DSES_VP_YZ
#undef DSES_VP_X

typedef uint32_t f4u __attribute__((ext_vector_type(4)));

// Buffer resource over `bytes` bytes from `base`.  The hardware range check covers
// the per-lane (VGPR) offset only; the stream loads below address by scalar offset
// and stay inside their arrays by construction.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, int64_t bytes)
{
    // word 3: 32-bit data format, no swizzle (raw buffer)
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}

// The same descriptor as four scalar words, for the asm loads below.
__device__ __forceinline__ f4u desc_words(const void *base, int64_t bytes)
{
    const uint64_t p = (uint64_t)(uintptr_t)base;
    f4u d;
    d.x = __builtin_amdgcn_readfirstlane((uint32_t)p);
    d.y = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    d.z = (uint32_t)bytes;
    d.w = 0x00020000u;
    return d;
}

// Byte offsets of the x, y and z arrays of a point set held as int32 arrays of
// `stride` entries (z is array zsel: 2, or 3 for the reference's 2^-15 z).
struct SoaOffs {
    int o0, o1, o2;
};
__device__ __forceinline__ SoaOffs soa_offs(int stride, int zsel)
{
    return SoaOffs{0, 4 * stride, 4 * zsel * stride};
}

// Points j .. j+3 (x, y, z) of such a set: three 16-byte loads, the same address
// on every lane.  Issued from asm together with soa_wait so that each wait covers
// exactly the group it needs: the compiler's own wait placement at this loop
// depth sometimes drains every load in flight (vmcnt(0)), stalling each group
// for a full memory round trip.  Every group issued here must be waited for
// (soa_wait) before its registers die, or a late load could overwrite registers
// the compiler has reused.
__device__ __forceinline__ void soa_issue4(const f4u &desc, const SoaOffs &so, int j, f4u &x,
                                           f4u &y, f4u &z)
{
    const int o0 = so.o0 + 4 * j, o1 = so.o1 + 4 * j, o2 = so.o2 + 4 * j;
    asm volatile("buffer_load_dwordx4 %0, off, %3, %4\n\t"
                 "buffer_load_dwordx4 %1, off, %3, %5\n\t"
                 "buffer_load_dwordx4 %2, off, %3, %6"
                 : "=&v"(x), "=&v"(y), "=&v"(z)
                 : "s"(desc), "s"(o0), "s"(o1), "s"(o2));
}

// Sources j + 4h .. j + 4h + 3 of a sorted-source slot (x array of ns int32 at
// byte 0, then the 64-bit yz array at byte 4 ns), h = hoff / 16 per lane: x
// through hoff, the yz pairs of sources 4h, 4h + 1 and 4h + 2, 4h + 3 through
// 2 hoff.
__device__ __forceinline__ void src_issue_lanes(const f4u &desc, int ns, int j, uint32_t hoff,
                                                uint32_t hoff2, f4u &x, f4u &yz01, f4u &yz23)
{
    const int o0 = 4 * j, o1 = 4 * ns + 8 * j, o2 = o1 + 16;
    asm volatile("buffer_load_dwordx4 %0, %3, %5, %6 offen\n\t"
                 "buffer_load_dwordx4 %1, %4, %5, %7 offen\n\t"
                 "buffer_load_dwordx4 %2, %4, %5, %8 offen"
                 : "=&v"(x), "=&v"(yz01), "=&v"(yz23)
                 : "v"(hoff), "v"(hoff2), "s"(desc), "s"(o0), "s"(o1), "s"(o2));
}

// Wait until all but the newest N vector-memory operations are complete; the
// group's registers pass through the asm so no use can be scheduled before it.
template <int N>
__device__ __forceinline__ void soa_wait(f4u &x, f4u &y, f4u &z)
{
    static_assert(N == 0 || N == 3, "soa_wait<0> or soa_wait<3>");
    if (N == 3)
        asm volatile("s_waitcnt vmcnt(3)" : "+v"(x), "+v"(y), "+v"(z));
    else
        asm volatile("s_waitcnt vmcnt(0)" : "+v"(x), "+v"(y), "+v"(z));
}

// One int32 of such a set at byte offset `off` (+ the per-lane offset vo).
__device__ __forceinline__ uint32_t load1(__amdgpu_buffer_rsrc_t rs, uint32_t vo, int off)
{
    return __builtin_amdgcn_raw_buffer_load_b32(rs, vo, off, 0);
}

// Votes of one lane point (Lx, Ly, Lz) against four streamed points (x, y, z).
// LREF: the lane holds a reference point Y and the stream source points P, else
// the reverse; either way D = Y - P per axis.
template <int CW, bool WIDE, bool LREF, bool XT = true>
__device__ __forceinline__ void vote4(f4u x, f4u y, f4u z, uint32_t Lx, uint32_t Ly, uint32_t Lz,
                                      const VoteConst &v)
{
    uint32_t dx[4], dy[4], dz[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        dx[q] = LREF ? Lx - x[q] : x[q] - Lx;
        dy[q] = LREF ? Ly - y[q] : y[q] - Ly;
        dz[q] = LREF ? Lz - z[q] : z[q] - Lz;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) vote_pair<CW, WIDE, XT>(dx[q], dy[q], dz[q], v);
}

// Votes of the lane source point P against the streamed reference points
// [j0, j1): groups of 4 points with two groups in flight, then single points.
// The streamed coordinates come through the vector memory path (buffer loads):
// scalar loads would share the LDS counter, and waiting for them would also wait
// for every outstanding ds_add of the wave.
template <int CW, bool WIDE>
__device__ __forceinline__ void vote_span(const f4u &desc, __amdgpu_buffer_rsrc_t rs,
                                          const SoaOffs &so, int j0, int j1, uint32_t Px,
                                          uint32_t Py, uint32_t Pz, const VoteConst &v)
{
    int j = j0;
    if (j + 4 <= j1) {
        f4u ax, ay, az, bx, by, bz;
        soa_issue4(desc, so, j, ax, ay, az);
        for (; j + 8 <= j1; j += 8) {
            soa_issue4(desc, so, j + 4, bx, by, bz);
            soa_wait<3>(ax, ay, az);
            vote4<CW, WIDE, false>(ax, ay, az, Px, Py, Pz, v);
            soa_issue4(desc, so, min(j + 8, j1 - 4), ax, ay, az);
            soa_wait<3>(bx, by, bz);
            vote4<CW, WIDE, false>(bx, by, bz, Px, Py, Pz, v);
        }
        soa_wait<0>(ax, ay, az);          // the last group issued, used or not
        if (j + 4 <= j1) {
            vote4<CW, WIDE, false>(ax, ay, az, Px, Py, Pz, v);
            j += 4;
        }
    }
    for (; j < j1; ++j) {
        const uint32_t yx = load1(rs, 0, so.o0 + 4 * j), yy = load1(rs, 0, so.o1 + 4 * j);
        const uint32_t yz = load1(rs, 0, so.o2 + 4 * j);
        vote_pair<CW, WIDE>(yx - Px, yy - Py, yz - Pz, v);
    }
}

// Values that never vote: a padding source (every coordinate INT32_MIN) or a
// padding lane point (INT32_MAX): with every real coordinate below 2^29 in
// magnitude, each difference they take part in lies at 2^30 or more from the
// range [0, 2^28) of a voting one, also with each other (-1).
constexpr uint32_t kPadSrc = 0x80000000u;
constexpr uint32_t kPadRef = 0x7FFFFFFFu;

// A lane's two reference points (vote_slab's sorted layout): x, and y and z as
// one 64-bit value (y << 32) | (z + 2^31).
struct LanePts {
    uint32_t x0, x1;
    uint64_t yz0, yz1;
};

// The sorted sources keep x, and -((y << 32) | (z + 2^31)) as one 64-bit value, so
// one 64-bit add gives both differences of a pair: the low word is
// D_z = z_ref - z_src (mod 2^32) and the high word y_ref - y_src - [D_z < 0]
// (the bias 2^31 makes the unsigned borrow that of the signed difference).  A
// pair with D_z < 0 fails the z test, so every pair that votes has its exact D_y.
__device__ __forceinline__ uint64_t yz_pack(uint32_t y, uint32_t z)
{
    return ((uint64_t)y << 32) | (uint64_t)(z + 0x80000000u);
}

__device__ __forceinline__ uint64_t add64(uint64_t a, uint64_t b)
{
    uint64_t r;
    asm("v_lshl_add_u64 %0, %1, 0, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Votes of a lane's two reference points against four streamed sources: each
// 48 bytes a lane loads serve eight pairs (the vector-memory return path, 64
// bytes per clock per CU, bounded the vote at one point per lane).
template <int CW, bool WIDE, bool XT>
__device__ __forceinline__ void vote8(f4u x, f4u yz01, f4u yz23, const LanePts &L,
                                      const VoteConst &v)
{
    typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
    const u64x2 n01 = __builtin_bit_cast(u64x2, yz01), n23 = __builtin_bit_cast(u64x2, yz23);
    uint32_t dx0[4], dx1[4];
    uint64_t e0[4], e1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint64_t nq = q < 2 ? n01[q] : n23[q - 2];
        dx0[q] = L.x0 - x[q];
        dx1[q] = L.x1 - x[q];
        e0[q] = add64(L.yz0, nq);
        e1[q] = add64(L.yz1, nq);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        vote_pair<CW, WIDE, XT>(dx0[q], (uint32_t)(e0[q] >> 32), (uint32_t)e0[q], v);
        vote_pair<CW, WIDE, XT>(dx1[q], (uint32_t)(e1[q] >> 32), (uint32_t)e1[q], v);
    }
}

// Votes of the lane's reference points against the streamed sources [j0, j1),
// j1 - j0 a multiple of 4: in each whole block of B = 4 * 64 / (lanes per copy of
// the group) points, lane sub-group h (its hoff = 16 h bytes) takes points
// 4h .. 4h + 3; the r < B points after the last whole block go in r / S steps
// (S = B / 4 sub-groups), sub-group h taking point S q + h in step q (every index
// stays below j1).  A whole block inside [i0, i1) (the window's interior) is voted
// without the x test; the choice is a uniform branch per block, so the loads stay
// one pipeline, two blocks in flight, across the whole range.
template <int CW, bool WIDE>
__device__ __forceinline__ void vote_span_lanes(const f4u &desc, __amdgpu_buffer_rsrc_t rs, int ns,
                                                int j0, int j1, int i0, int i1, int B,
                                                uint32_t hoff, const LanePts &L,
                                                const VoteConst &v)
{
    const int jb = B > 4 ? j0 + (j1 - j0) / B * B : j1;   // B == 4: no tail
    const uint32_t hoff2 = 2u * hoff;
    for (int t = jb; t < j1; t += B >> 2) {
        // with 8 sub-groups the last step may reach 4 points past j1: those lanes
        // take padding (their loads stay inside the slot's arrays)
        const uint32_t vo = 4u * (uint32_t)(t - jb) + (hoff >> 2);
        uint32_t px = load1(rs, vo, 4 * jb);
        uint64_t nyz = ((uint64_t)load1(rs, 2u * vo, 4 * ns + 8 * jb + 4) << 32) |
                       (uint64_t)load1(rs, 2u * vo, 4 * ns + 8 * jb);
        if (t + (int)(hoff >> 4) >= j1) {
            px = kPadSrc;
            nyz = 0x8000000000000000ull;        // -yz_pack(kPadSrc, kPadSrc)
        }
        const uint64_t e0 = add64(L.yz0, nyz), e1 = add64(L.yz1, nyz);
        vote_pair<CW, WIDE>(L.x0 - px, (uint32_t)(e0 >> 32), (uint32_t)e0, v);
        vote_pair<CW, WIDE>(L.x1 - px, (uint32_t)(e1 >> 32), (uint32_t)e1, v);
    }
    j1 = jb;
    if (j0 >= j1) return;
    f4u ax, ay, az, bx, by, bz;
    int j = j0;
    src_issue_lanes(desc, ns, j, hoff, hoff2, ax, ay, az);
    for (; j + 2 * B <= j1; j += 2 * B) {
        src_issue_lanes(desc, ns, j + B, hoff, hoff2, bx, by, bz);
        soa_wait<3>(ax, ay, az);
        if (j >= i0 && j + B <= i1)
            vote8<CW, WIDE, false>(ax, ay, az, L, v);
        else
            vote8<CW, WIDE, true>(ax, ay, az, L, v);
        src_issue_lanes(desc, ns, min(j + 2 * B, j1 - B), hoff, hoff2, ax, ay, az);
        soa_wait<3>(bx, by, bz);
        if (j + B >= i0 && j + 2 * B <= i1)
            vote8<CW, WIDE, false>(bx, by, bz, L, v);
        else
            vote8<CW, WIDE, true>(bx, by, bz, L, v);
    }
    soa_wait<0>(ax, ay, az);              // the last block issued, used or not
    if (j + B <= j1) vote8<CW, WIDE, true>(ax, ay, az, L, v);
}

// Source bucket of a fixed-point x coordinate: (P - sb_lo) >> sb_shift, clamped
// to the table.  Monotone in P, which is all the vote windows rely on.
__device__ __forceinline__ int src_bucket(const SweepArgs &a, int32_t P)
{
    return min(max(P - a.sb_lo, 0) >> a.sb_shift, a.sb_n - 1);
}

// Index range [lo, hi) of the rotation's x-sorted sources whose pairs with any
// reference point of slab-relative x in [ymin, ymax] can fall in the slab's np
// x-planes: 0 <= Y - P < np 2^16 means ymin - np 2^16 < P <= ymax, exactly (the
// arithmetic is integer).  Bucketing is monotone in P, so buckets
// b(ymin - np 2^16 + 1) .. b(ymax) hold every voting source; the per-pair test
// decides the rest.  [ilo, ihi) is the window's interior: sources whose pairs with
// every such reference point fall in the slab's x-planes, ymax - np 2^16 < P <=
// ymin, taken as the whole buckets strictly inside that range (an edge bucket, and
// the two end buckets that also hold clamped values, are left out).
__device__ __forceinline__ void src_window(const SweepArgs &a, __amdgpu_buffer_rsrc_t trs,
                                           int bmin, int bmax, int32_t ymin, int32_t ymax,
                                           int np, int &lo, int &hi, int &ilo, int &ihi)
{
    // the table holds buckets bmin .. bmax only (0 below, n above)
    const int blo = max(src_bucket(a, ymin - (np << 16) + 1), bmin);
    const int bhi = max(src_bucket(a, ymax) + 1, bmin);
    const int bif = max(src_bucket(a, ymax - (np << 16)) + 1, bmin);
    const int bie = max(src_bucket(a, ymin + 1), bmin);
    // the four loads issued unconditionally (one memory round trip), then n selected
    const int tlo = (int)__builtin_amdgcn_raw_buffer_load_b32(trs, 4 * min(blo, bmax), 0, 0);
    const int thi = (int)__builtin_amdgcn_raw_buffer_load_b32(trs, 4 * min(bhi, bmax), 0, 0);
    const int tif = (int)__builtin_amdgcn_raw_buffer_load_b32(trs, 4 * min(bif, bmax), 0, 0);
    const int tie = (int)__builtin_amdgcn_raw_buffer_load_b32(trs, 4 * min(bie, bmax), 0, 0);
    lo = blo > bmax ? a.g.n : tlo;
    hi = bhi > bmax ? a.g.n : thi;
    ilo = bif > bmax ? a.g.n : tif;
    ihi = bie <= bif ? ilo : (bie > bmax ? a.g.n : tie);
}

// Votes of all pairs whose bin falls in the box x-planes [x0, x0 + np) into the
// LDS counters.  Work units are (lane group, part of the group's stream range),
// G parts per group; waves take units one at a time from an LDS counter
// (cleared with the slab), so a wave whose ranges were short takes more units
// instead of idling at the slab's closing barrier.
//   sorted: a lane group is 2^(lg+1) consecutive points of the x-sorted
//           reference, two per lane (points j and j + 2^lg of the group for lane
//           j), held by each of the wave's 64 >> lg lane sub-groups; the stream is
//           the window of the rotation's x-sorted sources, padded to a multiple
//           of 4 and taken in blocks of B = 256 >> lg sources (sub-group h takes
//           4h .. 4h + 3) plus a strided tail (vote_span_lanes);
//   else:   lanes hold 64 rotated sources, the stream is the whole reference.
// lg is a template constant (one instantiation per lane-group size): as a
// run-time value it cost 1.5% of the sweep.
template <int CW, int LG, bool SORTED, bool WIDE>
__device__ void vote_slab(const SweepArgs &a, const float *R, int x0, int np, uint32_t *hist,
                          int slot)
{
    const Geom &g = a.g;
    const int tid = threadIdx.x, lane = tid & 63;
    const uint32_t Sy = g.size[1], Sz = g.size[2];
    const uint32_t syw = (uint32_t)g.row_words, sxw = syw * Sy;
    VoteConst v;
    v.npx = (uint32_t)np << 16;
    v.syx = Sy << 16;
    v.szx = Sz << (CW == 16 ? 15 : 16);
    v.sx = WIDE ? sxw : 4u * sxw;
    v.sy = WIDE ? syw : 4u * syw;
    v.base = (uint32_t)(size_t)(__attribute__((address_space(3))) uint32_t *)hist;
    const uint32_t xofs = (uint32_t)x0 << 16;
    const int m = g.m;
    const int zsel = CW == 16 ? 3 : 2;         // the reference's z array for this width
    uint32_t *ctr = hist + kHistWordsMax + kUnitCounter;
    if (SORTED) {
        constexpr int lg = LG;
        const int gsz = 1 << lg;               // lanes per copy of the group
        const int gref = 2 * gsz;              // reference points per group
        const int B = 256 >> lg;
        const int ngr = (m + gref - 1) / gref;
        const int G = a.vote_parts > 0 ? a.vote_parts : vote_parts_auto(ngr);
        const int total = ngr * G;
        const uint32_t hoff = 16u * (uint32_t)(lane >> lg);
        // part boundaries lo + B * (nb * p * gmul / 8192), nb the window's blocks:
        // nb <= kSortMax / 4 and p * gmul < 8192, so the product stays below 2^32
        const uint32_t gmul = 8192u / (uint32_t)G;
        const int64_t ns = src_stride(a.scratch_stride);
        const int32_t *sp = a.scratch + (size_t)slot * slot_words(a.scratch_stride);
        const f4u sdesc = desc_words(sp, 12 * ns);
        const __amdgpu_buffer_rsrc_t srs = rsrc(sp, 12 * ns);
        const __amdgpu_buffer_rsrc_t yrs = rsrc(a.yq, 16 * (int64_t)m);
        const __amdgpu_buffer_rsrc_t trs = rsrc(sp + 3 * ns, 4 * (kSrcBuckets + 1));
        const uint32_t *scr = hist + kHistWordsMax;
        const int bmin = (int)__builtin_amdgcn_readfirstlane(scr[kSrcBmin]);
        const int bmax = (int)__builtin_amdgcn_readfirstlane(scr[kSrcBmax]);
        for (;;) {
            int u = 0;
            if (lane == 0) u = (int)atomicAdd(ctr, 1u);
            u = __builtin_amdgcn_readfirstlane(u);
            if (u >= total) break;
            const int part = G == 1 ? 0 : u / ngr;
            const int gi = u - part * ngr;
            const int j = gi * gref + (lane & (gsz - 1));
            // padding points (index >= m) never vote; their loads stay inside yq
            const uint32_t yo0 = 4u * (uint32_t)min(j, m - 1);
            const uint32_t yo1 = 4u * (uint32_t)min(j + gsz, m - 1);
            uint32_t x0 = load1(yrs, yo0, 0), y0 = load1(yrs, yo0, 4 * m);
            uint32_t z0 = load1(yrs, yo0, 4 * zsel * m);
            uint32_t x1 = load1(yrs, yo1, 0), y1 = load1(yrs, yo1, 4 * m);
            uint32_t z1 = load1(yrs, yo1, 4 * zsel * m);
            if (j >= m) x0 = y0 = z0 = kPadRef;
            if (j + gsz >= m) x1 = y1 = z1 = kPadRef;
            LanePts L;
            L.x0 = x0 - xofs;
            L.x1 = x1 - xofs;
            L.yz0 = yz_pack(y0, z0);
            L.yz1 = yz_pack(y1, z1);
            // the group's x range: its first and last point (the reference is sorted),
            // read from the first lane sub-group
            const int last = min(m - gi * gref, gref) - 1;
            const int32_t ymin = (int32_t)__builtin_amdgcn_readlane(L.x0, 0);
            const int32_t ymax = (int32_t)(last < gsz ? __builtin_amdgcn_readlane(L.x0, last)
                                                      : __builtin_amdgcn_readlane(L.x1, last - gsz));
            int lo, hi, ilo, ihi;
            src_window(a, trs, bmin, bmax, ymin, ymax, np, lo, hi, ilo, ihi);
            lo = uni(lo);
            hi = uni(max(hi, lo));
            // a multiple of 4 inside the padded arrays: the extra points are
            // sources outside the window or padding, rejected by the range tests
            const int len4 = (hi - lo + 3) & ~3;
            hi = min((int)ns, lo + len4);
            lo = hi - len4;
            // the interior rounded inwards to the same multiples of 4 (it lies inside
            // the window, and only real sources are in it)
            int i0 = lo + ((max(uni(ilo), lo) - lo + 3) & ~3);
            int i1 = lo + ((min(uni(ihi), hi) - lo) & ~3);
            if (i1 <= i0) i0 = i1 = hi;
            const uint32_t nb = (uint32_t)(len4 >> 2);
            const int j0 = uni(lo + 4 * (int)((nb * (uint32_t)part * gmul) >> 13));
            const int j1 = part + 1 == G
                               ? hi
                               : uni(lo + 4 * (int)((nb * (uint32_t)(part + 1) * gmul) >> 13));
            vote_span_lanes<CW, WIDE>(sdesc, srs, (int)ns, j0, j1, i0, i1, B, hoff, L, v);
        }
    } else {
        const int nsg = (g.n + 63) >> 6;
        const int G = a.vote_parts > 0 ? a.vote_parts : vote_parts_auto(nsg);
        const int total = nsg * G;
        const f4u rdesc = desc_words(a.yq, 16 * (int64_t)m);
        const __amdgpu_buffer_rsrc_t rrs = rsrc(a.yq, 16 * (int64_t)m);
        const SoaOffs so = soa_offs(m, zsel);
        const double Sz = CW == 16 ? g.S15 : g.S16;
        for (;;) {
            int u = 0;
            if (lane == 0) u = (int)atomicAdd(ctr, 1u);
            u = __builtin_amdgcn_readfirstlane(u);
            if (u >= total) break;
            const int part = u / nsg;
            const int i = (u - part * nsg) * 64 + lane;
            uint32_t Px = kPadSrc, Py = kPadSrc, Pz = kPadSrc;      // padding lanes never vote
            if (i < g.n) {
                int32_t qx, qy, qz;
                rotate_quant(R, a.src[3 * i], a.src[3 * i + 1], a.src[3 * i + 2], g.S16, Sz, qx,
                             qy, qz);
                Px = (uint32_t)qx;
                Py = (uint32_t)qy;
                Pz = (uint32_t)qz;
            }
            // the slab's first plane folded into the source: D_x = Y_x - (P_x + x0 2^16)
            Px += xofs;
            const int j0 = uni((int)((int64_t)m * part / G));
            const int j1 = uni((int)((int64_t)m * (part + 1) / G));
            vote_span<CW, WIDE>(rdesc, rrs, so, j0, j1, Px, Py, Pz, v);
        }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // asm-issued LDS atomics
}

// A source's (y, z) pair as the reference's: (y << 32) | (z + 2^31).
__device__ __forceinline__ uint64_t yz_src(int32_t y, int32_t z)
{
    return ((uint64_t)(uint32_t)y << 32) | (uint64_t)((uint32_t)z + 0x80000000u);
}

// Bucket-sort the rotated sources of one rotation, in fixed point, by x into this
// workgroup's scratch slot (x, y, z arrays) and write the bucket table after
// them, so that the vote can restrict each reference lane group to the sources
// whose pairs can land in the current slab.
template <int CW>
__device__ void sort_sources(const SweepArgs &a, const float *R, uint32_t *lds, uint32_t *scr,
                             int slot)
{
    const Geom &g = a.g;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t *cnt = lds;                       // kSrcBuckets counters
    uint32_t *key = lds + kSrcBuckets;         // per source: bucket << 16 | rank
    const int64_t ns = src_stride(a.scratch_stride);
    int32_t *ox = a.scratch + (size_t)slot * slot_words(a.scratch_stride);
    uint64_t *oyz = reinterpret_cast<uint64_t *>(ox + ns);
    int32_t *T = ox + 3 * ns;
    const double S16 = g.S16, Sz = CW == 16 ? g.S15 : g.S16;
    for (int b = tid; b < a.sb_n; b += kBlock) cnt[b] = 0u;
    __syncthreads();
    // the first kCarry points of each thread stay in registers between the two
    // passes (no second load and rotation)
    constexpr int kCarry = 4;
    int32_t cpx[kCarry], cpy[kCarry], cpz[kCarry];
    uint32_t ckey[kCarry];
#pragma unroll
    for (int r = 0; r < kCarry; ++r) {
        const int i = tid + r * kBlock;
        if (i < g.n) {
            rotate_quant(R, a.src[3 * i], a.src[3 * i + 1], a.src[3 * i + 2], S16, Sz, cpx[r],
                         cpy[r], cpz[r]);
            const int b = src_bucket(a, cpx[r]);
            ckey[r] = ((uint32_t)b << 16) | atomicAdd(&cnt[b], 1u);
        }
    }
    for (int i = tid + kCarry * kBlock; i < g.n; i += kBlock) {
        int32_t px, py, pz;
        rotate_quant(R, a.src[3 * i], a.src[3 * i + 1], a.src[3 * i + 2], S16, Sz, px, py, pz);
        const int b = src_bucket(a, px);
        key[i] = ((uint32_t)b << 16) | atomicAdd(&cnt[b], 1u);
    }
    __syncthreads();
    // exclusive prefix sum of the bucket counts: each thread owns `per` consecutive
    // buckets; the offsets stay in LDS, and the table entries of the lowest to the
    // highest occupied bucket go to the slot (below that range the table is 0 and
    // above it n, which the vote takes without reading it).  The two bounds are
    // the unique buckets where the prefix leaves 0 and where it reaches n.
    constexpr int kPerMax = kSrcBuckets / kBlock;
    const int per = a.sb_n / kBlock;
    uint32_t loc[kPerMax], sum = 0;
#pragma unroll
    for (int q = 0; q < kPerMax; ++q) {
        loc[q] = q < per ? cnt[per * tid + q] : 0u;
        sum += loc[q];
    }
    uint32_t incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) scr[112 + wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < wave; ++w) run += scr[112 + w];
    const uint32_t n = (uint32_t)g.n;
#pragma unroll
    for (int q = 0; q < kPerMax; ++q) {
        if (q < per) {
            const int b = per * tid + q;
            cnt[b] = run;
            if (loc[q] != 0u) {
                if (run == 0u) scr[kSrcBmin] = (uint32_t)b;
                if (run + loc[q] == n) scr[kSrcBmax] = (uint32_t)b;
            }
            if (run + loc[q] != 0u && run < n) T[b] = (int32_t)run;
            run += loc[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kCarry; ++r) {
        const int i = tid + r * kBlock;
        if (i < g.n) {
            const uint32_t pos = cnt[ckey[r] >> 16] + (ckey[r] & 0xFFFFu);
            ox[pos] = cpx[r];
            oyz[pos] = 0ull - yz_src(cpy[r], cpz[r]);
        }
    }
    for (int i = tid + kCarry * kBlock; i < g.n; i += kBlock) {
        int32_t px, py, pz;
        rotate_quant(R, a.src[3 * i], a.src[3 * i + 1], a.src[3 * i + 2], S16, Sz, px, py, pz);
        const uint32_t kk = key[i];
        const uint32_t pos = cnt[kk >> 16] + (kk & 0xFFFFu);
        ox[pos] = px;
        oyz[pos] = 0ull - yz_src(py, pz);
    }
    // padding up to the padded stride: windows padded to a multiple of 4 may
    // stream it, and no pair with it passes the range tests
    if (tid < (int)(ns - g.n)) {
        ox[g.n + tid] = (int32_t)kPadSrc;
        oyz[g.n + tid] = 0ull - yz_src((int32_t)kPadSrc, (int32_t)kPadSrc);
    }
    __syncthreads();
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Wave64 maximum / minimum of an unsigned value by DPP lane moves (no LDS round
// trip): pairs and quads by quad permutations, eight and sixteen lanes by the
// half-row and row mirrors, then row 0 into row 1 and row 2 into row 3
// (row_bcast:15), rows 0-1 into rows 2-3 (row_bcast:31); lane 63 holds the
// result, read back as a wave-uniform value.  Lanes a move does not write keep
// the identity, so inactive sources never change the result.
template <bool MAX>
__device__ __forceinline__ uint32_t wave_ext_u32(uint32_t v)
{
    const int id = MAX ? 0 : -1;
    auto op = [](uint32_t a, uint32_t b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0xB1, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x4E, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x141, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x140, 0xF, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x142, 0xA, 0xF, false));
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x143, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) { return wave_ext_u32<true>(v); }
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) { return wave_ext_u32<false>(v); }

// Largest counter of a slab (words4 uint4 of counters), workgroup-uniform;
// `mine` receives the largest counter among this thread's own words.
template <int CW>
__device__ uint32_t slab_max(const uint32_t *hist, int words4, uint32_t *scr, uint32_t &mine)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint4 *h4 = reinterpret_cast<const uint4 *>(hist);
    uint32_t mx = 0;
    if (CW == 16) {
        u16x2 m = {0, 0};
        for (int w = tid; w < words4; w += kBlock) {
            const uint4 v = h4[w];
            m = __builtin_elementwise_max(m, __builtin_bit_cast(u16x2, v.x));
            m = __builtin_elementwise_max(m, __builtin_bit_cast(u16x2, v.y));
            m = __builtin_elementwise_max(m, __builtin_bit_cast(u16x2, v.z));
            m = __builtin_elementwise_max(m, __builtin_bit_cast(u16x2, v.w));
        }
        mx = max((uint32_t)m.x, (uint32_t)m.y);
    } else {
        for (int w = tid; w < words4; w += kBlock) {
            const uint4 v = h4[w];
            mx = max(mx, max(max(v.x, v.y), max(v.z, v.w)));
        }
    }
    mine = mx;
    mx = wave_max_u32(mx);
    if (lane == 0) scr[8 + wave] = mx;
    __syncthreads();
    uint32_t r = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) r = max(r, scr[8 + w]);
    // no closing barrier: every hist read came before the barrier above, and
    // scr[8..23] is written next by the next slab's scan, two barriers later
    return r;
}

// Lowest position (word index * 2 + half for 16-bit counters) whose count is c.
// Only threads whose own largest counter (`mine` of slab_max) is c can hold it,
// so the others skip the scan.
template <int CW>
__device__ uint32_t slab_first(const uint32_t *hist, int words4, uint32_t c, uint32_t pos0,
                               uint32_t *scr, uint32_t mine)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint4 *h4 = reinterpret_cast<const uint4 *>(hist);
    uint32_t best = 0xFFFFFFFFu;
    const int wend = mine == c ? words4 : 0;
    for (int w = tid; w < wend && best == 0xFFFFFFFFu; w += kBlock) {
        const uint4 v = h4[w];
        const uint32_t e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 3; q >= 0; --q) {
            if (CW == 16) {
                if ((e[q] >> 16) == c) best = 2u * (4u * w + q) + 1u;
                if ((e[q] & 0xFFFFu) == c) best = 2u * (4u * w + q);
            } else if (e[q] == c) {
                best = 4u * w + q;
            }
        }
    }
    best = wave_min_u32(best);
    if (lane == 0) scr[24 + wave] = best;
    __syncthreads();
    uint32_t r = 0xFFFFFFFFu;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) r = min(r, scr[24 + w]);
    // no closing barrier (its own scratch words, hist reads before the barrier)
    return pos0 + r;
}

// Out of line: inlined, the power function's code sits inside every sweep kernel
// and slowed the C2 sweep by 1.2% although only DSES_TRUNC_LP calls it.
__device__ __attribute__((noinline)) float lp_pow(float x, float p) { return powf(x, p); }

__device__ __forceinline__ float rho(int metric, float d, float dmetric, float d2, float eps,
                                     float tau, float lp)
{
    switch (metric) {
    case DSES_TRUNC_L2: return fminf(d, tau);
    case DSES_TLS: return fminf(d2, tau * tau);
    case DSES_INLIERS: return d < eps ? 0.0f : 1.0f;
    case DSES_TRUNC_LP: return lp_pow(fminf(d, tau), lp);
    default: return fminf(dmetric, tau);          // DSES_TRUNC_L1
    }
}

// Nearest-neighbour terms for one query point.
struct NN {
    float d2;   // squared Euclidean distance to the nearest reference point
    float l1;   // L1 distance to the L1-nearest reference point (TRUNC_L1 only)
};

__device__ __forceinline__ float d2_of(float qx, float qy, float qz, float yx, float yy, float yz)
{
    const float dx = qx - yx, dy = qy - yy, dz = qz - yz;
    return fmaf(dz, dz, fmaf(dy, dy, __fmul_rn(dx, dx)));
}

__device__ __forceinline__ void nn_brute(const float *yt, int m, int j0, int j1, float qx,
                                         float qy, float qz, bool want_l1, NN &nn)
{
    const kfloat yx = kc(yt), yy = kc(yt + m), yz = kc(yt + 2 * m);
    float best = INFINITY, bl1 = INFINITY;
    int j = j0;
    if (!want_l1) {
        float b2 = INFINITY, b3 = INFINITY, b4 = INFINITY;
        for (; j + 4 <= j1; j += 4) {
            best = fminf(best, d2_of(qx, qy, qz, yx[j], yy[j], yz[j]));
            b2 = fminf(b2, d2_of(qx, qy, qz, yx[j + 1], yy[j + 1], yz[j + 1]));
            b3 = fminf(b3, d2_of(qx, qy, qz, yx[j + 2], yy[j + 2], yz[j + 2]));
            b4 = fminf(b4, d2_of(qx, qy, qz, yx[j + 3], yy[j + 3], yz[j + 3]));
        }
        best = fminf(fminf(best, b2), fminf(b3, b4));
        for (; j < j1; ++j) best = fminf(best, d2_of(qx, qy, qz, yx[j], yy[j], yz[j]));
    } else {
        for (; j < j1; ++j) {
            const float dx = qx - yx[j], dy = qy - yy[j], dz = qz - yz[j];
            best = fminf(best, fmaf(dz, dz, fmaf(dy, dy, __fmul_rn(dx, dx))));
            bl1 = fminf(bl1, fabsf(dx) + fabsf(dy) + fabsf(dz));
        }
    }
    nn.d2 = best;
    nn.l1 = bl1;
}

// Exact truncated NN through the cell grid: every reference point within the
// cell pitch (>= r) of q lies in the 3x3x3 cells around q's cell.  Beyond r the
// robust terms saturate, so the result equals brute force.
__device__ __forceinline__ void nn_grid(const CellGrid &cg, float qx, float qy, float qz,
                                        bool want_l1, NN &nn)
{
    const int cx = cvt_flr(__fmul_rn(qx - cg.lo[0], cg.inv));
    const int cy = cvt_flr(__fmul_rn(qy - cg.lo[1], cg.inv));
    const int cz = cvt_flr(__fmul_rn(qz - cg.lo[2], cg.inv));
    float best = INFINITY, bl1 = INFINITY;
    const float4 *pt = reinterpret_cast<const float4 *>(cg.pts);
    // (written without cz - 1 / cz + 1 overflowing when the conversion saturates)
    const int zlo = cz > 0 ? cz - 1 : 0, zhi = cz < cg.dim[2] - 1 ? cz + 1 : cg.dim[2] - 1;
    const int ncell = cg.dim[0] * cg.dim[1] * cg.dim[2];
    const __amdgpu_buffer_rsrc_t st = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t *>(cg.start), 0, 4 * (ncell + 1), 0x00020000);
    // a row's start and end offsets are at most 3 entries apart: one 16-byte load
    // (bounds-checked by the descriptor) brings both; ez (1..3) indexes the end
    const int ez = zhi - zlo + 1;
    // the bounds of all nine rows first, so their loads are in flight together; a
    // row outside the grid reads at an offset past the table, which the descriptor
    // turns into zeros (an empty row)
    int rb[9], re[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const uint32_t ix = (uint32_t)cx + (uint32_t)(r / 3) - 1u;
        const uint32_t iy = (uint32_t)cy + (uint32_t)(r % 3) - 1u;
        const bool ok = zlo <= zhi && ix < (uint32_t)cg.dim[0] && iy < (uint32_t)cg.dim[1];
        const int off =
            ok ? 4 * (((int)ix * cg.dim[1] + (int)iy) * cg.dim[2] + zlo) : 0x7FFFFFF0;
        const f4u s4 = __builtin_amdgcn_raw_buffer_load_b128(st, off, 0, 0);
        rb[r] = (int)s4.x;
        re[r] = (int)(ez == 1 ? s4.y : (ez == 2 ? s4.z : s4.w));
    }
#pragma unroll
    for (int r = 0; r < 9; ++r)
        for (int j = rb[r]; j < re[r]; ++j) {
            const float4 y = pt[j];
            const float dx = qx - y.x, dy = qy - y.y, dz = qz - y.z;
            best = fminf(best, fmaf(dz, dz, fmaf(dy, dy, __fmul_rn(dx, dx))));
            if (want_l1) bl1 = fminf(bl1, fabsf(dx) + fabsf(dy) + fabsf(dz));
        }
    nn.d2 = best;
    nn.l1 = bl1;
}

// Distance-field value of voxel (ix, iy, iz); r outside the grid.
__device__ __forceinline__ float df_at(const Field &f, int ix, int iy, int iz)
{
    const uint32_t R = (uint32_t)f.res;
    if ((uint32_t)ix < R && (uint32_t)iy < R && (uint32_t)iz < R)
        return f.val[((size_t)ix * R + iy) * R + iz];
    return f.r;
}

// Nearest-voxel lookup: idx_a = floor((q_a - lo_a) * inv_a); r outside the grid.
__device__ __forceinline__ float df_nearest(const Field &f, float qx, float qy, float qz)
{
    return df_at(f, cvt_flr(__fmul_rn(qx - f.lo[0], f.inv[0])),
                 cvt_flr(__fmul_rn(qy - f.lo[1], f.inv[1])),
                 cvt_flr(__fmul_rn(qz - f.lo[2], f.inv[2])));
}

// Trilinear lookup: u_a = (q_a - lo_a) * inv_a - 1/2 in voxel-centre units, the
// eight centres floor(u) + {0, 1} weighted by the fractional parts (a centre
// outside the grid counts as r); r when every centre is outside along an axis
// (u_a < -1 or u_a >= res, NaN included).
__device__ __forceinline__ float df_trilinear(const Field &f, float qx, float qy, float qz)
{
    const float ux = __fmul_rn(qx - f.lo[0], f.inv[0]) - 0.5f;
    const float uy = __fmul_rn(qy - f.lo[1], f.inv[1]) - 0.5f;
    const float uz = __fmul_rn(qz - f.lo[2], f.inv[2]) - 0.5f;
    const float R = (float)f.res;
    if (!(ux >= -1.0f && ux < R && uy >= -1.0f && uy < R && uz >= -1.0f && uz < R)) return f.r;
    const float fx = floorf(ux), fy = floorf(uy), fz = floorf(uz);
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    const float wx = ux - fx, wy = uy - fy, wz = uz - fz;
    float c[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const float v0 = df_at(f, ix + a, iy + b, iz), v1 = df_at(f, ix + a, iy + b, iz + 1);
            c[a][b] = fmaf(wz, v1 - v0, v0);
        }
    const float e0 = fmaf(wy, c[0][1] - c[0][0], c[0][0]);
    const float e1 = fmaf(wy, c[1][1] - c[1][0], c[1][0]);
    return fmaf(wx, e1 - e0, e0);
}

// Score candidate {R_k, t_k = b delta} (Eq. (1)/(2): sum over the source of the
// robust distance to the nearest reference point, and the inliers) with the
// whole workgroup, and write its record.  kScoreNone writes the record unscored
// (error +inf, 0 inliers).
template <int SCORER>
__device__ void score_candidate(const SweepArgs &a, int k, const float *R, int bx, int by, int bz,
                                uint32_t votes, uint32_t *lds)
{
    const Geom &g = a.g;
    uint32_t *hist = lds;
    uint32_t *scr = lds + kHistWordsMax;          // kScratchWords words
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (SCORER == kScoreNone || SCORER == kScoreVotes) {
        if (tid == 0) {
            dses_record rec;
            rec.bin[0] = bx;
            rec.bin[1] = by;
            rec.bin[2] = bz;
            rec.votes = votes;
            rec.inliers = SCORER == kScoreVotes ? (int32_t)votes : 0;
            rec.error = SCORER == kScoreVotes ? 0.0f : INFINITY;
            a.rec[k] = rec;
        }
        return;
    }
    const float tx = __fmul_rn((float)bx, g.delta);
    const float ty = __fmul_rn((float)by, g.delta);
    const float tz = __fmul_rn((float)bz, g.delta);
    const bool want_l1 = g.metric == DSES_TRUNC_L1;
    float err = 0.0f;
    int inl = 0;
    float *part = reinterpret_cast<float *>(hist);
    for (int c0 = 0; c0 < g.n; c0 += kBlock) {
        const ChunkLayout L = (SCORER == DSES_SCORER_BRUTE)
                                  ? chunk_layout(c0, g.n, wave, lane)
                                  : ChunkLayout{kWaves, 1, 0, c0 + tid, true};
        NN nn;
        nn.d2 = INFINITY;
        nn.l1 = INFINITY;
        float D = 0.0f;
        const bool valid = L.active && L.i < g.n;
        if (SCORER == DSES_SCORER_BRUTE) {
            if (L.active) {
                float qx = 1.0e7f, qy = 1.0e7f, qz = 1.0e7f;
                if (valid) {
                    float px, py, pz;
                    rotate(R, a.src[3 * L.i], a.src[3 * L.i + 1], a.src[3 * L.i + 2], px, py, pz);
                    qx = px + tx;
                    qy = py + ty;
                    qz = pz + tz;
                }
                const int j0 = uni((int)((int64_t)g.m * L.part / L.G));
                const int j1 = uni((int)((int64_t)g.m * (L.part + 1) / L.G));
                nn_brute(a.yt, g.m, j0, j1, qx, qy, qz, want_l1, nn);
            }
        } else if (valid) {
            float px, py, pz;
            rotate(R, a.src[3 * L.i], a.src[3 * L.i + 1], a.src[3 * L.i + 2], px, py, pz);
            const float qx = px + tx, qy = py + ty, qz = pz + tz;
            if (SCORER == DSES_SCORER_GRID)
                nn_grid(a.grid, qx, qy, qz, want_l1, nn);
            else
                D = a.field.lookup == DSES_DF_TRILINEAR ? df_trilinear(a.field, qx, qy, qz)
                                                        : df_nearest(a.field, qx, qy, qz);
        }
        if (SCORER == DSES_SCORER_BRUTE && L.G > 1) {
            // combine the reference partitions of each source point
            const int slot = L.part * L.sw * 64 + (wave % L.sw) * 64 + lane;
            if (L.active) {
                part[slot] = nn.d2;
                if (want_l1) part[kBlock + slot] = nn.l1;
            }
            __syncthreads();
            if (L.active && L.part == 0) {
                for (int p = 1; p < L.G; ++p) {
                    const int o = p * L.sw * 64 + (wave % L.sw) * 64 + lane;
                    nn.d2 = fminf(nn.d2, part[o]);
                    if (want_l1) nn.l1 = fminf(nn.l1, part[kBlock + o]);
                }
            }
            __syncthreads();
        }
        if (valid && L.part == 0) {
            if (SCORER == DSES_SCORER_DF) {
                err += rho(g.metric, D, D, D * D, g.eps, g.tau, g.lp);
                inl += D < g.eps ? 1 : 0;
            } else {
                const float d = sqrtf(nn.d2);
                const float dm = want_l1 ? nn.l1 : d;
                err += rho(g.metric, d, dm, nn.d2, g.eps, g.tau, g.lp);
                inl += d < g.eps ? 1 : 0;
            }
        }
    }
    // fixed-order workgroup reduction
    err = wave_sum(err);
    inl = wave_isum(inl);
    float *fscr = reinterpret_cast<float *>(scr);
    if (lane == 0) { fscr[64 + wave] = err; scr[96 + wave] = (uint32_t)inl; }
    __syncthreads();
    if (tid == 0) {
        float e = 0.0f;
        int c = 0;
        for (int q = 0; q < kWaves; ++q) { e += fscr[64 + q]; c += (int)scr[96 + q]; }
        dses_record rec;
        rec.bin[0] = bx;
        rec.bin[1] = by;
        rec.bin[2] = bz;
        rec.votes = votes;
        rec.inliers = c;
        rec.error = e;
        a.rec[k] = rec;
    }
    __syncthreads();                          // LDS scratch reused by the caller
}

// The vote of one slab with the lane-group size and source layout of this call.
template <int CW, bool WIDE>
__device__ __forceinline__ void vote_slab_any(const SweepArgs &a, const float *R, int x0, int np,
                                              uint32_t *hist, int slot, bool sorted, int lg)
{
    if (!sorted)
        vote_slab<CW, 6, false, WIDE>(a, R, x0, np, hist, slot);
    else if (lg == 3)
        vote_slab<CW, 3, true, WIDE>(a, R, x0, np, hist, slot);
    else if (lg == 4)
        vote_slab<CW, 4, true, WIDE>(a, R, x0, np, hist, slot);
    else
        vote_slab<CW, 5, true, WIDE>(a, R, x0, np, hist, slot);
}

// Vote, mode and score one rotation k with the whole workgroup; `slot` selects
// the workgroup's source-sort scratch.  Writes a.rec[k].
template <int CW, int SCORER>
__device__ void sweep_one(const SweepArgs &a, int k, uint32_t *lds, int slot)
{
    const Geom &g = a.g;
    uint32_t *hist = lds;
    uint32_t *scr = lds + kHistWordsMax;          // kScratchWords words
    const int tid = threadIdx.x;
    const uint32_t Sy = g.size[1];
    const uint32_t RW = (uint32_t)g.row_words;
    const bool sorted = a.scratch != nullptr;
    const int lg = a.lane_group == 16   ? 3
                   : a.lane_group == 32 ? 4
                   : a.lane_group == 64 ? 5
                                        : lane_group_log2(g.m, g.n, g.size[0], a.ref_x_extent,
                                                          a.vote_parts);
  {
    float R[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) R[e] = kc(a.rot)[9 * k + e];
    if (sorted) sort_sources<CW>(a, R, lds, scr, slot);

    // ---------------- vote + mode over the slabs ----------------
    // Barriers per slab: after the clear, after the vote, and one inside each
    // scan (after its per-wave partials); the scans read hist only before theirs,
    // so the next slab's clear (or the scoring) needs no further barrier.
    uint32_t best_c = 0, best_p = 0xFFFFFFFFu;
    for (int slab = 0; slab < g.nslabs; ++slab) {
        const int x0 = slab * g.pps;
        const int np = min(g.pps, g.size[0] - x0);
        const int words = np * (int)Sy * (int)RW;
        const int words4 = (words + 3) >> 2;
        uint4 *h4 = reinterpret_cast<uint4 *>(hist);
        for (int w = tid; w < words4; w += kBlock) h4[w] = make_uint4(0, 0, 0, 0);
        if (tid == 0) scr[kUnitCounter] = 0u;
        __syncthreads();
        if (g.wide)
            vote_slab_any<CW, true>(a, R, x0, np, hist, slot, sorted, lg);
        else
            vote_slab_any<CW, false>(a, R, x0, np, hist, slot, sorted, lg);
        __syncthreads();
        // the slab's largest count first (cheap), and only when it beats the best of
        // the earlier slabs its lowest position (a later slab never wins a tie: its
        // positions are higher)
        const uint32_t pos0 = (uint32_t)x0 * Sy * RW * (CW == 16 ? 2u : 1u);
        uint32_t mine;
        const uint32_t smax = slab_max<CW>(hist, words4, scr, mine);
        if (smax > best_c) {
            best_p = slab_first<CW>(hist, words4, smax, pos0, scr, mine);
            best_c = smax;
        }
    }

    dses_record rec;
    if (best_c == 0) {
        if (tid == 0) {
            rec.bin[0] = rec.bin[1] = rec.bin[2] = 0;
            rec.votes = 0;
            rec.inliers = 0;
            rec.error = INFINITY;
            a.rec[k] = rec;
        }
        return;
    }
    // position -> box-relative bin
    const uint32_t w = CW == 16 ? best_p >> 1 : best_p;
    const uint32_t row = w / RW;
    const int cz = (int)((w - row * RW) * (CW == 16 ? 2u : 1u) + (CW == 16 ? (best_p & 1u) : 0u));
    const int cy = (int)(row % Sy), cx = (int)(row / Sy);
    const int bx = cx + g.klo[0], by = cy + g.klo[1], bz = cz + g.klo[2];
    score_candidate<SCORER>(a, k, R, bx, by, bz, best_c, lds);
  }
}

template <int CW, int SCORER>
__global__ void __launch_bounds__(kBlock) k_sweep(SweepArgs a)
{
    __shared__ __align__(16) uint32_t lds[kLdsWords];
    for (int k = blockIdx.x; k < a.k; k += gridDim.x) sweep_one<CW, SCORER>(a, k, lds, blockIdx.x);
}

template <int CW, int SC>
static hipError_t launch_one(const SweepArgs &a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL((k_sweep<CW, SC>), dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

// grid: persistent workgroups (each sweeps rotations blockIdx.x, +gridDim.x, ...);
// with a.scratch set it must not exceed the number of scratch slots.
hipError_t launch_sweep(const SweepArgs &a, int scorer, int grid, hipStream_t stream)
{
    if (a.k <= 0) return hipSuccess;
    if (grid > a.k) grid = a.k;
    if (a.g.counter_bits == 16) {
        switch (scorer) {
        case kScoreNone: return launch_one<16, kScoreNone>(a, grid, stream);
        case kScoreVotes: return launch_one<16, kScoreVotes>(a, grid, stream);
        case DSES_SCORER_BRUTE: return launch_one<16, DSES_SCORER_BRUTE>(a, grid, stream);
        case DSES_SCORER_GRID: return launch_one<16, DSES_SCORER_GRID>(a, grid, stream);
        default: return launch_one<16, DSES_SCORER_DF>(a, grid, stream);
        }
    }
    switch (scorer) {
    case kScoreNone: return launch_one<32, kScoreNone>(a, grid, stream);
    case kScoreVotes: return launch_one<32, kScoreVotes>(a, grid, stream);
    case DSES_SCORER_BRUTE: return launch_one<32, DSES_SCORER_BRUTE>(a, grid, stream);
    case DSES_SCORER_GRID: return launch_one<32, DSES_SCORER_GRID>(a, grid, stream);
    default: return launch_one<32, DSES_SCORER_DF>(a, grid, stream);
    }
}

// --------------------------------------------------------------------------
// q-pruned scoring (the pruning step of Alg. 2): after a vote-only sweep
// (kScoreNone records), M* = the largest vote count, and only rotations with
// M_k >= q M* are scored.  The comparison is made in double precision on the
// integer counts and the float q, so it is exact and reproducible on the host.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_max_votes(const dses_record *rec, int32_t K,
                                                    uint32_t *mstar, uint32_t *cursor)
{
    __shared__ uint32_t sm[16];
    uint32_t m = 0;
    for (int k = threadIdx.x; k < K; k += blockDim.x) m = max(m, rec[k].votes);
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t r = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = max(r, sm[w]);
        *mstar = r;
        *cursor = 0u;                    // work cursor of the pruned scoring
    }
}

__device__ __forceinline__ bool keep_candidate(uint32_t votes, uint32_t mstar, float q)
{
    return votes > 0u && (double)votes >= (double)q * (double)mstar;
}

constexpr int kPruneChunk = 32;          // rotations per cursor fetch

template <int SCORER>
__global__ void __launch_bounds__(kBlock) k_score_pruned(SweepArgs a, float q,
                                                         const uint32_t *mstar, uint32_t *cursor)
{
    __shared__ __align__(16) uint32_t lds[kLdsWords];
    const uint32_t ms = __builtin_amdgcn_readfirstlane(*(kint)(const int32_t *)mstar);
    for (;;) {
        if (threadIdx.x == 0) lds[kLdsWords - 1] = atomicAdd(cursor, (uint32_t)kPruneChunk);
        __syncthreads();
        const int k0 = __builtin_amdgcn_readfirstlane((int)lds[kLdsWords - 1]);
        __syncthreads();
        if (k0 >= a.k) break;
        const int k1 = min(a.k, k0 + kPruneChunk);
        for (int k = k0; k < k1; ++k) {
            const dses_record r = a.rec[k];
            if (!keep_candidate(r.votes, ms, q)) continue;
            float R[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) R[e] = kc(a.rot)[9 * k + e];
            score_candidate<SCORER>(a, k, R, r.bin[0], r.bin[1], r.bin[2], r.votes, lds);
        }
    }
}

// --------------------------------------------------------------------------
// Alg. 1, the pure exhaustive search: every rotation with every lattice
// translation b delta of the box.  One workgroup per rotation holds the rotated
// sources in LDS; each thread scores whole translations (the error summed over
// the source in index order, nearest reference point by the cell grid or by
// brute force) and keeps its best; a workgroup reduction picks the rotation's
// best translation (smaller error, then more inliers, then the lower linear
// index of b).  The record carries votes = 1 (Alg. 1 has no vote).
// --------------------------------------------------------------------------
__device__ __forceinline__ bool exh_better(float e, int i, uint32_t u, float oe, int oi,
                                           uint32_t ou)
{
    if (oe < e) return true;
    if (oe > e) return false;
    if (oi != i) return oi > i;
    return ou < u;
}

template <int SCORER>
__global__ void __launch_bounds__(kBlock) k_exhaustive(SweepArgs a)
{
    __shared__ float sp[3 * kExhaustiveMaxSrc];
    __shared__ float re[kWaves];
    __shared__ int ri[kWaves];
    __shared__ uint32_t ru[kWaves];
    const Geom &g = a.g;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = g.n;
    const uint32_t sz = (uint32_t)g.size[2], syz = (uint32_t)g.size[1] * sz;
    const uint32_t T = (uint32_t)g.size[0] * syz;
    const bool want_l1 = g.metric == DSES_TRUNC_L1;
    for (int k = blockIdx.x; k < a.k; k += gridDim.x) {
        float R[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) R[e] = kc(a.rot)[9 * k + e];
        for (int i = tid; i < n; i += kBlock)
            rotate(R, a.src[3 * i], a.src[3 * i + 1], a.src[3 * i + 2], sp[i], sp[n + i],
                   sp[2 * n + i]);
        __syncthreads();
        float be = INFINITY;
        int bi = 0;
        uint32_t bu = 0xFFFFFFFFu;
        for (uint32_t u = (uint32_t)tid; u < T; u += kBlock) {
            const uint32_t ux = u / syz, uy = (u - ux * syz) / sz, uz = u - ux * syz - uy * sz;
            const float tx = __fmul_rn((float)(g.klo[0] + (int)ux), g.delta);
            const float ty = __fmul_rn((float)(g.klo[1] + (int)uy), g.delta);
            const float tz = __fmul_rn((float)(g.klo[2] + (int)uz), g.delta);
            float err = 0.0f;
            int inl = 0;
            for (int i = 0; i < n; ++i) {
                const float qx = sp[i] + tx, qy = sp[n + i] + ty, qz = sp[2 * n + i] + tz;
                NN nn;
                if (SCORER == DSES_SCORER_GRID)
                    nn_grid(a.grid, qx, qy, qz, want_l1, nn);
                else
                    nn_brute(a.yt, g.m, 0, g.m, qx, qy, qz, want_l1, nn);
                const float d = sqrtf(nn.d2);
                err += rho(g.metric, d, want_l1 ? nn.l1 : d, nn.d2, g.eps, g.tau, g.lp);
                inl += d < g.eps ? 1 : 0;
            }
            if (exh_better(be, bi, bu, err, inl, u)) { be = err; bi = inl; bu = u; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const float oe = __shfl_xor(be, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            const uint32_t ou = (uint32_t)__shfl_xor((int)bu, off, 64);
            if (exh_better(be, bi, bu, oe, oi, ou)) { be = oe; bi = oi; bu = ou; }
        }
        if (lane == 0) { re[wave] = be; ri[wave] = bi; ru[wave] = bu; }
        __syncthreads();
        if (tid == 0) {
            float e = re[0];
            int c = ri[0];
            uint32_t w = ru[0];
            for (int q = 1; q < kWaves; ++q)
                if (exh_better(e, c, w, re[q], ri[q], ru[q])) { e = re[q]; c = ri[q]; w = ru[q]; }
            const uint32_t ux = w / syz, uy = (w - ux * syz) / sz, uz = w - ux * syz - uy * sz;
            dses_record rec;
            rec.bin[0] = g.klo[0] + (int)ux;
            rec.bin[1] = g.klo[1] + (int)uy;
            rec.bin[2] = g.klo[2] + (int)uz;
            rec.votes = 1u;
            rec.inliers = c;
            rec.error = e;
            a.rec[k] = rec;
        }
        __syncthreads();                       // sp and the reduction slots are reused
    }
}

hipError_t launch_exhaustive(const SweepArgs &a, int scorer, int grid, hipStream_t stream)
{
    if (a.k <= 0) return hipSuccess;
    if (a.g.n > kExhaustiveMaxSrc) return hipErrorInvalidValue;
    if (grid > a.k) grid = a.k;
    if (scorer == DSES_SCORER_BRUTE)
        hipLaunchKernelGGL(k_exhaustive<DSES_SCORER_BRUTE>, dim3(grid), dim3(kBlock), 0, stream, a);
    else
        hipLaunchKernelGGL(k_exhaustive<DSES_SCORER_GRID>, dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_score_pruned(const SweepArgs &a, int scorer, float q, uint32_t *mstar,
                               uint32_t *cursor, int grid, hipStream_t stream)
{
    if (a.k <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_max_votes, dim3(1), dim3(1024), 0, stream,
                       static_cast<const dses_record *>(a.rec), a.k, mstar, cursor);
    if (grid > a.k) grid = a.k;
    switch (scorer) {
    case DSES_SCORER_BRUTE:
        hipLaunchKernelGGL(k_score_pruned<DSES_SCORER_BRUTE>, dim3(grid), dim3(kBlock), 0, stream,
                           a, q, mstar, cursor);
        break;
    case DSES_SCORER_GRID:
        hipLaunchKernelGGL(k_score_pruned<DSES_SCORER_GRID>, dim3(grid), dim3(kBlock), 0, stream,
                           a, q, mstar, cursor);
        break;
    default:
        hipLaunchKernelGGL(k_score_pruned<DSES_SCORER_DF>, dim3(grid), dim3(kBlock), 0, stream,
                           a, q, mstar, cursor);
        break;
    }
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// selection: argmin over records of (error, -inliers, index)
// --------------------------------------------------------------------------
__device__ __forceinline__ bool sel_better(float e, int i, int k, float oe, int oi, int ok)
{
    // true if (oe, oi, ok) beats (e, i, k); k < 0 means "none"
    if (ok < 0) return false;
    if (k < 0) return true;
    if (oe < e) return true;
    if (oe > e) return false;
    if (oi > i) return true;
    if (oi < i) return false;
    return ok < k;
}

__device__ void select_body(const dses_record *rec, int32_t K, const float *rot, float delta,
                            DevResult *res, const uint32_t *status, float *se, int *si, int *sk,
                            int *sv)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float be = INFINITY;
    int bi = 0, bk = -1, nvalid = 0;
    for (int k = tid; k < K; k += blockDim.x) {
        const dses_record r = rec[k];
        if (r.votes == 0) continue;
        ++nvalid;
        if (sel_better(be, bi, bk, r.error, r.inliers, k)) { be = r.error; bi = r.inliers; bk = k; }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const float oe = __shfl_xor(be, off, 64);
        const int oi = __shfl_xor(bi, off, 64), ok = __shfl_xor(bk, off, 64);
        if (sel_better(be, bi, bk, oe, oi, ok)) { be = oe; bi = oi; bk = ok; }
        nvalid += __shfl_xor(nvalid, off, 64);
    }
    if (lane == 0) { se[wave] = be; si[wave] = bi; sk[wave] = bk; sv[wave] = nvalid; }
    __syncthreads();
    if (tid == 0) {
        float e = INFINITY;
        int i = 0, k = -1, nv = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            nv += sv[w];
            if (sel_better(e, i, k, se[w], si[w], sk[w])) { e = se[w]; i = si[w]; k = sk[w]; }
        }
        res->rot_index = k;
        res->n_valid = nv;
        res->bad_input = status ? status[0] : 0u;
        if (k >= 0) {
            const dses_record r = rec[k];
            res->votes = r.votes;
            res->inliers = r.inliers;
            res->error = r.error;
            for (int a2 = 0; a2 < 3; ++a2) res->t[a2] = __fmul_rn((float)r.bin[a2], delta);
            for (int e2 = 0; e2 < 9; ++e2) res->R[e2] = rot[9 * (size_t)k + e2];
        }
    }
}

__global__ void __launch_bounds__(1024) k_select(const dses_record *rec, int32_t K,
                                                 const float *rot, float delta, DevResult *res,
                                                 const uint32_t *status)
{
    __shared__ float se[16];
    __shared__ int si[16], sk[16], sv[16];
    select_body(rec, K, rot, delta, res, status, se, si, sk, sv);
}

hipError_t launch_select(const dses_record *rec, int32_t k, const float *rot, float delta,
                         DevResult *res, const uint32_t *status, hipStream_t stream)
{
    hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, stream, rec, k, rot, delta, res,
                       status);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// top-k: the k best candidates in selection order.  An entry is the triple
// (error bits, ~inliers, index), compared as unsigned integers: for the
// non-negative errors of valid candidates the float order equals the bit order,
// ~inliers puts more inliers first, and the index breaks the remaining ties, so
// the order is exactly the one of sel_better.  Rotations without an in-box vote
// become (all ones), after every valid entry.
// --------------------------------------------------------------------------
constexpr int kTopChunk = 2048;     // entries sorted per workgroup and pass

struct TopEntry {
    uint32_t e, ninl, idx;
};

__device__ __forceinline__ bool top_less(const TopEntry &a, const TopEntry &b)
{
    if (a.e != b.e) return a.e < b.e;
    if (a.ninl != b.ninl) return a.ninl < b.ninl;
    return a.idx < b.idx;
}

// One pass: workgroup b sorts entries [b * kTopChunk, ...) in LDS (bitonic) and
// writes its first k to out[b * k, ...).  FROM_REC: the entries are built from
// records (index = position), else read from a previous pass.
template <bool FROM_REC>
__global__ void __launch_bounds__(1024) k_topk_pass(const void *in, int32_t count, int32_t k,
                                                    TopEntry *out)
{
    __shared__ uint32_t se[kTopChunk], sn[kTopChunk], si[kTopChunk];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTopChunk;
    for (int q = tid; q < kTopChunk; q += blockDim.x) {
        TopEntry t{0xffffffffu, 0xffffffffu, 0xffffffffu};
        const int64_t g = base + q;
        if (g < count) {
            if (FROM_REC) {
                const dses_record r = static_cast<const dses_record *>(in)[g];
                if (r.votes != 0) t = TopEntry{__float_as_uint(r.error), ~(uint32_t)r.inliers,
                                               (uint32_t)g};
            } else {
                t = static_cast<const TopEntry *>(in)[g];
            }
        }
        se[q] = t.e;
        sn[q] = t.ninl;
        si[q] = t.idx;
    }
    __syncthreads();
    for (int size = 2; size <= kTopChunk; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < kTopChunk / 2; t += blockDim.x) {
                const int i = 2 * stride * (t / stride) + (t % stride), j = i + stride;
                const bool up = (i & size) == 0;
                const TopEntry a{se[i], sn[i], si[i]}, b{se[j], sn[j], si[j]};
                if (top_less(b, a) == up) {
                    se[i] = b.e; sn[i] = b.ninl; si[i] = b.idx;
                    se[j] = a.e; sn[j] = a.ninl; si[j] = a.idx;
                }
            }
            __syncthreads();
        }
    if (tid < k) out[(int64_t)blockIdx.x * k + tid] = TopEntry{se[tid], sn[tid], si[tid]};
}

__global__ void k_topk_emit(const TopEntry *top, int32_t k, const dses_record *rec, float delta,
                            dses_candidate *out)
{
    const int t = threadIdx.x;
    if (t >= k) return;
    dses_candidate c{-1, 0, INFINITY, 0u, {0.0f, 0.0f, 0.0f}};
    const TopEntry e = top[t];
    if (e.idx != 0xffffffffu) {
        const dses_record r = rec[e.idx];
        c.rot_index = (int32_t)e.idx;
        c.inliers = r.inliers;
        c.error = r.error;
        c.votes = r.votes;
        for (int a = 0; a < 3; ++a) c.t[a] = __fmul_rn((float)r.bin[a], delta);
    }
    out[t] = c;
}

size_t topk_scratch_bytes(int32_t K, int32_t k)
{
    return (size_t)((K + kTopChunk - 1) / kTopChunk) * (size_t)k * sizeof(TopEntry);
}

hipError_t launch_topk(const dses_record *rec, int32_t K, int32_t k, float delta, void *scr_a,
                       void *scr_b, dses_candidate *out, hipStream_t stream)
{
    int32_t count = K;
    int blocks = (count + kTopChunk - 1) / kTopChunk;
    auto *a = static_cast<TopEntry *>(scr_a), *b = static_cast<TopEntry *>(scr_b);
    hipLaunchKernelGGL(k_topk_pass<true>, dim3(blocks), dim3(1024), 0, stream,
                       static_cast<const void *>(rec), count, k, a);
    while (blocks > 1) {
        count = blocks * k;
        blocks = (count + kTopChunk - 1) / kTopChunk;
        hipLaunchKernelGGL(k_topk_pass<false>, dim3(blocks), dim3(1024), 0, stream,
                           static_cast<const void *>(a), count, k, b);
        std::swap(a, b);
    }
    hipLaunchKernelGGL(k_topk_emit, dim3(1), dim3(64), 0, stream, a, k, rec, delta, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// batched registration: one persistent launch over a work list of
// (instance, rotation tile) items, most expensive first, fetched dynamically.
// Each rotation runs the same sweep_one() as the single-registration kernel, so
// a registration's records do not depend on what it is batched with.
// --------------------------------------------------------------------------
// In-kernel completion of a batched instance (serving): after its tile the
// workgroup adds the tile's rotations to the instance's count; the one that
// brings it to K selects the result exactly as k_select does, returns the count
// to zero for the slot's next instance and raises the flag the host polls.
// Records are written by thread 0 only (sweep_one), so its release fence before
// the count covers the tile.
__device__ void finish_item(const BatchArgs &b, const BatchItem &w, const SweepArgs &a,
                            uint32_t *lds)
{
    uint32_t *last = lds + kLdsWords - 2;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t cnt = (uint32_t)(w.k1 - w.k0);
        const uint32_t prev = atomicAdd(b.done_rot + w.inst, cnt);
        const bool done = prev + cnt == (uint32_t)a.k;
        if (done) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the others' records
        *last = done ? 1u : 0u;
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane((int)*last) == 0) return;
    // selection scratch in the (now unused) vote array
    float *se = reinterpret_cast<float *>(lds);
    int *si = reinterpret_cast<int *>(lds + 16), *sk = si + 16, *sv = si + 32;
    select_body(a.rec, a.k, a.rot, a.g.delta, b.res + w.inst, nullptr, se, si, sk, sv);
    if (threadIdx.x == 0) {
        atomicExch(b.done_rot + w.inst, 0u);
        __threadfence_system();                   // the result before the flag
        __hip_atomic_store(b.done_flag + w.inst, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
}

template <int SCORER>
__global__ void __launch_bounds__(kBlock) k_sweep_batch(BatchArgs b)
{
    __shared__ __align__(16) uint32_t lds[kLdsWords];
    const int n_items = __builtin_amdgcn_readfirstlane(*(kint)(const int32_t *)b.header);
    for (;;) {
        if (threadIdx.x == 0) lds[kLdsWords - 1] = atomicAdd(b.cursor, 1u) - b.cursor_base;
        __syncthreads();
        const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)lds[kLdsWords - 1]);
        __syncthreads();
        if (it >= (uint32_t)n_items) break;
        const BatchItem w = kload(b.items + it);
        SweepArgs a = kload(b.inst + w.inst);
        int slot = blockIdx.x;
        if (b.scratch && a.scratch) {
            // this launch's slot; the instance's own stride lays out the arrays in it
            a.scratch = b.scratch + (size_t)blockIdx.x * (size_t)b.scratch_slot;
            slot = 0;
        }
        for (int k = w.k0; k < w.k1; ++k) {
            if (a.g.counter_bits == 16)
                sweep_one<16, SCORER>(a, k, lds, slot);
            else
                sweep_one<32, SCORER>(a, k, lds, slot);
        }
        if (b.done_rot) finish_item(b, w, a, lds);
    }
}

hipError_t launch_sweep_batch(const BatchArgs &b, int scorer, int grid, hipStream_t stream)
{
    switch (scorer) {
    case DSES_SCORER_BRUTE:
        hipLaunchKernelGGL(k_sweep_batch<DSES_SCORER_BRUTE>, dim3(grid), dim3(kBlock), 0, stream, b);
        break;
    case DSES_SCORER_GRID:
        hipLaunchKernelGGL(k_sweep_batch<DSES_SCORER_GRID>, dim3(grid), dim3(kBlock), 0, stream, b);
        break;
    default:
        hipLaunchKernelGGL(k_sweep_batch<DSES_SCORER_DF>, dim3(grid), dim3(kBlock), 0, stream, b);
        break;
    }
    return hipGetLastError();
}

__global__ void k_stage_batch(const StageDesc *d, const int32_t *header)
{
    const int count = header[1];
    for (int inst = blockIdx.y; inst < count; inst += gridDim.y) {
        const StageDesc sd = d[inst];
        for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < sd.m; j += gridDim.x * blockDim.x)
            stage_point(sd.tgt, sd.perm ? sd.perm[j] : j, j, sd.m, sd.S16, sd.S15, sd.klo, sd.yq,
                        sd.yt);
    }
}

// The same selection by one wave64 with shuffles only.  It uses no LDS, so it
// can start on a CU next to a sweep workgroup of another launch (the served
// path overlaps launches) instead of waiting for a CU to drain.
__device__ void select_wave(const dses_record *rec, int32_t K, const float *rot, float delta,
                            DevResult *res, const uint32_t *status)
{
    const int lane = threadIdx.x;
    float be = INFINITY;
    int bi = 0, bk = -1, nvalid = 0;
    for (int k = lane; k < K; k += 64) {
        const dses_record r = rec[k];
        if (r.votes == 0) continue;
        ++nvalid;
        if (sel_better(be, bi, bk, r.error, r.inliers, k)) { be = r.error; bi = r.inliers; bk = k; }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const float oe = __shfl_xor(be, off, 64);
        const int oi = __shfl_xor(bi, off, 64), ok = __shfl_xor(bk, off, 64);
        if (sel_better(be, bi, bk, oe, oi, ok)) { be = oe; bi = oi; bk = ok; }
        nvalid += __shfl_xor(nvalid, off, 64);
    }
    if (lane == 0) {
        res->rot_index = bk;
        res->n_valid = nvalid;
        res->bad_input = status ? status[0] : 0u;
        if (bk >= 0) {
            const dses_record r = rec[bk];
            res->votes = r.votes;
            res->inliers = r.inliers;
            res->error = r.error;
            for (int a2 = 0; a2 < 3; ++a2) res->t[a2] = __fmul_rn((float)r.bin[a2], delta);
            for (int e2 = 0; e2 < 9; ++e2) res->R[e2] = rot[9 * (size_t)bk + e2];
        }
    }
}

__global__ void __launch_bounds__(64) k_select_batch(const SelectDesc *d, const int32_t *header)
{
    const int count = header[1];
    for (int inst = blockIdx.x; inst < count; inst += gridDim.x) {
        const SelectDesc sd = d[inst];
        select_wave(sd.rec, sd.k, sd.rot, sd.delta, sd.res, sd.status);
    }
}

hipError_t launch_batch_aux(const StageDesc *stage, const SelectDesc *sel, const int32_t *header,
                            int max_count, int which, hipStream_t stream)
{
    const int gy = max_count < 1 ? 1 : (max_count > 65535 ? 65535 : max_count);
    if (which == 0)
        hipLaunchKernelGGL(k_stage_batch, dim3(16, gy), dim3(256), 0, stream, stage, header);
    else
        hipLaunchKernelGGL(k_select_batch, dim3(gy), dim3(64), 0, stream, sel, header);
    return hipGetLastError();
}

}  // namespace dses
