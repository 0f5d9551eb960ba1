/*
 * DSES CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of Direct Semi-Exhaustive
 * Search (Cheng et al., "A Direct Semi-Exhaustive Search Method for Robust,
 * Partial-to-Full Point Cloud Registration"), used by the tests, by the smoke
 * check and by the CPU-baseline leg of the benchmark to check the HIP path.
 * Nothing in the product links or calls this file.  It shares no code, header or
 * constant with the HIP library.
 *
 * Precision.  Everything is computed in IEEE double from the float32 input bits,
 * which promote exactly.  The translation bin of a point pair is the plain
 * definition of ROUND in Alg. 2 (Lemma 2, Eq. (5)):
 *     u = (y_j - R x_i) / delta    (per axis, true division),   b = floor(u + 1/2),
 * the nearest lattice point b*delta, halves rounded up.  A pair whose u + 1/2 lies
 * within mu bin units of an integer on some axis is *fragile*: any evaluation of u
 * that is accurate to mu (a float32 kernel is, by orders of magnitude) may put it
 * in the neighbouring bin across that face instead.  For every bin the vote keeps
 * the count cnt(b) by the definition and two fragility counts,
 *     out(b): fragile pairs counted in b that may belong elsewhere,
 *     in(b):  fragile pairs counted elsewhere (or outside the box) that may belong to b,
 * so any such evaluation counts a number of pairs in [cnt - out, cnt + in] in b.
 * From these the mode is *pinned* (every such evaluation has the same mode b*,
 * tie-break included) or ambiguous; an ambiguous rotation's admissible modes are
 * the bins with cnt + in >= max over bins of (cnt - out).
 *
 * The same reading applies to the voxel of a distance-field lookup (the field is
 * this library's own scorer variant, not the paper's): the voxel of q is
 * floor((q - lo)/h) in double, and a coordinate within mu_df voxel units of a
 * voxel face makes the point's value an interval over the voxels it may fall in.
 *
 * A secondary mode (lib_zbits = 15 or 16) takes both decisions instead by the
 * library's documented formulas: the fixed-point bin decision with z at 2^-lib_zbits
 * bins (lib_bin_of_pair) and the single-precision voxel decision (df_voxel_of_f32).
 * It exists only for a labelled, secondary bit-exactness check; every parity
 * claim rests on the double-precision definition.
 *
 * Build: gcc -O2 -std=gnu11 -ffp-contract=off -fPIC -shared -pthread -lm
 * (-ffp-contract=off keeps every rounding step exactly as written).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

enum { ORC_TRUNC_L2 = 0, ORC_INLIERS = 1, ORC_TLS = 2, ORC_TRUNC_L1 = 3, ORC_TRUNC_LP = 4,
       ORC_VOTES = 5 };
enum { ORC_DF_NEAREST = 0, ORC_DF_TRILINEAR = 1 };

/* Per-rotation outcome of Alg. 2, one row of the candidate list (80 bytes). */
typedef struct {
    int32_t bin[3];     /* mode bin b* (t* = delta * b*), lattice units            */
    uint32_t votes;     /* M = cnt(b*): vote count of the mode bin                  */
    int32_t inliers;    /* #{i : d_i < eps} at t*                                   */
    int32_t boundary;   /* #{i : |d_i - eps| <= 1e-6}, reported, not compared      */
    double error;       /* e(R, t*) under the chosen metric                        */
    int32_t valid;      /* 0 when no pair voted inside the translation box         */
    int32_t rot;        /* index of the rotation in the caller's list              */
    uint32_t votes_lo;  /* cnt(b*) - out(b*)                                       */
    uint32_t votes_hi;  /* cnt(b*) + in(b*)                                        */
    uint32_t lo_max;    /* max over bins of cnt - out                              */
    int32_t pinned;     /* 1: the mode (and validity) is the same for every        */
                        /*    evaluation accurate to mu                            */
    int32_t frag;       /* fragile pairs with an effect inside the box             */
    int32_t inl_frag;   /* points whose distance-field value is fragile and whose  */
                        /*    inlier decision depends on the voxel taken           */
    double err_lo;      /* error range over the fragile voxel choices              */
    double err_hi;      /*   (both equal error for the exact scorer)               */
} orc_record;

/* ------------------------------------------------------------------------ */
/* Translation box (Sec. IV-B: the vote array spans the translation search   */
/* range).  Lattice points b*delta with t_min <= b*delta <= t_max per axis,   */
/* with a 1e-4 bin-unit tolerance so that a range end which is a multiple of  */
/* delta up to float rounding is included.                                   */
/* ------------------------------------------------------------------------ */
int orc_box(float delta, const float *t_min, const float *t_max, int32_t *k_lo, int32_t *size)
{
    if (!(delta > 0.0f) || !isfinite(delta)) return -1;
    for (int a = 0; a < 3; ++a) {
        double lo = ceil((double)t_min[a] / (double)delta - 1e-4);
        double hi = floor((double)t_max[a] / (double)delta + 1e-4);
        if (!(hi >= lo) || hi - lo + 1 > 4096 || fabs(lo) > 1e6 || fabs(hi) > 1e6) return -1;
        k_lo[a] = (int32_t)lo;
        size[a] = (int32_t)(hi - lo + 1);
    }
    return 0;
}

static size_t lin_of(const int32_t *b, const int32_t *k_lo, const int32_t *size)
{
    return ((size_t)(b[0] - k_lo[0]) * size[1] + (size_t)(b[1] - k_lo[1])) * size[2] +
           (size_t)(b[2] - k_lo[2]);
}

static int in_box(const int32_t *b, const int32_t *k_lo, const int32_t *size)
{
    for (int a = 0; a < 3; ++a)
        if (b[a] < k_lo[a] || b[a] >= k_lo[a] + size[a]) return 0;
    return 1;
}

static void bin_of_lin(size_t l, const int32_t *k_lo, const int32_t *size, int32_t *b)
{
    b[2] = (int32_t)(l % (size_t)size[2]) + k_lo[2];
    b[1] = (int32_t)((l / (size_t)size[2]) % (size_t)size[1]) + k_lo[1];
    b[0] = (int32_t)(l / ((size_t)size[1] * size[2])) + k_lo[0];
}

/* R x in double: row a of R dotted with x, left to right. */
static void rotate64(const float *R, const float *x, double *p)
{
    for (int a = 0; a < 3; ++a)
        p[a] = (double)R[3 * a] * x[0] + (double)R[3 * a + 1] * x[1] + (double)R[3 * a + 2] * x[2];
}

/* ------------------------------------------------------------------------ */
/* Lemma 2 / Alg. 2 first loop, by the definition: for one rotation, every   */
/* pair (i, j) votes for b = floor((y_j - R x_i)/delta + 1/2); the mode is    */
/* the bin with the largest count, ties to the lowest linear index (x         */
/* slowest; the paper is silent).  Fills the dense count and fragility arrays */
/* (each nbins long) and the summary below.                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t mode[3];
    uint32_t M, lo, hi, lo_max;
    int32_t pinned, frag;
} vote_info;

static void vote64(const float *src, int32_t n, const float *tgt, int32_t m, const float *R,
                   double delta, double mu, const int32_t *k_lo, const int32_t *size,
                   uint32_t *cnt, uint32_t *outf, uint32_t *inf, vote_info *vi)
{
    const size_t nbins = (size_t)size[0] * size[1] * size[2];
    memset(cnt, 0, nbins * sizeof(uint32_t));
    memset(outf, 0, nbins * sizeof(uint32_t));
    memset(inf, 0, nbins * sizeof(uint32_t));
    int32_t frag = 0;
    for (int32_t i = 0; i < n; ++i) {
        double p[3];
        rotate64(R, src + 3 * i, p);
        for (int32_t j = 0; j < m; ++j) {
            const float *y = tgt + 3 * j;
            int32_t b[3], alt[3];
            int mask = 0, far = 0;
            for (int a = 0; a < 3; ++a) {
                double u = ((double)y[a] - p[a]) / delta;
                double w = u + 0.5;
                double f = floor(w);
                /* two bins or more outside the box: neither b nor a neighbour is in it */
                if (!(f >= k_lo[a] - 1.5 && f <= (double)k_lo[a] + size[a] + 0.5)) {
                    far = 1;
                    break;
                }
                b[a] = (int32_t)f;
                double frac = w - f;            /* in [0, 1) */
                alt[a] = b[a];
                if (frac < mu) { alt[a] = b[a] - 1; mask |= 1 << a; }
                else if (frac > 1.0 - mu) { alt[a] = b[a] + 1; mask |= 1 << a; }
            }
            if (far) continue;
            if (!mask) {
                if (in_box(b, k_lo, size)) cnt[lin_of(b, k_lo, size)] += 1;
                continue;
            }
            /* a fragile pair: the definition's bin (combination 0) and every bin
               reached by moving across some of its near faces */
            int effect = 0;
            for (int c = 0; c < 8; ++c) {
                if (c & ~mask) continue;
                int32_t v[3];
                for (int a = 0; a < 3; ++a) v[a] = ((c >> a) & 1) ? alt[a] : b[a];
                if (!in_box(v, k_lo, size)) continue;
                size_t l = lin_of(v, k_lo, size);
                effect = 1;
                if (c == 0) { cnt[l] += 1; outf[l] += 1; }
                else inf[l] += 1;
            }
            frag += effect;
        }
    }
    /* mode: the first largest count; `before` / `after` track the largest count
       at lower / higher linear index than the current best */
    uint32_t best = 0, before = 0, after = 0;
    size_t arg = 0;
    for (size_t l = 0; l < nbins; ++l) {
        if (cnt[l] > best) { before = best; best = cnt[l]; arg = l; after = 0; }
        else if (cnt[l] > after && l > arg) after = cnt[l];
    }
    int any_in = 0;
    for (size_t l = 0; l < nbins; ++l) {
        if (!inf[l]) continue;
        any_in = 1;
        uint32_t h = cnt[l] + inf[l];
        if (l < arg && h > before) before = h;
        if (l > arg && h > after) after = h;
    }
    bin_of_lin(arg, k_lo, size, vi->mode);
    vi->M = best;
    vi->lo = best - outf[arg];
    vi->hi = best + inf[arg];
    vi->frag = frag;
    if (best == 0)
        vi->pinned = !any_in;         /* no pair can vote in the box */
    else
        vi->pinned = vi->lo > before && vi->lo >= after;
    if (vi->pinned) {
        vi->lo_max = vi->lo;          /* lo(b*) >= hi(b) >= lo(b) for every b */
    } else {
        uint32_t L = 0;
        for (size_t l = 0; l < nbins; ++l)
            if (cnt[l] - outf[l] > L) L = cnt[l] - outf[l];
        vi->lo_max = L;
    }
}

/* Exported for the pins and for admissibility queries: one rotation, dense arrays
   (cnt, out, in) of size[0]*size[1]*size[2] entries each, x slowest.
   info = {mode_x, mode_y, mode_z, M, lo, hi, lo_max, pinned, frag}. */
int orc_vote64(const float *src, int32_t n, const float *tgt, int32_t m, const float *R,
               float delta, double mu, const int32_t *k_lo, const int32_t *size, uint32_t *cnt,
               uint32_t *outf, uint32_t *inf, int32_t *info)
{
    if (n < 0 || m < 0 || !(delta > 0.0f) || !(mu >= 0.0 && mu < 0.5)) return -1;
    vote_info vi;
    vote64(src, n, tgt, m, R, (double)delta, mu, k_lo, size, cnt, outf, inf, &vi);
    info[0] = vi.mode[0]; info[1] = vi.mode[1]; info[2] = vi.mode[2];
    info[3] = (int32_t)vi.M; info[4] = (int32_t)vi.lo; info[5] = (int32_t)vi.hi;
    info[6] = (int32_t)vi.lo_max; info[7] = vi.pinned; info[8] = vi.frag;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* SECONDARY CHECK ONLY: the library's documented fixed-point form of the    */
/* bin decision.  With S_F = (1/delta) 2^F in double (F = 16 on x and y,     */
/* F = zbits on z),                                                          */
/*   Y_a = rint(y_a S_F + (1/2 - k_lo_a) 2^F),                               */
/*   p_a = (R_a0 x_x + R_a1 x_y) + R_a2 x_z,                                 */
/*   P_a = rint(p_a S_F clamped to [-2^30, 2^30]),                           */
/*   c_a = floor((Y_a - P_a) / 2^F)           (box-relative),                 */
/* every product and sum one rounded double operation, rint rounding halves  */
/* to even.  It agrees with the definition except for pairs within 2^-zbits   */
/* bins of a face; it is used for a labelled bit-exactness check of the      */
/* kernel's arithmetic, never for parity.                                    */
/* ------------------------------------------------------------------------ */
static int32_t q_rint(double v) { return (int32_t)nearbyint(v); }

static void lib_quant_src(const float *R, const float *x, const double *S, int32_t *P)
{
    for (int a = 0; a < 3; ++a) {
        double p = (double)R[3 * a + 0] * (double)x[0];
        p = p + (double)R[3 * a + 1] * (double)x[1];
        p = p + (double)R[3 * a + 2] * (double)x[2];
        double v = p * S[a];
        v = v < -1073741824.0 ? -1073741824.0 : (v > 1073741824.0 ? 1073741824.0 : v);
        P[a] = q_rint(v);
    }
}

static int lib_bin_of_pair(const float *y, const int32_t *P, const double *S, const int *F,
                           const int32_t *k_lo, const int32_t *size, int32_t *c)
{
    int inside = 1;
    for (int a = 0; a < 3; ++a) {
        double v = (double)y[a] * S[a];
        v = v + (0.5 - (double)k_lo[a]) * ldexp(1.0, F[a]);
        const int64_t D = (int64_t)q_rint(v) - (int64_t)P[a];
        c[a] = (int32_t)(D >> F[a]);          /* floor: arithmetic shift */
        if (c[a] < 0 || c[a] >= size[a]) inside = 0;
    }
    return inside;
}

uint32_t orc_vote_lib(const float *src, int32_t n, const float *tgt, int32_t m, const float *R,
                      float delta, int32_t zbits, const int32_t *k_lo, const int32_t *size,
                      uint32_t *hist, int32_t *mode_bin)
{
    const size_t nbins = (size_t)size[0] * size[1] * size[2];
    const double s = 1.0 / (double)delta;
    const int F[3] = {16, 16, zbits};
    const double S[3] = {s * 65536.0, s * 65536.0, s * ldexp(1.0, zbits)};
    memset(hist, 0, nbins * sizeof(uint32_t));
    for (int32_t i = 0; i < n; ++i) {
        int32_t P[3];
        lib_quant_src(R, src + 3 * i, S, P);
        for (int32_t j = 0; j < m; ++j) {
            int32_t c[3];
            if (lib_bin_of_pair(tgt + 3 * j, P, S, F, k_lo, size, c))
                hist[((size_t)c[0] * size[1] + c[1]) * size[2] + c[2]] += 1;
        }
    }
    uint32_t best = 0;
    size_t arg = 0;
    for (size_t l = 0; l < nbins; ++l)
        if (hist[l] > best) { best = hist[l]; arg = l; }
    bin_of_lin(arg, k_lo, size, mode_bin);
    return best;
}

/* The library's single-precision rotation of a source point for scoring,
   p_a = fma(R_a2, x_z, fma(R_a1, x_y, R_a0 * x_x)) (secondary checks only). */
static void rotate_f32(const float *R, const float *x, float *p)
{
    for (int a = 0; a < 3; ++a) {
        float acc = R[3 * a + 0] * x[0];
        acc = fmaf(R[3 * a + 1], x[1], acc);
        acc = fmaf(R[3 * a + 2], x[2], acc);
        p[a] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Eq. (1)/(2): for a query q, min over the reference cloud of ||y_j - q||.  */
/* Brute force over every reference point, in double.                       */
/* ------------------------------------------------------------------------ */
static double nn_dist(const double *q, const float *tgt, int32_t m, int l1)
{
    double best = INFINITY;
    for (int32_t j = 0; j < m; ++j) {
        double dx = (double)tgt[3 * j + 0] - q[0];
        double dy = (double)tgt[3 * j + 1] - q[1];
        double dz = (double)tgt[3 * j + 2] - q[2];
        double d = l1 ? fabs(dx) + fabs(dy) + fabs(dz) : sqrt(dx * dx + dy * dy + dz * dz);
        if (d < best) best = d;
    }
    return best;
}

void orc_nn(const double *q, int32_t nq, const float *tgt, int32_t m, int32_t l1, double *out)
{
    for (int32_t i = 0; i < nq; ++i) out[i] = nn_dist(q + 3 * i, tgt, m, l1);
}

/* Robust per-point error rho(d) for the metrics of Sec. III / IV-B; lp is the */
/* exponent of the truncated Lp objective (p < 1: the sparsity norms that the */
/* paper allows in place of the L1 norm).                                     */
static double rho(int metric, double d, double tau, double eps, double lp)
{
    switch (metric) {
    case ORC_TRUNC_L2: return d < tau ? d : tau;                    /* sum min(d, tau)     */
    case ORC_TLS:      return d < tau ? d * d : tau * tau;          /* sum min(d^2, tau^2) */
    case ORC_INLIERS:  return d < eps ? 0.0 : 1.0;                  /* L0^{m1}: N - inliers */
    case ORC_TRUNC_L1: return d < tau ? d : tau;                    /* with the L1 NN dist  */
    case ORC_TRUNC_LP: return pow(d < tau ? d : tau, lp);           /* sum min(d, tau)^p   */
    default:           return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 error loop for one candidate {R, t}: e = sum_i rho(min_j ||.||),   */
/* summed over the source X and minimised over the reference Y as in         */
/* Eq. (1)/(2) (X is the partial view, Y the full object).                   */
/* ------------------------------------------------------------------------ */
static void score_candidate(const float *src, int32_t n, const float *tgt, int32_t m,
                            const float *R, const double *t, int metric, double eps, double tau,
                            double lp, orc_record *rec)
{
    double err = 0.0;
    int32_t inl = 0, bnd = 0;
    for (int32_t i = 0; i < n; ++i) {
        double q[3];
        rotate64(R, src + 3 * i, q);
        for (int a = 0; a < 3; ++a) q[a] += t[a];
        double d2 = nn_dist(q, tgt, m, 0);
        double d = metric == ORC_TRUNC_L1 ? nn_dist(q, tgt, m, 1) : d2;
        if (d2 < eps) ++inl;
        if (fabs(d2 - eps) <= 1e-6) ++bnd;
        err += rho(metric, d, tau, eps, lp);
    }
    rec->inliers = inl;
    rec->boundary = bnd;
    rec->error = err;
    rec->err_lo = err;
    rec->err_hi = err;
    rec->inl_frag = 0;
}

/* ------------------------------------------------------------------------ */
/* Voxel distance field of the reference (one per target): a res^3 grid over */
/* the reference bounding box padded by r = max(tau, eps), voxel centres     */
/*   c_a = lo_a + (idx_a + 1/2) h_a,                                          */
/* value D = min(min_j ||c - y_j||, r) in double.  The box parameters are     */
/* defined in single precision (they are the field's definition, not a       */
/* result):                                                                  */
/*   lo_a = min_j y_a - r,  hi_a = max_j y_a + r,  h_a = (hi_a - lo_a)/res,   */
/*   inv_a = 1/h_a                                         (float arithmetic) */
/* Outside the padded box every point is farther than r from the reference,  */
/* so the field's value there is r.                                          */
/* ------------------------------------------------------------------------ */
void orc_df_params(const float *tgt, int32_t m, float r, int32_t res, float *lo, float *h,
                   float *inv)
{
    for (int a = 0; a < 3; ++a) {
        float mn = tgt[a], mx = tgt[a];
        for (int32_t j = 1; j < m; ++j) {
            float v = tgt[3 * j + a];
            if (v < mn) mn = v;
            if (v > mx) mx = v;
        }
        float l = mn - r, u = mx + r;
        float ext = u - l;
        lo[a] = l;
        h[a] = ext / (float)res;
        inv[a] = 1.0f / h[a];
    }
}

typedef struct {
    const float *tgt; int32_t m; float r; int32_t res;
    const float *lo; const float *h; double *field;
    int32_t begin, end;
} df_job;

static void *df_worker(void *arg)
{
    df_job *jb = (df_job *)arg;
    const int32_t res = jb->res;
    for (int32_t ix = jb->begin; ix < jb->end; ++ix)
        for (int32_t iy = 0; iy < res; ++iy)
            for (int32_t iz = 0; iz < res; ++iz) {
                double c[3] = {(double)jb->lo[0] + (ix + 0.5) * (double)jb->h[0],
                               (double)jb->lo[1] + (iy + 0.5) * (double)jb->h[1],
                               (double)jb->lo[2] + (iz + 0.5) * (double)jb->h[2]};
                double d = nn_dist(c, jb->tgt, jb->m, 0);
                jb->field[((size_t)ix * res + iy) * res + iz] = d < jb->r ? d : (double)jb->r;
            }
    return NULL;
}

static int n_threads(int32_t want)
{
    if (want > 0) return want;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

int orc_df_build(const float *tgt, int32_t m, float r, int32_t res, int32_t nthreads,
                 float *lo, float *h, float *inv, double *field)
{
    if (m <= 0 || res <= 0 || !(r > 0.0f)) return -1;
    orc_df_params(tgt, m, r, res, lo, h, inv);
    int nt = n_threads(nthreads);
    if (nt > res) nt = res;
    pthread_t th[256];
    df_job jobs[256];
    if (nt > 256) nt = 256;
    for (int w = 0; w < nt; ++w) {
        jobs[w] = (df_job){tgt, m, r, res, lo, h, field, (int32_t)((int64_t)res * w / nt),
                           (int32_t)((int64_t)res * (w + 1) / nt)};
        pthread_create(&th[w], NULL, df_worker, &jobs[w]);
    }
    for (int w = 0; w < nt; ++w) pthread_join(th[w], NULL);
    return 0;
}

typedef struct {
    const double *field; int32_t res; float r; const float *lo; const float *h;
    const float *inv; int lookup; double mu;
} df_view;

/* Field value at voxel idx; r outside the grid. */
static double df_at(const df_view *f, const int32_t *idx)
{
    for (int a = 0; a < 3; ++a)
        if (idx[a] < 0 || idx[a] >= f->res) return (double)f->r;
    return f->field[((size_t)idx[0] * f->res + idx[1]) * f->res + idx[2]];
}

/* Nearest-voxel lookup of a double query: the voxel is floor((q - lo)/h) per
   axis.  Returns the definition's value in *D and the smallest / largest value
   over the voxels reachable by moving across faces within mu voxel units. */
static void df_nearest64(const df_view *f, const double *q, double *D, double *Dmin,
                         double *Dmax)
{
    int32_t idx[3], alt[3];
    int mask = 0;
    for (int a = 0; a < 3; ++a) {
        double u = (q[a] - (double)f->lo[a]) / (double)f->h[a];
        double w = floor(u);
        if (!(w >= -1.5 && w <= f->res + 0.5)) {    /* far outside: every neighbour too */
            idx[a] = alt[a] = -2;
            continue;
        }
        idx[a] = alt[a] = (int32_t)w;
        double frac = u - w;
        if (frac < f->mu) { alt[a] = idx[a] - 1; mask |= 1 << a; }
        else if (frac > 1.0 - f->mu) { alt[a] = idx[a] + 1; mask |= 1 << a; }
    }
    *D = *Dmin = *Dmax = df_at(f, idx);
    for (int c = 1; c < 8; ++c) {
        if (c & ~mask) continue;
        int32_t v[3];
        for (int a = 0; a < 3; ++a) v[a] = ((c >> a) & 1) ? alt[a] : idx[a];
        double d = df_at(f, v);
        if (d < *Dmin) *Dmin = d;
        if (d > *Dmax) *Dmax = d;
    }
}

/* Trilinear lookup: the field's values at the voxel centres (r at virtual centres
   outside the grid) interpolated linearly along each axis.  Continuous in q, so
   it has no fragile decision. */
static double df_trilinear64(const df_view *f, const double *q)
{
    int32_t i0[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) {
        double u = (q[a] - (double)f->lo[a]) / (double)f->h[a] - 0.5;
        if (!(u >= -1.0 && u < (double)f->res)) return (double)f->r;   /* all corners out */
        double w = floor(u);
        i0[a] = (int32_t)w;
        fr[a] = u - w;
    }
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
        int32_t v[3];
        double wgt = 1.0;
        for (int a = 0; a < 3; ++a) {
            int hi = (c >> (2 - a)) & 1;
            v[a] = i0[a] + hi;
            wgt *= hi ? fr[a] : 1.0 - fr[a];
        }
        acc += wgt * df_at(f, v);
    }
    return acc;
}

/* Exported for the pins: per-query field values of double queries q (nq x 3):
   D by the lookup's definition, Dmin / Dmax over the fragile voxel choices. */
int orc_df_query(const double *q, int32_t nq, const double *field, int32_t res, float r,
                 const float *lo, const float *h, int32_t lookup, double mu, double *D,
                 double *Dmin, double *Dmax)
{
    if (res <= 0 || !(r > 0.0f) || !(mu >= 0.0 && mu < 0.5)) return -1;
    if (lookup != ORC_DF_NEAREST && lookup != ORC_DF_TRILINEAR) return -1;
    df_view f = {field, res, r, lo, h, NULL, lookup, mu};
    for (int32_t i = 0; i < nq; ++i) {
        if (lookup == ORC_DF_TRILINEAR)
            D[i] = Dmin[i] = Dmax[i] = df_trilinear64(&f, q + 3 * i);
        else
            df_nearest64(&f, q + 3 * i, &D[i], &Dmin[i], &Dmax[i]);
    }
    return 0;
}

static void score_candidate_df64(const float *src, int32_t n, const float *R, const double *t,
                                 int metric, double eps, double tau, double lp, const df_view *f,
                                 orc_record *rec)
{
    double err = 0.0, elo = 0.0, ehi = 0.0;
    int32_t inl = 0, bnd = 0, ifr = 0;
    for (int32_t i = 0; i < n; ++i) {
        double q[3], D, Dmin, Dmax;
        rotate64(R, src + 3 * i, q);
        for (int a = 0; a < 3; ++a) q[a] += t[a];
        if (f->lookup == ORC_DF_TRILINEAR) {
            D = Dmin = Dmax = df_trilinear64(f, q);
        } else {
            df_nearest64(f, q, &D, &Dmin, &Dmax);
        }
        if (D < eps) ++inl;
        if (fabs(D - eps) <= 1e-6) ++bnd;
        if ((Dmin < eps) != (Dmax < eps)) ++ifr;
        double e = rho(metric, D, tau, eps, lp);
        double e1 = rho(metric, Dmin, tau, eps, lp), e2 = rho(metric, Dmax, tau, eps, lp);
        err += e;
        elo += e1 < e2 ? e1 : e2;   /* every rho here is non-decreasing in d */
        ehi += e1 < e2 ? e2 : e1;
    }
    rec->inliers = inl;
    rec->boundary = bnd;
    rec->error = err;
    rec->err_lo = elo;
    rec->err_hi = ehi;
    rec->inl_frag = ifr;
}

/* SECONDARY CHECK ONLY: the library's documented single-precision lookup,
   q = fma-chain(R x) + t in float, idx_a = floor((q_a - lo_a) * inv_a). */
static int df_voxel_of_f32(const float *q, const float *lo, const float *inv, int32_t res,
                           int32_t *idx)
{
    int inside = 1;
    for (int a = 0; a < 3; ++a) {
        float u = q[a] - lo[a];
        u = u * inv[a];
        idx[a] = (int32_t)floorf(u);
        if (idx[a] < 0 || idx[a] >= res) inside = 0;
    }
    return inside;
}

static void score_candidate_df_f32(const float *src, int32_t n, const float *R, const float *tf,
                                   int metric, double eps, double tau, double lp,
                                   const df_view *f, orc_record *rec)
{
    double err = 0.0;
    int32_t inl = 0, bnd = 0;
    for (int32_t i = 0; i < n; ++i) {
        float p[3], q[3];
        int32_t idx[3];
        rotate_f32(R, src + 3 * i, p);
        for (int a = 0; a < 3; ++a) q[a] = p[a] + tf[a];
        double D = df_voxel_of_f32(q, f->lo, f->inv, f->res, idx) ? df_at(f, idx) : (double)f->r;
        if (D < eps) ++inl;
        if (fabs(D - eps) <= 1e-6) ++bnd;
        err += rho(metric, D, tau, eps, lp);
    }
    rec->inliers = inl;
    rec->boundary = bnd;
    rec->error = err;
    rec->err_lo = err;
    rec->err_hi = err;
    rec->inl_frag = 0;
}

/* Score one candidate {R, delta * bin} with the chosen scorer. */
static void score_bin(const float *src, int32_t n, const float *tgt, int32_t m, const float *R,
                      const int32_t *bin, float delta, int metric, double eps, double tau,
                      double lp, const df_view *f, int lib_zbits, orc_record *rec)
{
    if (f->field && lib_zbits) {
        float tf[3];
        for (int a = 0; a < 3; ++a) tf[a] = (float)bin[a] * delta;
        score_candidate_df_f32(src, n, R, tf, metric, eps, tau, lp, f, rec);
        return;
    }
    double t[3];
    for (int a = 0; a < 3; ++a) t[a] = (double)bin[a] * (double)delta;
    if (f->field)
        score_candidate_df64(src, n, R, t, metric, eps, tau, lp, f, rec);
    else
        score_candidate(src, n, tgt, m, R, t, metric, eps, tau, lp, rec);
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 over a list of rotations (q = 0: every candidate is scored).       */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *src; int32_t n; const float *tgt; int32_t m;
    const float *rots; const int32_t *which; const int32_t *bins;
    float delta; double mu; const int32_t *k_lo; const int32_t *size;
    int metric; double eps, tau, lp; int lib_zbits;
    df_view f;
    orc_record *out;
    int32_t begin, end;
} reg_job;

static void *reg_worker(void *arg)
{
    reg_job *jb = (reg_job *)arg;
    const size_t nbins = (size_t)jb->size[0] * jb->size[1] * jb->size[2];
    uint32_t *cnt = (uint32_t *)malloc(nbins * sizeof(uint32_t));
    uint32_t *outf = (uint32_t *)malloc(nbins * sizeof(uint32_t));
    uint32_t *inf = (uint32_t *)malloc(nbins * sizeof(uint32_t));
    if (!cnt || !outf || !inf) { free(cnt); free(outf); free(inf); return (void *)1; }
    for (int32_t u = jb->begin; u < jb->end; ++u) {
        int32_t k = jb->which ? jb->which[u] : u;
        const float *R = jb->rots + 9 * (size_t)k;
        orc_record *rec = &jb->out[u];
        memset(rec, 0, sizeof(*rec));
        rec->rot = k;
        if (jb->lib_zbits) {
            rec->votes = orc_vote_lib(jb->src, jb->n, jb->tgt, jb->m, R, jb->delta, jb->lib_zbits,
                                      jb->k_lo, jb->size, cnt, rec->bin);
            rec->votes_lo = rec->votes_hi = rec->lo_max = rec->votes;
            rec->pinned = 1;
        } else {
            vote_info vi;
            vote64(jb->src, jb->n, jb->tgt, jb->m, R, (double)jb->delta, jb->mu, jb->k_lo,
                   jb->size, cnt, outf, inf, &vi);
            for (int a = 0; a < 3; ++a) rec->bin[a] = vi.mode[a];
            rec->votes = vi.M;
            rec->votes_lo = vi.lo;
            rec->votes_hi = vi.hi;
            rec->lo_max = vi.lo_max;
            rec->pinned = vi.pinned;
            rec->frag = vi.frag;
        }
        rec->valid = rec->votes > 0;
        if (!rec->valid) { rec->error = rec->err_lo = rec->err_hi = INFINITY; continue; }
        if (jb->metric == ORC_VOTES) {
            /* Thm. 3 ranking: no scoring, the mode count stands for the L0^{m1}
             * inlier count and the error is 0 for every valid candidate */
            rec->inliers = (int32_t)rec->votes;
            continue;
        }
        score_bin(jb->src, jb->n, jb->tgt, jb->m, R, rec->bin, jb->delta, jb->metric, jb->eps,
                  jb->tau, jb->lp, &jb->f, jb->lib_zbits, rec);
    }
    free(cnt);
    free(outf);
    free(inf);
    return NULL;
}

/* Scores of given (rotation, bin) pairs, no vote: for the candidates whose mode
   is ambiguous, each admissible bin is scored by this. */
static void *bins_worker(void *arg)
{
    reg_job *jb = (reg_job *)arg;
    for (int32_t u = jb->begin; u < jb->end; ++u) {
        int32_t k = jb->which[u];
        orc_record *rec = &jb->out[u];
        memset(rec, 0, sizeof(*rec));
        rec->rot = k;
        for (int a = 0; a < 3; ++a) rec->bin[a] = jb->bins[3 * u + a];
        rec->valid = 1;
        rec->pinned = 1;
        score_bin(jb->src, jb->n, jb->tgt, jb->m, jb->rots + 9 * (size_t)k, rec->bin, jb->delta,
                  jb->metric, jb->eps, jb->tau, jb->lp, &jb->f, jb->lib_zbits, rec);
    }
    return NULL;
}

static int run_jobs(reg_job *proto, int32_t count, int32_t nthreads, void *(*fn)(void *))
{
    int nt = n_threads(nthreads);
    if (nt > 256) nt = 256;
    if (nt > count) nt = count > 0 ? count : 1;
    pthread_t th[256];
    reg_job jobs[256];
    for (int w = 0; w < nt; ++w) {
        jobs[w] = *proto;
        jobs[w].begin = (int32_t)((int64_t)count * w / nt);
        jobs[w].end = (int32_t)((int64_t)count * (w + 1) / nt);
        pthread_create(&th[w], NULL, fn, &jobs[w]);
    }
    int bad = 0;
    for (int w = 0; w < nt; ++w) {
        void *ret = NULL;
        pthread_join(th[w], &ret);
        if (ret) bad = 1;
    }
    return bad ? -1 : 0;
}

static int job_setup(reg_job *jb, const float *src, int32_t n, const float *tgt, int32_t m,
                     const float *rots, int32_t k, const int32_t *which, int32_t count,
                     float eps, float delta, float tau, int32_t metric, float lp, double mu,
                     int32_t lib_zbits, const double *field, int32_t res, const float *lo,
                     const float *h, const float *inv, int32_t df_lookup, double mu_df,
                     int32_t *k_lo, int32_t *size, const float *t_min, const float *t_max)
{
    if (n <= 0 || m <= 0 || k <= 0 || count < 0 || !(eps > 0.0f)) return -1;
    if (metric < ORC_TRUNC_L2 || metric > ORC_VOTES || !(lp > 0.0f && lp <= 1.0f)) return -1;
    if (!(mu >= 0.0 && mu < 0.5) || !(mu_df >= 0.0 && mu_df < 0.5)) return -1;
    if (df_lookup != ORC_DF_NEAREST && df_lookup != ORC_DF_TRILINEAR) return -1;
    if (lib_zbits != 0 && lib_zbits != 15 && lib_zbits != 16) return -1;
    if (orc_box(delta, t_min, t_max, k_lo, size)) return -1;
    if (which)
        for (int32_t u = 0; u < count; ++u)
            if (which[u] < 0 || which[u] >= k) return -1;
    memset(jb, 0, sizeof(*jb));
    jb->src = src; jb->n = n; jb->tgt = tgt; jb->m = m; jb->rots = rots; jb->which = which;
    jb->delta = delta; jb->mu = mu; jb->k_lo = k_lo; jb->size = size; jb->metric = metric;
    jb->eps = eps; jb->tau = tau; jb->lp = lp; jb->lib_zbits = lib_zbits;
    jb->f = (df_view){field, res, eps > tau ? eps : tau, lo, h, inv, df_lookup, mu_df};
    return 0;
}

/*
 * Run Alg. 2 on the rotations listed in `which` (NULL: all k of them), writing one
 * record per listed rotation.  `field` != NULL selects distance-field scoring with
 * the grid from orc_df_build() (df_lookup: 0 nearest voxel, 1 trilinear).  mu and
 * mu_df are the fragility margins in bin and voxel units.  lib_zbits = 15 or 16 selects
 * the secondary library formulas (0: the definition).  Returns 0, or -1 on invalid
 * input or no memory.
 */
int orc_records(const float *src, int32_t n, const float *tgt, int32_t m, const float *rots,
                int32_t k, const int32_t *which, int32_t count, float eps, float delta, float tau,
                const float *t_min, const float *t_max, int32_t metric, float lp, double mu,
                int32_t lib_zbits, const double *field, int32_t res, const float *lo,
                const float *h, const float *inv, int32_t df_lookup, double mu_df,
                int32_t nthreads, orc_record *out)
{
    int32_t k_lo[3], size[3];
    reg_job jb;
    if (job_setup(&jb, src, n, tgt, m, rots, k, which, count, eps, delta, tau, metric, lp, mu,
                  lib_zbits, field, res, lo, h, inv, df_lookup, mu_df, k_lo, size, t_min, t_max))
        return -1;
    if (!which) count = k;
    jb.out = out;
    return run_jobs(&jb, count, nthreads, reg_worker);
}

/* Score the candidates {R_which[u], delta * bins[u]} (no vote); one record each. */
int orc_score_bins(const float *src, int32_t n, const float *tgt, int32_t m, const float *rots,
                   int32_t k, const int32_t *which, const int32_t *bins, int32_t count,
                   float eps, float delta, float tau, int32_t metric, float lp, int32_t lib_zbits,
                   const double *field, int32_t res, const float *lo, const float *h,
                   const float *inv, int32_t df_lookup, double mu_df, int32_t nthreads,
                   orc_record *out)
{
    int32_t k_lo[3], size[3];
    const float wide_lo[3] = {-1.0f, -1.0f, -1.0f}, wide_hi[3] = {1.0f, 1.0f, 1.0f};
    reg_job jb;
    if (!which || !bins || metric == ORC_VOTES) return -1;
    if (job_setup(&jb, src, n, tgt, m, rots, k, which, count, eps, delta, tau, metric, lp, 0.0,
                  lib_zbits, field, res, lo, h, inv, df_lookup, mu_df, k_lo, size, wide_lo,
                  wide_hi))
        return -1;
    jb.bins = bins;
    jb.out = out;
    return run_jobs(&jb, count, nthreads, bins_worker);
}

/*
 * Final step of Alg. 2: the candidate minimising the error.  Ties (the paper is
 * silent) go to more inliers, then the lower rotation index.  Returns the index
 * into `recs`, or -1 when no candidate is valid.
 */
int32_t orc_select(const orc_record *recs, int32_t count)
{
    int32_t best = -1;
    for (int32_t u = 0; u < count; ++u) {
        if (!recs[u].valid) continue;
        if (best < 0 || recs[u].error < recs[best].error ||
            (recs[u].error == recs[best].error && recs[u].inliers > recs[best].inliers))
            best = u;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1, the pure exhaustive search: every rotation of the list with every  */
/* lattice translation b delta of the box, each scored as in Alg. 2's error   */
/* loop (sum over the source, brute-force nearest reference point).  Writes   */
/* per rotation the best translation (smaller error, then more inliers, then  */
/* the lower linear index of b, x slowest); `votes` is 1 (Alg. 1 has no vote) */
/* and `valid` 1.  The best pose overall is orc_select() over these records.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *src; int32_t n; const float *tgt; int32_t m; const float *rots;
    float delta; const int32_t *k_lo; const int32_t *size;
    int metric; double eps, tau, lp;
    orc_record *out; int32_t begin, end;
} exh_job;

static void *exh_worker(void *arg)
{
    exh_job *jb = (exh_job *)arg;
    for (int32_t k = jb->begin; k < jb->end; ++k) {
        const float *R = jb->rots + 9 * (size_t)k;
        orc_record best;
        memset(&best, 0, sizeof(best));
        best.error = INFINITY;
        int have = 0;
        for (int32_t a = 0; a < jb->size[0]; ++a)
            for (int32_t b = 0; b < jb->size[1]; ++b)
                for (int32_t c = 0; c < jb->size[2]; ++c) {
                    const int32_t bin[3] = {jb->k_lo[0] + a, jb->k_lo[1] + b, jb->k_lo[2] + c};
                    double t[3];
                    for (int ax = 0; ax < 3; ++ax) t[ax] = (double)bin[ax] * (double)jb->delta;
                    orc_record r;
                    memset(&r, 0, sizeof(r));
                    score_candidate(jb->src, jb->n, jb->tgt, jb->m, R, t, jb->metric, jb->eps,
                                    jb->tau, jb->lp, &r);
                    /* lexicographic order: the first strictly better one wins, so ties
                       keep the lower linear index */
                    if (!have || r.error < best.error ||
                        (r.error == best.error && r.inliers > best.inliers)) {
                        best = r;
                        for (int ax = 0; ax < 3; ++ax) best.bin[ax] = bin[ax];
                        have = 1;
                    }
                }
        best.votes = best.votes_lo = best.votes_hi = best.lo_max = 1;
        best.valid = 1;
        best.pinned = 1;
        best.rot = k;
        jb->out[k] = best;
    }
    return NULL;
}

int orc_exhaustive(const float *src, int32_t n, const float *tgt, int32_t m, const float *rots,
                   int32_t k, float eps, float delta, float tau, const float *t_min,
                   const float *t_max, int32_t metric, float lp, int32_t nthreads,
                   orc_record *out)
{
    int32_t k_lo[3], size[3];
    if (n <= 0 || m <= 0 || k <= 0 || !(eps > 0.0f)) return -1;
    if (metric < ORC_TRUNC_L2 || metric > ORC_TRUNC_LP || !(lp > 0.0f && lp <= 1.0f)) return -1;
    if (orc_box(delta, t_min, t_max, k_lo, size)) return -1;
    int nt = n_threads(nthreads);
    if (nt > 256) nt = 256;
    if (nt > k) nt = k;
    pthread_t th[256];
    exh_job jobs[256];
    for (int w = 0; w < nt; ++w) {
        jobs[w] = (exh_job){src, n, tgt, m, rots, delta, k_lo, size, metric, (double)eps,
                            (double)tau, (double)lp, out, (int32_t)((int64_t)k * w / nt),
                            (int32_t)((int64_t)k * (w + 1) / nt)};
        pthread_create(&th[w], NULL, exh_worker, &jobs[w]);
    }
    for (int w = 0; w < nt; ++w) pthread_join(th[w], NULL);
    return 0;
}
