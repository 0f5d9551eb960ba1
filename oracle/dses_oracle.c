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
 * Precision.  All geometry that produces a real-valued result (rotated points,
 * nearest-neighbour distances, errors, distance-field values) is computed in
 * IEEE double.  Two steps turn floating point into an integer: the translation
 * bin of a point pair (ROUND in Alg. 2) and the voxel a query falls in for
 * distance-field scoring.  The paper fixes no precision for them, so both take
 * the decision in the kernel's precision, IEEE single, by the formulas written
 * out in bin_of_pair() and df_voxel_of() (the same formulas the library's
 * header documents).  Counts, modes and voxel indices are then exact integers.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -pthread -lm
 * (-ffp-contract=off keeps the single-precision steps exactly as written).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

enum { ORC_TRUNC_L2 = 0, ORC_INLIERS = 1, ORC_TLS = 2, ORC_TRUNC_L1 = 3, ORC_TRUNC_LP = 4,
       ORC_VOTES = 5 };

/* Per-rotation outcome of Alg. 2, one row of the candidate list. */
typedef struct {
    int32_t bin[3];     /* mode bin b* (t* = delta * b*), lattice units            */
    uint32_t votes;     /* M: vote count of the mode bin                           */
    int32_t inliers;    /* #{i : d_i < eps}                                        */
    int32_t boundary;   /* #{i : |d_i - eps| <= 1e-6}, reported, not compared      */
    double error;       /* e(R, t*) under the chosen metric                        */
    int32_t valid;      /* 0 when no pair voted inside the translation box         */
    int32_t pad;
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

/* ------------------------------------------------------------------------ */
/* ROUND(y_j - R x_i, delta) of Alg. 2, taken in single precision:          */
/*   s      = 1/delta                                   (float division)     */
/*   p_a    = fma(R_a2, x_z, fma(R_a1, x_y, R_a0 * x_x)) (float)             */
/*   Y_a    = (y_a * s) + (0.5 - k_lo_a)                (two float roundings)*/
/*   P_a    = p_a * s                                   (float)              */
/*   c_a    = floor(Y_a - P_a)                          (float subtract)     */
/* so c_a = floor((y_a - p_a)/delta + 1/2) - k_lo_a, the box-relative index   */
/* of the nearest lattice point.  The pair votes iff 0 <= c_a < size_a.      */
/* ------------------------------------------------------------------------ */
static void rotate_f32(const float *R, const float *x, float *p)
{
    for (int a = 0; a < 3; ++a) {
        float acc = R[3 * a + 0] * x[0];
        acc = fmaf(R[3 * a + 1], x[1], acc);
        acc = fmaf(R[3 * a + 2], x[2], acc);
        p[a] = acc;
    }
}

static int bin_of_pair(const float *y, const float *p, float s, const int32_t *k_lo,
                       const int32_t *size, int32_t *c)
{
    int inside = 1;
    for (int a = 0; a < 3; ++a) {
        float ofs = 0.5f - (float)k_lo[a];
        float Y = y[a] * s;
        Y = Y + ofs;
        float P = p[a] * s;
        float u = Y - P;
        c[a] = (int32_t)floorf(u);
        if (c[a] < 0 || c[a] >= size[a]) inside = 0;
    }
    return inside;
}

/* ------------------------------------------------------------------------ */
/* Lemma 2 / Alg. 2 first loop: for one rotation, count every rotated pair   */
/* translation into the dense vote array over the box and take its mode.    */
/* Mode tie-break (the paper is silent): the lowest linear index, x slowest. */
/* Returns the mode count M (0 if no pair voted).                            */
/* ------------------------------------------------------------------------ */
uint32_t orc_vote(const float *src, int32_t n, const float *tgt, int32_t m, const float *R,
                  float delta, const int32_t *k_lo, const int32_t *size, uint32_t *hist,
                  int32_t *mode_bin)
{
    const size_t nbins = (size_t)size[0] * size[1] * size[2];
    const float s = 1.0f / delta;
    memset(hist, 0, nbins * sizeof(uint32_t));
    for (int32_t i = 0; i < n; ++i) {
        float p[3];
        rotate_f32(R, src + 3 * i, p);
        for (int32_t j = 0; j < m; ++j) {
            int32_t c[3];
            if (bin_of_pair(tgt + 3 * j, p, s, k_lo, size, c))
                hist[((size_t)c[0] * size[1] + c[1]) * size[2] + c[2]] += 1;
        }
    }
    uint32_t best = 0;
    size_t arg = 0;
    for (size_t l = 0; l < nbins; ++l)
        if (hist[l] > best) { best = hist[l]; arg = l; }
    mode_bin[2] = (int32_t)(arg % size[2]) + k_lo[2];
    mode_bin[1] = (int32_t)((arg / size[2]) % size[1]) + k_lo[1];
    mode_bin[0] = (int32_t)(arg / ((size_t)size[1] * size[2])) + k_lo[0];
    return best;
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
/* exponent of the truncated Lp objective (p < 1: the sparsity norms the paper */
/* admits as "any desired norm").                                             */
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
        const float *x = src + 3 * i;
        double q[3];
        for (int a = 0; a < 3; ++a)
            q[a] = (double)R[3 * a] * x[0] + (double)R[3 * a + 1] * x[1] +
                   (double)R[3 * a + 2] * x[2] + t[a];
        double d2 = nn_dist(q, tgt, m, 0);
        double d = metric == ORC_TRUNC_L1 ? nn_dist(q, tgt, m, 1) : d2;
        if (d2 < eps) ++inl;
        if (fabs(d2 - eps) <= 1e-6) ++bnd;
        err += rho(metric, d, tau, eps, lp);
    }
    rec->inliers = inl;
    rec->boundary = bnd;
    rec->error = err;
}

/* ------------------------------------------------------------------------ */
/* Voxel distance field of the reference (one per target): a res^3 grid over */
/* the reference bounding box padded by r = max(tau, eps), voxel centres     */
/*   c_a = lo_a + (idx_a + 1/2) h_a,                                          */
/* value D = min(min_j ||c - y_j||, r) in double.  The box parameters are     */
/* single precision so that both sides share them bit for bit:              */
/*   lo_a = min_j y_a - r,  hi_a = max_j y_a + r,  h_a = (hi_a - lo_a)/res,   */
/*   inv_a = 1/h_a                                         (float arithmetic) */
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

/* Voxel of a single-precision query: idx_a = floor((q_a - lo_a) * inv_a).  */
static int df_voxel_of(const float *q, const float *lo, const float *inv, int32_t res,
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

/* Distance-field scoring of one candidate: the query q = R x + t is formed in */
/* single precision (the same rotate_f32 chain, then + t), its voxel decided  */
/* by df_voxel_of(); outside the grid the distance exceeds r, so D = r.       */
static void score_candidate_df(const float *src, int32_t n, const float *R, const float *tf,
                               int metric, double eps, double tau, double lp, float r,
                               int32_t res, const float *lo, const float *inv,
                               const double *field, orc_record *rec)
{
    double err = 0.0;
    int32_t inl = 0, bnd = 0;
    for (int32_t i = 0; i < n; ++i) {
        float p[3], q[3];
        int32_t idx[3];
        rotate_f32(R, src + 3 * i, p);
        for (int a = 0; a < 3; ++a) q[a] = p[a] + tf[a];
        double D = df_voxel_of(q, lo, inv, res, idx)
                       ? field[((size_t)idx[0] * res + idx[1]) * res + idx[2]]
                       : (double)r;
        if (D < eps) ++inl;
        if (fabs(D - eps) <= 1e-6) ++bnd;
        err += rho(metric, D, tau, eps, lp);
    }
    rec->inliers = inl;
    rec->boundary = bnd;
    rec->error = err;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 over a list of rotations (q = 0: every candidate is scored).       */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *src; int32_t n; const float *tgt; int32_t m;
    const float *rots; const int32_t *which; int32_t count;
    float delta; const int32_t *k_lo; const int32_t *size;
    int metric; double eps, tau, lp;
    /* distance-field mode (field == NULL: brute force) */
    const double *field; float r; int32_t res; const float *lo; const float *inv;
    orc_record *out;
    int32_t begin, end;
} reg_job;

static void *reg_worker(void *arg)
{
    reg_job *jb = (reg_job *)arg;
    const size_t nbins = (size_t)jb->size[0] * jb->size[1] * jb->size[2];
    uint32_t *hist = (uint32_t *)malloc(nbins * sizeof(uint32_t));
    if (!hist) return (void *)1;
    for (int32_t u = jb->begin; u < jb->end; ++u) {
        int32_t k = jb->which ? jb->which[u] : u;
        const float *R = jb->rots + 9 * (size_t)k;
        orc_record *rec = &jb->out[u];
        memset(rec, 0, sizeof(*rec));
        rec->votes = orc_vote(jb->src, jb->n, jb->tgt, jb->m, R, jb->delta, jb->k_lo, jb->size,
                              hist, rec->bin);
        rec->valid = rec->votes > 0;
        if (!rec->valid) { rec->error = INFINITY; continue; }
        if (jb->metric == ORC_VOTES) {
            /* Thm. 3 ranking: no scoring, the mode count stands for the L0^{m1}
             * inlier count and the error is 0 for every valid candidate */
            rec->inliers = (int32_t)rec->votes;
            rec->error = 0.0;
            continue;
        }
        if (jb->field) {
            float tf[3];
            for (int a = 0; a < 3; ++a) tf[a] = (float)rec->bin[a] * jb->delta;
            score_candidate_df(jb->src, jb->n, R, tf, jb->metric, jb->eps, jb->tau, jb->lp, jb->r,
                               jb->res, jb->lo, jb->inv, jb->field, rec);
        } else {
            double t[3];
            for (int a = 0; a < 3; ++a) t[a] = (double)rec->bin[a] * (double)jb->delta;
            score_candidate(jb->src, jb->n, jb->tgt, jb->m, R, t, jb->metric, jb->eps, jb->tau,
                            jb->lp, rec);
        }
    }
    free(hist);
    return NULL;
}

/*
 * Run Alg. 2 on the rotations listed in `which` (NULL: all k of them), writing one
 * record per listed rotation.  `field` != NULL selects distance-field scoring with
 * the grid from orc_df_build().  Returns 0, or -1 on invalid input / no memory.
 */
int orc_records(const float *src, int32_t n, const float *tgt, int32_t m, const float *rots,
                int32_t k, const int32_t *which, int32_t count, float eps, float delta, float tau,
                const float *t_min, const float *t_max, int32_t metric, float lp,
                const double *field, int32_t res, const float *lo, const float *inv,
                int32_t nthreads, orc_record *out)
{
    int32_t k_lo[3], size[3];
    if (n <= 0 || m <= 0 || k <= 0 || count < 0 || !(eps > 0.0f)) return -1;
    if (metric < ORC_TRUNC_L2 || metric > ORC_VOTES || !(lp > 0.0f && lp <= 1.0f)) return -1;
    if (orc_box(delta, t_min, t_max, k_lo, size)) return -1;
    if (which)
        for (int32_t u = 0; u < count; ++u)
            if (which[u] < 0 || which[u] >= k) return -1;
    if (!which) count = k;
    int nt = n_threads(nthreads);
    if (nt > 256) nt = 256;
    if (nt > count) nt = count > 0 ? count : 1;
    pthread_t th[256];
    reg_job jobs[256];
    float r = eps > tau ? eps : tau;
    for (int w = 0; w < nt; ++w) {
        jobs[w] = (reg_job){src, n, tgt, m, rots, which, count, delta, k_lo, size, metric,
                            (double)eps, (double)tau, (double)lp, field, r, res, lo, inv, out,
                            (int32_t)((int64_t)count * w / nt),
                            (int32_t)((int64_t)count * (w + 1) / nt)};
        pthread_create(&th[w], NULL, reg_worker, &jobs[w]);
    }
    int bad = 0;
    for (int w = 0; w < nt; ++w) {
        void *ret = NULL;
        pthread_join(th[w], &ret);
        if (ret) bad = 1;
    }
    return bad ? -1 : 0;
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
        best.votes = 1;
        best.valid = 1;
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
