/*
 * moco oracle: a plain, slow FP64 CPU brute force of the translation search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or constant with the HIP
 * path.
 *
 * Everything is written from the paper's definitions (Dubbs, Guevara,
 * Peterka, Yuste, "moco: Fast Motion Correction for Calcium Imaging",
 * arXiv:1506.06039), section 2 "Mathematical Development", with 0-based
 * indices:
 *
 *   - the objective f_{s,t}: the sum over the overlap set D_{s,t} of
 *     (a[i+s][j+t] - b[i][j])^2, divided by Area(D_{s,t})            (sec. 2, objective)
 *   - D_{s,t}: the pairs (i,j) for which both (i,j) and (i+s,j+t) lie
 *     inside the m x n image                                          (sec. 2, overlap set)
 *   - the search over every (s,t) with max(|s|,|t|) < w, the argmin,
 *     then the x2 upsampling step that evaluates f at (2s+u, 2t+v),
 *     u,v in {-1,0,1}, on the finer grid and keeps the minimum, once per
 *     level of downsampling                                           (sec. 2, last paragraph)
 *   - "downsampled": a 2x2 box mean (the paper names no filter; this is
 *     the reading used throughout), odd trailing row/column dropped.
 *
 * No blocking, no fusion, no reordering: every f value is one FP64
 * accumulator, i outer and j inner, divided last.
 *
 * Tie order of the argmin (the paper is silent): the lexicographic minimum of
 * (f, max(|s|,|t|), |s|+|t|, s, t); f is compared exactly in FP64, and a NaN
 * f is ordered as +infinity.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int imax(int x, int y) { return x > y ? x : y; }
static int iabs(int x) { return x < 0 ? -x : x; }

/* 2x2 box mean, floor(m/2) x floor(n/2); row-major in and out. */
void oracle_downsample(const double *x, int m, int n, double *y)
{
    int mc = m / 2, nc = n / 2;
    for (int i = 0; i < mc; ++i)
        for (int j = 0; j < nc; ++j) {
            double s = x[(size_t)(2 * i) * n + 2 * j] + x[(size_t)(2 * i) * n + 2 * j + 1] +
                       x[(size_t)(2 * i + 1) * n + 2 * j] + x[(size_t)(2 * i + 1) * n + 2 * j + 1];
            y[(size_t)i * nc + j] = s / 4.0;
        }
}

/* Area(D_{s,t}) by its definition: the count of i in [0,m) with i+s in
 * [0,m), times the same count for j. */
double oracle_area(int m, int n, int s, int t)
{
    int ci = 0, cj = 0;
    for (int i = 0; i < m; ++i)
        if (i + s >= 0 && i + s < m) ++ci;
    for (int j = 0; j < n; ++j)
        if (j + t >= 0 && j + t < n) ++cj;
    return (double)ci * (double)cj;
}

/* f_{s,t} straight from the objective: one accumulator, divide last.
 * Returns NaN when D_{s,t} is empty. */
double oracle_f(const double *a, const double *b, int m, int n, int s, int t)
{
    double acc = 0.0;
    double area = 0.0;
    for (int i = 0; i < m; ++i) {
        if (i + s < 0 || i + s >= m) continue;
        for (int j = 0; j < n; ++j) {
            if (j + t < 0 || j + t >= n) continue;
            double d = a[(size_t)(i + s) * n + (j + t)] - b[(size_t)i * n + j];
            acc += d * d;
            area += 1.0;
        }
    }
    return acc / area;
}

/* The three sums of the energy split at one shift, each by its own plain
 * definition over D_{s,t}: out = { sum a^2, sum b^2, sum a*b, Area }.
 * Used by tests to pin the identity Area*f = A + B - 2h and the per-stage
 * quantities of the GPU path. */
void oracle_terms(const double *a, const double *b, int m, int n, int s, int t, double out[4])
{
    double ea = 0.0, eb = 0.0, h = 0.0, area = 0.0;
    for (int i = 0; i < m; ++i) {
        if (i + s < 0 || i + s >= m) continue;
        for (int j = 0; j < n; ++j) {
            if (j + t < 0 || j + t >= n) continue;
            double av = a[(size_t)(i + s) * n + (j + t)];
            double bv = b[(size_t)i * n + j];
            ea += av * av;
            eb += bv * bv;
            h += av * bv;
            area += 1.0;
        }
    }
    out[0] = ea;
    out[1] = eb;
    out[2] = h;
    out[3] = area;
}

/* Every f_{s,t} with max(|s|,|t|) < w, written as surf[(s+w-1)*(2w-1) + (t+w-1)]. */
void oracle_surface(const double *a, const double *b, int m, int n, int w, double *surf)
{
    int W = 2 * w - 1;
    for (int s = -(w - 1); s <= w - 1; ++s)
        for (int t = -(w - 1); t <= w - 1; ++t)
            surf[(size_t)(s + w - 1) * W + (t + w - 1)] = oracle_f(a, b, m, n, s, t);
}

/* Strict "better" relation of the tie order: returns 1 when (f1,s1,t1)
 * precedes (f2,s2,t2). */
static int precedes(double f1, int s1, int t1, double f2, int s2, int t2)
{
    double g1 = isnan(f1) ? INFINITY : f1;
    double g2 = isnan(f2) ? INFINITY : f2;
    if (g1 != g2) return g1 < g2;
    int r1 = imax(iabs(s1), iabs(t1)), r2 = imax(iabs(s2), iabs(t2));
    if (r1 != r2) return r1 < r2;
    int l1 = iabs(s1) + iabs(t1), l2 = iabs(s2) + iabs(t2);
    if (l1 != l2) return l1 < l2;
    if (s1 != s2) return s1 < s2;
    return t1 < t2;
}

/* Result record of one frame. */
typedef struct {
    int32_t coarse_s, coarse_t; /* argmin on the searched grid            */
    int32_t shift_s, shift_t;   /* final shift (after the refine if ds)   */
    double fmin;                /* f at the coarse argmin                 */
    double gap_c;               /* second-best minus best, coarse surface */
    double frefine[9];          /* f at (2s*+u, 2t*+v), [u+1][v+1]        */
    double gap_r;               /* second-best minus best of the nine     */
    double kappa;               /* (A+B)/(Area*fmin) at the coarse argmin */
} oracle_result;

/* Best and second-best of the nine f at (2s+u, 2t+v), u,v in {-1,0,1}, on one
 * level's images (m x n); f9 (may be NULL) receives the nine values. */
static void nine(const double *a, const double *b, int m, int n, int s0, int t0, double *f9,
                 int *bs, int *bt, double *best, double *second)
{
    double rb = NAN, rsec = INFINITY;
    int rs = 0, rt = 0, rhave = 0;
    for (int u = -1; u <= 1; ++u)
        for (int v = -1; v <= 1; ++v) {
            int s = 2 * s0 + u, t = 2 * t0 + v;
            double f = oracle_f(a, b, m, n, s, t);
            if (f9) f9[(u + 1) * 3 + (v + 1)] = f;
            if (!rhave || precedes(f, s, t, rb, rs, rt)) {
                if (rhave) {
                    double g = isnan(rb) ? INFINITY : rb;
                    if (g < rsec) rsec = g;
                }
                rb = f;
                rs = s;
                rt = t;
                rhave = 1;
            } else {
                double g = isnan(f) ? INFINITY : f;
                if (g < rsec) rsec = g;
            }
        }
    *bs = rs;
    *bt = rt;
    *best = rb;
    *second = rsec;
}

/* Align one frame a against template b (both m x n, FP64).  surf may be NULL.
 * Follows the search of section 2: downsample both `levels` times (0: not at
 * all), score every shift of the window on the coarsest images, take the
 * argmin, then at each finer level multiply it by two and keep the best of
 * the nine evaluations around it, down to full resolution.  pa, pb: room for
 * the downsampled images of every level (m*n/2 each suffices). */
static void align_one(const double *a, const double *b, int m, int n, int w, int levels,
                      double *pa, double *pb, double *surf, oracle_result *r)
{
    /* the image pyramid: level 0 is the frame itself */
    const double *la[8], *lb[8];
    int lm[8], ln[8];
    la[0] = a;
    lb[0] = b;
    lm[0] = m;
    ln[0] = n;
    size_t off = 0;
    for (int l = 1; l <= levels; ++l) {
        oracle_downsample(la[l - 1], lm[l - 1], ln[l - 1], pa + off);
        oracle_downsample(lb[l - 1], lm[l - 1], ln[l - 1], pb + off);
        la[l] = pa + off;
        lb[l] = pb + off;
        lm[l] = lm[l - 1] / 2;
        ln[l] = ln[l - 1] / 2;
        off += (size_t)lm[l] * ln[l];
    }
    const double *ga = la[levels], *gb = lb[levels];
    const int mg = lm[levels], ng = ln[levels];
    int W = 2 * w - 1;
    double best = NAN, second = INFINITY;
    int bs = 0, bt = 0, have = 0;
    for (int s = -(w - 1); s <= w - 1; ++s)
        for (int t = -(w - 1); t <= w - 1; ++t) {
            double f = oracle_f(ga, gb, mg, ng, s, t);
            if (surf) surf[(size_t)(s + w - 1) * W + (t + w - 1)] = f;
            if (!have || precedes(f, s, t, best, bs, bt)) {
                if (have) {
                    double gb_ = isnan(best) ? INFINITY : best;
                    if (gb_ < second) second = gb_;
                }
                best = f;
                bs = s;
                bt = t;
                have = 1;
            } else {
                double gf = isnan(f) ? INFINITY : f;
                if (gf < second) second = gf;
            }
        }
    r->coarse_s = bs;
    r->coarse_t = bt;
    r->fmin = best;
    r->gap_c = (W * W > 1) ? second - best : INFINITY;
    {
        double q[4];
        oracle_terms(ga, gb, mg, ng, bs, bt, q);
        r->kappa = (q[0] + q[1]) / (q[3] * best);
    }
    if (levels == 0) {
        r->shift_s = bs;
        r->shift_t = bt;
        for (int k = 0; k < 9; ++k) r->frefine[k] = NAN;
        r->gap_r = INFINITY;
        return;
    }
    int s = bs, t = bt;
    double rb = NAN, rsec = INFINITY;
    for (int l = levels - 1; l >= 0; --l)
        nine(la[l], lb[l], lm[l], ln[l], s, t, l == 0 ? r->frefine : NULL, &s, &t, &rb, &rsec);
    r->shift_s = s;
    r->shift_t = t;
    r->gap_r = rsec - rb;
}

/* Validation with the same rules as the library's boundary.  Returns 0 when
 * the arguments describe a valid search, -1 otherwise. */
int oracle_validate(int T, int m, int n, int w, int ds)
{
    if (T < 0 || m < 1 || n < 1 || w < 1) return -1;
    if (ds < 0 || ds > 4) return -1;
    int mg = m >> ds, ng = n >> ds;
    if (mg < 1 || ng < 1) return -1;
    if (w > mg || w > ng) return -1;
    return 0;
}

/* Align T frames (T x m x n, FP64) against one template (m x n, FP64).
 * Each output array holds T records (surf: T x (2w-1)^2, may be NULL).
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad input. */
int oracle_align(const double *frames, const double *tmpl, int T, int m, int n, int w, int ds,
                 int32_t *coarse, int32_t *shift, double *fmin, double *gap_c, double *frefine,
                 double *gap_r, double *kappa, double *surf, int nthreads)
{
    if (oracle_validate(T, m, n, w, ds) != 0) return -1;
    int W = 2 * w - 1;
    size_t mn = (size_t)m * n;
    size_t cn = mn / 2 + 1;   /* every downsampled level: m n (1/4 + 1/16 + ...) < m n / 3 */
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int failed = 0;
#pragma omp parallel
    {
        double *sa = (double *)malloc(cn * sizeof(double));
        double *sb = (double *)malloc(cn * sizeof(double));
        if (!sa || !sb) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int k = 0; k < T; ++k) {
            if (failed) continue;
            oracle_result r;
            align_one(frames + (size_t)k * mn, tmpl, m, n, w, ds, sa, sb,
                      surf ? surf + (size_t)k * W * W : NULL, &r);
            coarse[2 * k] = r.coarse_s;
            coarse[2 * k + 1] = r.coarse_t;
            shift[2 * k] = r.shift_s;
            shift[2 * k + 1] = r.shift_t;
            fmin[k] = r.fmin;
            gap_c[k] = r.gap_c;
            memcpy(frefine + 9 * (size_t)k, r.frefine, sizeof r.frefine);
            gap_r[k] = r.gap_r;
            kappa[k] = r.kappa;
        }
        free(sa);
        free(sb);
    }
    return failed ? -1 : 0;
}

/* The corrected stack and its mean image (sec. 2: every frame moved by its
 * translation is the motion-corrected video; sec. 3: the mean of the
 * corrected video, where each frame is black outside the overlap with the
 * template).  For frame k with shift (S,T): out[k][i][j] = a_k[i+S][j+T] when
 * 0 <= i+S < m and 0 <= j+T < n, else 0.  mean[i][j] = (sum over k in order of
 * out[k][i][j]) / T_frames.  out and mean may each be NULL. */
void oracle_apply(const double *frames, const int32_t *shifts, int T, int m, int n, double *out,
                  double *mean)
{
    const size_t plane = (size_t)m * n;
    if (mean)
        for (size_t p = 0; p < plane; ++p) mean[p] = 0.0;
    for (int k = 0; k < T; ++k) {
        const double *a = frames + (size_t)k * plane;
        const int S = shifts[2 * k], Tt = shifts[2 * k + 1];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) {
                const long long r = (long long)i + S, c = (long long)j + Tt;
                const double v = (r >= 0 && r < m && c >= 0 && c < n) ? a[r * n + c] : 0.0;
                if (out) out[(size_t)k * plane + (size_t)i * n + j] = v;
                if (mean) mean[(size_t)i * n + j] += v;
            }
    }
    if (mean && T > 0)
        for (size_t p = 0; p < plane; ++p) mean[p] /= (double)T;
}

/* Number of OpenMP threads a parallel region would use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
