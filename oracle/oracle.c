/*
 * Skeleton oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Every function is the plain definition of a skeleton from Section III of the
 * paper (map, reduce, scan derived from higher-order functions; mapoverlap as a
 * neighbourhood map), written out with no blocking, fusion or reordering.
 * Floating point: binary64 from the stored binary32 values, sequential sums in
 * index order.  Integers: unsigned modular arithmetic of the output width.
 *
 * Built with gcc -O2 -ffp-contract=off (no fast-math): no FMA contraction, no
 * reassociation, IEEE round-to-nearest-even throughout.
 */
#include "oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 1;

void oracle_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int oracle_get_threads(void) { return g_threads; }

/* ---------------------------------------------------------------- Map ---- */

/* The element function f(x, y; p0, p1) of a skeleton instance (Section III:
 * a skeleton is parameterised by a user function). */
static int elem_fn(int op, const double *p, int np, double x, double y,
                   double *res)
{
    switch (op) {
    case ORC_MAP_IDENTITY: *res = x; return 0;
    case ORC_MAP_AXPY:
        if (np < 1) return -1;
        *res = p[0] * x + y; return 0;
    case ORC_MAP_AFFINE:
        if (np < 2) return -1;
        *res = p[0] * x + p[1]; return 0;
    case ORC_MAP_TANH: *res = tanh(x); return 0;
    case ORC_MAP_AFFINE_TANH:
        if (np < 2) return -1;
        *res = tanh(p[0] * x + p[1]); return 0;
    case ORC_MAP_MUL: *res = x * y; return 0;
    case ORC_MAP_SQUARE: *res = x * x; return 0;
    default: return -1;
    }
}

static int needs_y(int op) { return op == ORC_MAP_AXPY || op == ORC_MAP_MUL; }

/* map: out[i] = f(x[i], y[i]) for every i (Section III, "map") */
int oracle_map_f32(int op, const double *params, int nparams, const float *x,
                   const float *y, int64_t n, double *out)
{
    double probe;
    if (elem_fn(op, params, nparams, 0.0, 0.0, &probe) != 0) return -1;
    if (needs_y(op) && y == NULL) return -1;
    if (n <= 0) return 0;
    int64_t i;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (i = 0; i < n; ++i) {
        double yi = y ? (double)y[i] : 0.0;
        elem_fn(op, params, nparams, (double)x[i], yi, &out[i]);
    }
    return 0;
}

/* ------------------------------------------------------------- Reduce ---- */

/* reduce: x[0] op x[1] op ... op x[n-1] (Section III, "reduce"), sequential */
double oracle_reduce_f32(int op, const float *x, int64_t n)
{
    double acc;
    if (op == ORC_MIN) acc = INFINITY;
    else if (op == ORC_MAX) acc = -INFINITY;
    else acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double v = (double)x[i];
        if (op == ORC_MIN) acc = v < acc ? v : acc;
        else if (op == ORC_MAX) acc = v > acc ? v : acc;
        else acc = acc + v;
    }
    return acc;
}

int oracle_reduce_segments_f32(int op, const float *x, int64_t n, const int64_t *off,
                               int64_t nseg, double *out)
{
    for (int64_t s = 0; s < nseg; ++s)
        if (off[s] < 0 || off[s + 1] < off[s] || off[s + 1] > n) return -1;
    for (int64_t s = 0; s < nseg; ++s)
        out[s] = oracle_reduce_f32(op, x + off[s], off[s + 1] - off[s]);
    return 0;
}

/* ------------------------------------------------ exactly rounded sums ---- */

/* The exact sum is kept as a short list of non-overlapping binary64 partials,
 * ordered by increasing magnitude; adding a value replaces the list by the
 * exact two-term splits of the running sum against each partial. */
#define MSUM_CAP 128

typedef struct {
    double p[MSUM_CAP];
    int len;
    int bad; /* a non-finite input or a list overflow was seen */
} msum;

static void msum_add(msum *m, double x)
{
    if (!isfinite(x)) { m->bad = 1; return; }
    int i = 0;
    for (int j = 0; j < m->len; ++j) {
        double y = m->p[j];
        if (fabs(x) < fabs(y)) { double t = x; x = y; y = t; }
        double hi = x + y;
        double lo = y - (hi - x); /* exact: |y| <= |x| */
        if (lo != 0.0) m->p[i++] = lo;
        x = hi;
    }
    if (i >= MSUM_CAP) { m->bad = 1; return; }
    m->p[i++] = x;
    m->len = i;
}

/* round the exact value sum(p) once to binary64 */
static double msum_round(const msum *m)
{
    if (m->bad) return NAN;
    int n = m->len;
    if (n == 0) return 0.0;
    double hi = m->p[--n], lo = 0.0;
    while (n > 0) {
        double x = hi, y = m->p[--n];
        hi = x + y;
        lo = y - (hi - x);
        if (lo != 0.0) break;
    }
    /* hi + lo is the sum of the top partials; if lo is exactly half an ulp of
     * hi and the remaining partials push the same way, round away from hi */
    if (n > 0 && ((lo < 0.0 && m->p[n - 1] < 0.0) || (lo > 0.0 && m->p[n - 1] > 0.0))) {
        double y = lo * 2.0;
        double x = hi + y;
        if (y == x - hi) hi = x;
    }
    return hi;
}

double oracle_fsum_f64(const double *x, int64_t n)
{
    msum m = {{0}, 0, 0};
    for (int64_t i = 0; i < n; ++i) msum_add(&m, x[i]);
    return msum_round(&m);
}

static double bf16_value(uint16_t h)
{
    uint32_t b = (uint32_t)h << 16;
    float f;
    memcpy(&f, &b, 4);
    return (double)f;
}

double oracle_sum_bf16_exact(const uint16_t *x, int64_t n)
{
    msum m = {{0}, 0, 0};
    for (int64_t i = 0; i < n; ++i) msum_add(&m, bf16_value(x[i]));
    return msum_round(&m);
}

double oracle_dot_bf16_exact(const uint16_t *x, const uint16_t *y, int64_t n)
{
    msum m = {{0}, 0, 0};
    for (int64_t i = 0; i < n; ++i) msum_add(&m, bf16_value(x[i]) * bf16_value(y[i]));
    return msum_round(&m);
}

double oracle_abs_sum_f32(const float *x, int64_t n)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc = acc + fabs((double)x[i]);
    return acc;
}

int32_t oracle_reduce_i32_i32(int op, const int32_t *x, int64_t n)
{
    if (op == ORC_SUM) {
        uint32_t acc = 0;
        for (int64_t i = 0; i < n; ++i) acc = acc + (uint32_t)x[i];
        return (int32_t)acc;
    }
    int32_t acc = op == ORC_MIN ? INT32_MAX : INT32_MIN;
    for (int64_t i = 0; i < n; ++i) {
        if (op == ORC_MIN) acc = x[i] < acc ? x[i] : acc;
        else acc = x[i] > acc ? x[i] : acc;
    }
    return acc;
}

int64_t oracle_reduce_i32_i64(int op, const int32_t *x, int64_t n)
{
    if (op == ORC_SUM) {
        uint64_t acc = 0;
        for (int64_t i = 0; i < n; ++i) acc = acc + (uint64_t)(int64_t)x[i];
        return (int64_t)acc;
    }
    int64_t acc = op == ORC_MIN ? INT64_MAX : INT64_MIN;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = x[i];
        if (op == ORC_MIN) acc = v < acc ? v : acc;
        else acc = v > acc ? v : acc;
    }
    return acc;
}

int64_t oracle_reduce_i64_i64(int op, const int64_t *x, int64_t n)
{
    if (op == ORC_SUM) {
        uint64_t acc = 0;
        for (int64_t i = 0; i < n; ++i) acc = acc + (uint64_t)x[i];
        return (int64_t)acc;
    }
    int64_t acc = op == ORC_MIN ? INT64_MAX : INT64_MIN;
    for (int64_t i = 0; i < n; ++i) {
        if (op == ORC_MIN) acc = x[i] < acc ? x[i] : acc;
        else acc = x[i] > acc ? x[i] : acc;
    }
    return acc;
}

/* ---------------------------------------------------------- MapReduce ---- */

/* map then reduce without a stored intermediate: op over i of f(x[i], y[i]) */
double oracle_mapreduce_f32(int map_op, const double *params, int nparams,
                            const float *x, const float *y, int64_t n,
                            int reduce_op, double *abs_sum)
{
    double acc, mag = 0.0, v;
    if (reduce_op == ORC_MIN) acc = INFINITY;
    else if (reduce_op == ORC_MAX) acc = -INFINITY;
    else acc = 0.0;
    if (needs_y(map_op) && y == NULL) return NAN;
    for (int64_t i = 0; i < n; ++i) {
        double yi = y ? (double)y[i] : 0.0;
        if (elem_fn(map_op, params, nparams, (double)x[i], yi, &v) != 0)
            return NAN;
        mag = mag + fabs(v);
        if (reduce_op == ORC_MIN) acc = v < acc ? v : acc;
        else if (reduce_op == ORC_MAX) acc = v > acc ? v : acc;
        else acc = acc + v;
    }
    if (abs_sum) *abs_sum = mag;
    return acc;
}

/* --------------------------------------------------------- MapOverlap ---- */

/* border rule: index j of a length-n axis.  Returns 1 and sets *k to the index
 * to read, or 0 when the element is the constant pad. */
static int border_index(int64_t j, int64_t n, int edge, int64_t *k)
{
    if (j >= 0 && j < n) { *k = j; return 1; }
    switch (edge) {
    case ORC_EDGE_CLAMP: *k = j < 0 ? 0 : n - 1; return 1;
    case ORC_EDGE_CYCLIC: {
        int64_t m = j % n;
        *k = m < 0 ? m + n : m;
        return 1;
    }
    default: return 0; /* ORC_EDGE_CONST */
    }
}

int oracle_mapoverlap1d_f32(const float *x, int64_t n, const float *w, int r,
                            int edge, float pad, double *out, double *mag)
{
    if (r < 0 || w == NULL) return -1;
    if (edge != ORC_EDGE_CLAMP && edge != ORC_EDGE_CONST &&
        edge != ORC_EDGE_CYCLIC)
        return -1;
    if (n <= 0) return 0;
    int64_t i;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (i = 0; i < n; ++i) {
        double acc = 0.0, m = 0.0;
        for (int k = 0; k <= 2 * r; ++k) {
            int64_t src;
            double v = border_index(i + k - r, n, edge, &src) ? (double)x[src]
                                                               : (double)pad;
            double t = (double)w[k] * v;
            acc = acc + t;
            m = m + fabs(t);
        }
        out[i] = acc;
        if (mag) mag[i] = m;
    }
    return 0;
}

/* W[a][b]: the given 2D weights, or the exact binary64 outer product of the
 * separable factors (a 24-bit by 24-bit product fits the 53-bit significand) */
static double weight2d(const float *w2d, const float *wy, const float *wx,
                       int rx, int a, int b)
{
    if (w2d) return (double)w2d[(int64_t)a * (2 * rx + 1) + b];
    return (double)wy[a] * (double)wx[b];
}

double oracle_mapoverlap2d_at_f32(const float *x, int64_t rows, int64_t cols,
                                  const float *w2d, const float *wy,
                                  const float *wx, int ry, int rx, int edge,
                                  float pad, int64_t i, int64_t j, double *mag)
{
    double acc = 0.0, m = 0.0;
    for (int a = 0; a <= 2 * ry; ++a) {
        for (int b = 0; b <= 2 * rx; ++b) {
            int64_t si, sj;
            int in_r = border_index(i + a - ry, rows, edge, &si);
            int in_c = border_index(j + b - rx, cols, edge, &sj);
            double v = (in_r && in_c) ? (double)x[si * cols + sj] : (double)pad;
            double t = weight2d(w2d, wy, wx, rx, a, b) * v;
            acc = acc + t;
            m = m + fabs(t);
        }
    }
    if (mag) *mag = m;
    return acc;
}

int oracle_mapoverlap2d_f32(const float *x, int64_t rows, int64_t cols,
                            const float *w2d, const float *wy, const float *wx,
                            int ry, int rx, int edge, float pad, double *out,
                            double *mag)
{
    if (ry < 0 || rx < 0) return -1;
    if (w2d == NULL && (wy == NULL || wx == NULL)) return -1;
    if (edge != ORC_EDGE_CLAMP && edge != ORC_EDGE_CONST &&
        edge != ORC_EDGE_CYCLIC)
        return -1;
    if (rows <= 0 || cols <= 0) return 0;
    int64_t i;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (i = 0; i < rows; ++i) {
        for (int64_t j = 0; j < cols; ++j) {
            double m;
            out[i * cols + j] = oracle_mapoverlap2d_at_f32(
                x, rows, cols, w2d, wy, wx, ry, rx, edge, pad, i, j, &m);
            if (mag) mag[i * cols + j] = m;
        }
    }
    return 0;
}

/* --------------------------------------------------------------- Scan ---- */

/* scan: running combination in index order (Section III, "scan").  The
 * exclusive form starts from the operator's identity. */
/* the reverse kinds visit the same indices from the end */
static int scan_kind_valid(int kind)
{
    return kind == ORC_INCLUSIVE || kind == ORC_EXCLUSIVE ||
           kind == ORC_REVERSE_INCLUSIVE || kind == ORC_REVERSE_EXCLUSIVE;
}
static int scan_excludes_self(int kind)
{
    return kind == ORC_EXCLUSIVE || kind == ORC_REVERSE_EXCLUSIVE;
}
static int64_t scan_index(int kind, int64_t t, int64_t n)
{
    return kind >= ORC_REVERSE_INCLUSIVE ? n - 1 - t : t;
}

#define ORC_SCAN_INT(NAME, TIN, TOUT, UACC, TMIN, TMAX)                       \
    int NAME(const TIN *x, int64_t n, int kind, int op, TOUT *out)             \
    {                                                                          \
        if (!scan_kind_valid(kind)) return -1;                                 \
        if (op != ORC_SUM && op != ORC_MIN && op != ORC_MAX) return -1;        \
        UACC sacc = 0;                                                         \
        TOUT macc = op == ORC_MIN ? TMAX : TMIN;                               \
        for (int64_t t = 0; t < n; ++t) {                                      \
            const int64_t i = scan_index(kind, t, n);                          \
            if (scan_excludes_self(kind))                                      \
                out[i] = op == ORC_SUM ? (TOUT)sacc : macc;                    \
            TOUT v = (TOUT)x[i];                                               \
            if (op == ORC_SUM) sacc = sacc + (UACC)v;                          \
            else if (op == ORC_MIN) macc = v < macc ? v : macc;                \
            else macc = v > macc ? v : macc;                                   \
            if (!scan_excludes_self(kind))                                     \
                out[i] = op == ORC_SUM ? (TOUT)sacc : macc;                    \
        }                                                                      \
        return 0;                                                              \
    }

ORC_SCAN_INT(oracle_scan_i32_i32, int32_t, int32_t, uint32_t, INT32_MIN,
             INT32_MAX)
ORC_SCAN_INT(oracle_scan_i32_i64, int32_t, int64_t, uint64_t, INT64_MIN,
             INT64_MAX)
ORC_SCAN_INT(oracle_scan_i64_i64, int64_t, int64_t, uint64_t, INT64_MIN,
             INT64_MAX)

int oracle_scan_f32(const float *x, int64_t n, int kind, int op, double *out,
                    double *mag)
{
    if (!scan_kind_valid(kind)) return -1;
    if (op != ORC_SUM && op != ORC_MIN && op != ORC_MAX) return -1;
    double acc = op == ORC_MIN ? INFINITY : (op == ORC_MAX ? -INFINITY : 0.0);
    double m = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        const int64_t i = scan_index(kind, t, n);
        if (scan_excludes_self(kind)) {
            out[i] = acc;
            if (mag) mag[i] = m;
        }
        double v = (double)x[i];
        if (op == ORC_SUM) acc = acc + v;
        else if (op == ORC_MIN) acc = v < acc ? v : acc;
        else acc = v > acc ? v : acc;
        m = m + fabs(v);
        if (!scan_excludes_self(kind)) {
            out[i] = acc;
            if (mag) mag[i] = m;
        }
    }
    return 0;
}

/* ------------------------------------------------------------ adjoints ---- */

/* partial derivatives of the element function at (x, y): df/dx, df/dy and
 * df/dp_k, from the definitions in elem_fn */
static void elem_partials(int op, const double *p, double x, double y, double *fx,
                          double *fy, double *fp0, double *fp1)
{
    *fx = 0.0; *fy = 0.0; *fp0 = 0.0; *fp1 = 0.0;
    switch (op) {
    case ORC_MAP_IDENTITY: *fx = 1.0; break;
    case ORC_MAP_AXPY: *fx = p[0]; *fy = 1.0; *fp0 = x; break;
    case ORC_MAP_AFFINE: *fx = p[0]; *fp0 = x; *fp1 = 1.0; break;
    case ORC_MAP_TANH: {
        double t = tanh(x);
        *fx = 1.0 - t * t;
        break;
    }
    case ORC_MAP_AFFINE_TANH: {
        double t = tanh(p[0] * x + p[1]);
        double d = 1.0 - t * t; /* tanh' at the pre-activation */
        *fx = p[0] * d;
        *fp0 = x * d;
        *fp1 = d;
        break;
    }
    case ORC_MAP_MUL: *fx = y; *fy = x; break;
    case ORC_MAP_SQUARE: *fx = 2.0 * x; break;
    default: break;
    }
}

int oracle_map_grad_f32(int op, const double *params, int nparams, const float *x,
                        const float *y, const float *g, int64_t n, double *dx,
                        double *dy, double *dparams, double *dparams_mag)
{
    double probe;
    if (elem_fn(op, params, nparams, 0.0, 0.0, &probe) != 0) return -1;
    if (needs_y(op) && (y == NULL || dy == NULL)) return -1;
    double s0 = 0.0, s1 = 0.0, m0 = 0.0, m1 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double fx, fy, fp0, fp1;
        double xi = (double)x[i], yi = y ? (double)y[i] : 0.0, gi = (double)g[i];
        elem_partials(op, params, xi, yi, &fx, &fy, &fp0, &fp1);
        dx[i] = gi * fx;
        if (needs_y(op)) dy[i] = gi * fy;
        s0 = s0 + gi * fp0;
        s1 = s1 + gi * fp1;
        m0 = m0 + fabs(gi * fp0);
        m1 = m1 + fabs(gi * fp1);
    }
    if (dparams) {
        if (nparams > 0) dparams[0] = s0;
        if (nparams > 1) dparams[1] = s1;
    }
    if (dparams_mag) {
        if (nparams > 0) dparams_mag[0] = m0;
        if (nparams > 1) dparams_mag[1] = m1;
    }
    return 0;
}

/* every forward term w[k] * x[e(i+k-r)] of out[i] sends w[k] * g[i] back to
 * the element it read */
int oracle_mapoverlap1d_adjoint_f32(const float *g, int64_t n, const float *w, int r,
                                    int edge, double *dx, double *mag)
{
    if (r < 0 || w == NULL) return -1;
    if (edge != ORC_EDGE_CLAMP && edge != ORC_EDGE_CONST &&
        edge != ORC_EDGE_CYCLIC)
        return -1;
    for (int64_t j = 0; j < n; ++j) {
        dx[j] = 0.0;
        if (mag) mag[j] = 0.0;
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k <= 2 * r; ++k) {
            int64_t src;
            if (!border_index(i + k - r, n, edge, &src)) continue; /* the pad */
            double t = (double)w[k] * (double)g[i];
            dx[src] = dx[src] + t;
            if (mag) mag[src] = mag[src] + fabs(t);
        }
    }
    return 0;
}

int oracle_mapoverlap2d_adjoint_f32(const float *g, int64_t rows, int64_t cols,
                                    const float *w2d, const float *wy,
                                    const float *wx, int ry, int rx, int edge,
                                    double *dx, double *mag)
{
    if (ry < 0 || rx < 0) return -1;
    if (w2d == NULL && (wy == NULL || wx == NULL)) return -1;
    if (edge != ORC_EDGE_CLAMP && edge != ORC_EDGE_CONST &&
        edge != ORC_EDGE_CYCLIC)
        return -1;
    for (int64_t s = 0; s < rows * cols; ++s) {
        dx[s] = 0.0;
        if (mag) mag[s] = 0.0;
    }
    for (int64_t i = 0; i < rows; ++i) {
        for (int64_t j = 0; j < cols; ++j) {
            for (int a = 0; a <= 2 * ry; ++a) {
                for (int b = 0; b <= 2 * rx; ++b) {
                    int64_t si, sj;
                    if (!border_index(i + a - ry, rows, edge, &si)) continue;
                    if (!border_index(j + b - rx, cols, edge, &sj)) continue;
                    double t = weight2d(w2d, wy, wx, rx, a, b) * (double)g[i * cols + j];
                    dx[si * cols + sj] = dx[si * cols + sj] + t;
                    if (mag) mag[si * cols + sj] = mag[si * cols + sj] + fabs(t);
                }
            }
        }
    }
    return 0;
}

/* -------------------------------------------------- call chain ---- */

/* The call chain Map -> MapOverlap 2D -> Reduce SUM (a composition of three
 * skeleton calls, Section V; each step as defined above, Section III), over
 * `fields` images of rows x cols stored back to back, each mapped with its own
 * borders:
 *     t = f(x)                       element by element, binary64
 *     s[f][i][j] = sum_ab W[a][b] * t[f][e(i+a-ry)][e(j+b-rx)]  (pad outside)
 *     loss = sum over f, i, j of s[f][i][j]          sequential, index order
 * No rounding between the steps.  *mag receives sum |W[a][b] * read value|
 * over every term, the magnitude the result's error is measured against. */
double oracle_chain_f32(int map_op, const double *params, int nparams, const float *x,
                        int64_t fields, int64_t rows, int64_t cols, const float *w2d,
                        const float *wy, const float *wx, int ry, int rx, int edge,
                        float pad, double *mag)
{
    double probe;
    if (elem_fn(map_op, params, nparams, 0.0, 0.0, &probe) != 0 || needs_y(map_op))
        return NAN;
    if (ry < 0 || rx < 0 || (w2d == NULL && (wy == NULL || wx == NULL))) return NAN;
    if (edge != ORC_EDGE_CLAMP && edge != ORC_EDGE_CONST && edge != ORC_EDGE_CYCLIC)
        return NAN;
    const int64_t img = rows * cols, n = fields * img;
    double *t = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!t) return NAN;
    for (int64_t i = 0; i < n; ++i)
        elem_fn(map_op, params, nparams, (double)x[i], 0.0, &t[i]);
    double loss = 0.0, m = 0.0;
    for (int64_t f = 0; f < fields; ++f) {
        const double *tf = t + f * img;
        for (int64_t i = 0; i < rows; ++i) {
            for (int64_t j = 0; j < cols; ++j) {
                double s = 0.0;
                for (int a = 0; a <= 2 * ry; ++a) {
                    for (int b = 0; b <= 2 * rx; ++b) {
                        int64_t si, sj;
                        int in_r = border_index(i + a - ry, rows, edge, &si);
                        int in_c = border_index(j + b - rx, cols, edge, &sj);
                        double v = (in_r && in_c) ? tf[si * cols + sj] : (double)pad;
                        double term = weight2d(w2d, wy, wx, rx, a, b) * v;
                        s = s + term;
                        m = m + fabs(term);
                    }
                }
                loss = loss + s;
            }
        }
    }
    free(t);
    if (mag) *mag = m;
    return loss;
}

/* Reverse mode through the same chain for the upstream gradient g1 of the
 * loss: the Reduce adjoint broadcasts g1 to every s; the MapOverlap adjoint
 * sends W[a][b] * g1 from every output back to the element its tap read
 * (nothing for pad reads); the Map adjoint multiplies by f's partials:
 *     dx[k] = gt[k] * df/dx(x[k]),   dparams[p] = sum_k gt[k] * df/dp_p(x[k]).
 * dx_mag[k] = |df/dx(x[k])| * sum |W[a][b] * g1| over the taps that reached k;
 * dparams_mag[p] the matching sums of absolute terms.  Any output pointer
 * but dx may be NULL. */
int oracle_chain_grad_f32(int map_op, const double *params, int nparams, const float *x,
                          int64_t fields, int64_t rows, int64_t cols, const float *w2d,
                          const float *wy, const float *wx, int ry, int rx, int edge,
                          double g1, double *dx, double *dx_mag, double *dparams,
                          double *dparams_mag)
{
    double probe;
    if (elem_fn(map_op, params, nparams, 0.0, 0.0, &probe) != 0 || needs_y(map_op))
        return -1;
    if (ry < 0 || rx < 0 || (w2d == NULL && (wy == NULL || wx == NULL))) return -1;
    if (edge != ORC_EDGE_CLAMP && edge != ORC_EDGE_CONST && edge != ORC_EDGE_CYCLIC)
        return -1;
    const int64_t img = rows * cols, n = fields * img;
    double *gt = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *gm = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!gt || !gm) {
        free(gt);
        free(gm);
        return -1;
    }
    for (int64_t f = 0; f < fields; ++f) {
        double *gtf = gt + f * img, *gmf = gm + f * img;
        for (int64_t i = 0; i < rows; ++i) {
            for (int64_t j = 0; j < cols; ++j) {
                for (int a = 0; a <= 2 * ry; ++a) {
                    for (int b = 0; b <= 2 * rx; ++b) {
                        int64_t si, sj;
                        if (!border_index(i + a - ry, rows, edge, &si)) continue;
                        if (!border_index(j + b - rx, cols, edge, &sj)) continue;
                        double term = weight2d(w2d, wy, wx, rx, a, b) * g1;
                        gtf[si * cols + sj] = gtf[si * cols + sj] + term;
                        gmf[si * cols + sj] = gmf[si * cols + sj] + fabs(term);
                    }
                }
            }
        }
    }
    double s0 = 0.0, s1 = 0.0, m0 = 0.0, m1 = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double fx, fy, fp0, fp1;
        elem_partials(map_op, params, (double)x[k], 0.0, &fx, &fy, &fp0, &fp1);
        dx[k] = gt[k] * fx;
        if (dx_mag) dx_mag[k] = gm[k] * fabs(fx);
        s0 = s0 + gt[k] * fp0;
        s1 = s1 + gt[k] * fp1;
        m0 = m0 + fabs(gt[k] * fp0);
        m1 = m1 + fabs(gt[k] * fp1);
    }
    if (dparams) {
        if (nparams > 0) dparams[0] = s0;
        if (nparams > 1) dparams[1] = s1;
    }
    if (dparams_mag) {
        if (nparams > 0) dparams_mag[0] = m0;
        if (nparams > 1) dparams_mag[1] = m1;
    }
    free(gt);
    free(gm);
    return 0;
}
