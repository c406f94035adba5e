/*
 * Skeleton oracle: a plain, slow, obviously correct CPU definition of what the
 * data-parallel skeletons compute.  TEST INFRASTRUCTURE ONLY -- the product
 * library never includes, links or calls this code; only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * Paper: Kessler, Dastgeer, Li, "Optimized Composition: Generating Efficient
 * Code for Heterogeneous Systems from Multi-Variant Components, Skeletons and
 * Containers" (arXiv:1405.2915).  Section III names the skeletons (map, scan,
 * reduce, derived from higher-order functions; mapoverlap among SkePU's
 * data-parallel skeletons) but gives no formulas.  Each function below states
 * the textbook higher-order-function definition it implements.
 *
 * Arithmetic: floating point is evaluated in IEEE binary64 from the stored
 * binary32 inputs, summed sequentially in index order (no blocking, no
 * reordering); integer arithmetic is modular in the unsigned type of the
 * output width (two's-complement wrap, no signed-overflow UB).
 *
 * Operation codes are this file's own; callers pass them by value.
 */
#ifndef SKEL_ORACLE_H
#define SKEL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element functions of Map / MapReduce (the "user function" of a skeleton
 * instance, Section III): f(x, y; p0, p1) */
enum {
    ORC_MAP_IDENTITY = 0,    /* x                 */
    ORC_MAP_AXPY = 1,        /* p0*x + y          */
    ORC_MAP_AFFINE = 2,      /* p0*x + p1         */
    ORC_MAP_TANH = 3,        /* tanh(x)           */
    ORC_MAP_AFFINE_TANH = 4, /* tanh(p0*x + p1)   */
    ORC_MAP_MUL = 5,         /* x*y               */
    ORC_MAP_SQUARE = 6       /* x*x               */
};

/* combining operator of Reduce / Scan */
enum { ORC_SUM = 0, ORC_MIN = 1, ORC_MAX = 2 };
/* scan kinds; the reverse forms combine from the end of the array (suffix
 * scans), which is also the adjoint of the forward sum scans */
enum { ORC_INCLUSIVE = 0, ORC_EXCLUSIVE = 1, ORC_REVERSE_INCLUSIVE = 2,
       ORC_REVERSE_EXCLUSIVE = 3 };
/* border handling of MapOverlap */
enum { ORC_EDGE_CLAMP = 0, ORC_EDGE_CONST = 1, ORC_EDGE_CYCLIC = 2 };

/* number of OpenMP threads used by the element-parallel loops (map, stencil);
 * reductions and scans are always sequential */
void oracle_set_threads(int n);
int oracle_get_threads(void);

/* Map: out[i] = f(x[i], y[i]).  y may be NULL for one-input functions.
 * Returns 0, or -1 for an unknown op / missing operand. */
int oracle_map_f32(int op, const double *params, int nparams, const float *x,
                   const float *y, int64_t n, double *out);

/* Reduce over binary32 input, evaluated in binary64.  SUM of n = 0 is 0,
 * MIN is +inf, MAX is -inf. */
double oracle_reduce_f32(int op, const float *x, int64_t n);
/* sum of |x[i]| in binary64: the magnitude scale of a floating-point sum */
double oracle_abs_sum_f32(const float *x, int64_t n);

/* Segmented Reduce: out[s] = reduce of x[off[s]] .. x[off[s+1]-1] for
 * 0 <= s < nseg (the Reduce definition applied to each segment).  Returns -1
 * if the offsets decrease or leave [0, n]. */
int oracle_reduce_segments_f32(int op, const float *x, int64_t n, const int64_t *off,
                               int64_t nseg, double *out);

/* Exactly rounded sums (the exact real sum, rounded once to binary64) by
 * Shewchuk's non-overlapping-partials algorithm ("Adaptive precision
 * floating-point arithmetic", 1997; the method of Python's math.fsum).
 * bfloat16 inputs are given as their 16-bit patterns.  The dot form sums the
 * products x[i]*y[i], each exact in binary64 (8-bit significands).
 * Non-finite inputs give NaN. */
double oracle_fsum_f64(const double *x, int64_t n);
double oracle_sum_bf16_exact(const uint16_t *x, int64_t n);
double oracle_dot_bf16_exact(const uint16_t *x, const uint16_t *y, int64_t n);

/* integer Reduce, wrapping in the output width */
int32_t oracle_reduce_i32_i32(int op, const int32_t *x, int64_t n);
int64_t oracle_reduce_i32_i64(int op, const int32_t *x, int64_t n);
int64_t oracle_reduce_i64_i64(int op, const int64_t *x, int64_t n);

/* MapReduce: r = reduce_op over i of f(x[i], y[i]).  *abs_sum (may be NULL)
 * receives sum of |f(x[i], y[i])|. */
double oracle_mapreduce_f32(int map_op, const double *params, int nparams,
                            const float *x, const float *y, int64_t n,
                            int reduce_op, double *abs_sum);

/* MapOverlap 1D (a weighted neighbourhood, correlation orientation):
 *   out[i] = sum_{k=0}^{2r} w[k] * x[e(i + k - r)]
 * e() is the border rule (clamp, constant pad, cyclic).  mag[i] (may be NULL)
 * receives sum_k |w[k] * x[e(i+k-r)]|.  Returns 0 or -1 on bad arguments. */
int oracle_mapoverlap1d_f32(const float *x, int64_t n, const float *w, int r,
                            int edge, float pad, double *out, double *mag);

/* MapOverlap 2D on a rows x cols row-major image:
 *   out[i][j] = sum_{a=0}^{2ry} sum_{b=0}^{2rx} W[a][b] * x[e(i+a-ry)][e(j+b-rx)]
 * W is w2d ((2ry+1) x (2rx+1) row-major) if w2d != NULL, else the outer
 * product wy[a]*wx[b] formed exactly in binary64. */
int oracle_mapoverlap2d_f32(const float *x, int64_t rows, int64_t cols,
                            const float *w2d, const float *wy, const float *wx,
                            int ry, int rx, int edge, float pad, double *out,
                            double *mag);
/* the same definition for the single output (i, j) */
double oracle_mapoverlap2d_at_f32(const float *x, int64_t rows, int64_t cols,
                                  const float *w2d, const float *wy,
                                  const float *wx, int ry, int rx, int edge,
                                  float pad, int64_t i, int64_t j, double *mag);

/* Scan (prefix combination):
 *   inclusive out[i] = x[0] op ... op x[i]
 *   exclusive out[0] = identity, out[i] = x[0] op ... op x[i-1]
 *   reverse inclusive out[i] = x[i] op ... op x[n-1]
 *   reverse exclusive out[n-1] = identity, out[i] = x[i+1] op ... op x[n-1]
 * Return 0, or -1 for a bad op / kind. */
int oracle_scan_i32_i32(const int32_t *x, int64_t n, int kind, int op,
                        int32_t *out);
int oracle_scan_i32_i64(const int32_t *x, int64_t n, int kind, int op,
                        int64_t *out);
int oracle_scan_i64_i64(const int64_t *x, int64_t n, int kind, int op,
                        int64_t *out);
/* floating-point Scan in binary64; mag[i] (may be NULL) is the sum of |x[j]|
 * over the terms of out[i] */
int oracle_scan_f32(const float *x, int64_t n, int kind, int op, double *out,
                    double *mag);

/* ------------------------------------------------------------ adjoints --
 * Reverse-mode derivatives of the skeletons, for a scalar loss L with
 * upstream gradient g = dL/d(out).  Each is the plain definition of the
 * transposed linear map (or of the chain rule), evaluated in binary64. */

/* Map: dx[i] = g[i] * df/dx(x[i], y[i]), dy[i] = g[i] * df/dy (only for the
 * two-input functions; dy may be NULL otherwise), and
 * dparams[k] = sum_i g[i] * df/dp_k (summed in index order; dparams may be
 * NULL; it has nparams entries).  dparams_mag[k] (may be NULL) receives
 * sum_i |g[i] * df/dp_k|.  Returns 0, or -1 for a bad op / operand. */
int oracle_map_grad_f32(int op, const double *params, int nparams, const float *x,
                        const float *y, const float *g, int64_t n, double *dx,
                        double *dy, double *dparams, double *dparams_mag);

/* MapOverlap 1D adjoint: the transpose of x -> out, applied to g:
 *   dx[j] = sum over (i, k) with e(i + k - r) = j of w[k] * g[i]
 * (a read of the constant pad contributes to no x).  mag[j] (may be NULL)
 * receives the sum of |w[k] * g[i]| over the same terms. */
int oracle_mapoverlap1d_adjoint_f32(const float *g, int64_t n, const float *w, int r,
                                    int edge, double *dx, double *mag);

/* MapOverlap 2D adjoint on a rows x cols image, same weights as the forward:
 *   dx[s][t] = sum over (i, j, a, b) with e(i+a-ry) = s, e(j+b-rx) = t of
 *              W[a][b] * g[i][j] */
int oracle_mapoverlap2d_adjoint_f32(const float *g, int64_t rows, int64_t cols,
                                    const float *w2d, const float *wy,
                                    const float *wx, int ry, int rx, int edge,
                                    double *dx, double *mag);

/* The call chain Map -> MapOverlap 2D -> Reduce SUM over `fields` images of
 * rows x cols stored back to back (a composition of skeleton calls, Section V):
 *   loss = sum_{f,i,j} sum_{a,b} W[a][b] * t_f[e(i+a-ry)][e(j+b-rx)],
 *   t = f(x; params) (one-input element functions only), pad outside for CONST.
 * Binary64 throughout, no rounding between the steps.  *mag (may be NULL)
 * receives the sum of |W[a][b] * read value| over every term.  Returns NaN for
 * bad arguments. */
double oracle_chain_f32(int map_op, const double *params, int nparams, const float *x,
                        int64_t fields, int64_t rows, int64_t cols, const float *w2d,
                        const float *wy, const float *wx, int ry, int rx, int edge,
                        float pad, double *mag);

/* Reverse mode through that chain for the loss's upstream gradient g1:
 *   gt = MapOverlap adjoint of (g1 everywhere);  dx = gt * df/dx;
 *   dparams[p] = sum_k gt[k] * df/dp_p (index order).
 * dx_mag, dparams, dparams_mag may be NULL.  Returns 0, or -1. */
int oracle_chain_grad_f32(int map_op, const double *params, int nparams, const float *x,
                          int64_t fields, int64_t rows, int64_t cols, const float *w2d,
                          const float *wy, const float *wx, int ry, int rx, int edge,
                          double g1, double *dx, double *dx_mag, double *dparams,
                          double *dparams_mag);

#ifdef __cplusplus
}
#endif
#endif
