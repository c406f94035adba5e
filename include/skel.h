/*
 * skel.h -- C ABI of libskel, a library of data-parallel skeletons over smart
 * containers for one AMD Instinct MI355X (gfx950) GPU.
 *
 * Source of the concepts: Kessler, Dastgeer, Li, "Optimized Composition:
 * Generating Efficient Code for Heterogeneous Systems from Multi-Variant
 * Components, Skeletons and Containers" (arXiv:1405.2915).
 *   - Section III: skeletons are generic components derived from higher-order
 *     functions (map, scan, reduce, ...; mapoverlap among the data-parallel
 *     ones), parameterised by a user function; every skeleton has several
 *     implementation variants, and an execution plan picks one per call
 *     context (problem size, ...).
 *   - Section II: conditional composition (selectability constraints per
 *     variant) and static / off-line-tuned selection.
 *   - Section IV: smart containers own the operand data, track where valid
 *     copies live (a software coherence protocol), copy lazily, and never let a
 *     stale copy be read.
 *   - Section V: calls are asynchronous; containers carry the dependences.
 *
 * The paper defines none of these operations by formula.  The definitions
 * stated with each call below are the textbook ones and are the contract.
 *
 * General conventions
 *   - Every call returns a skel_status and never aborts or throws.  On an
 *     error, skel_last_error() returns a message (thread-local, valid until
 *     the next call on the same thread).  Arguments are validated before any
 *     work is enqueued: a call that fails validation has no side effect.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Skeleton calls are asynchronous on it; results stay in device memory
 *     until a host acquire asks for them (Section V).
 *   - Element counts and sizes are int64_t; containers may hold up to 2^31
 *     elements per axis and more than 2^32 bytes.
 *   - Thread compatibility: distinct containers may be used from distinct
 *     threads; calls on one container must not overlap.
 *   - `variant` selects an implementation variant by index (see
 *     skel_variant_name), or SKEL_VARIANT_AUTO to let the library's execution
 *     plan choose from the call context.  Forcing a variant whose
 *     selectability constraint does not hold returns SKEL_E_UNSUPPORTED.
 */
#ifndef SKEL_H
#define SKEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum skel_status {
    SKEL_OK = 0,
    SKEL_E_INVAL = 1,       /* null pointer, unknown enum, bad count/radius  */
    SKEL_E_DTYPE = 2,       /* element type combination not supported        */
    SKEL_E_SHAPE = 3,       /* operand sizes do not match                    */
    SKEL_E_NOMEM = 4,       /* host or device allocation failed              */
    SKEL_E_STATE = 5,       /* container access conflict or uninitialised read */
    SKEL_E_UNSUPPORTED = 6, /* forced variant not selectable for this call   */
    SKEL_E_HIP = 7,         /* HIP runtime error (message has the HIP text)  */
    SKEL_E_NOINIT = 8,      /* skel_init has not been called                 */
    SKEL_E_TIMEOUT = 9      /* a kernel's bounded inter-workgroup wait expired */
} skel_status;

typedef enum skel_dtype {
    SKEL_F32 = 0,  /* IEEE binary32                          */
    SKEL_BF16 = 1, /* bfloat16 (storage only, computed in f32) */
    SKEL_I32 = 2,  /* two's-complement 32-bit                */
    SKEL_I64 = 3   /* two's-complement 64-bit                */
} skel_dtype;

typedef enum skel_place { SKEL_HOST = 0, SKEL_DEVICE = 1 } skel_place;
typedef enum skel_access { SKEL_READ = 1, SKEL_WRITE = 2, SKEL_RW = 3 } skel_access;

/* border rule of MapOverlap: replicate the edge element, read a constant
 * pad value, or wrap around (periodic) */
typedef enum skel_edge {
    SKEL_EDGE_CLAMP = 0,
    SKEL_EDGE_CONST = 1,
    SKEL_EDGE_CYCLIC = 2
} skel_edge;

/* scan kinds.  The reverse kinds combine from the end of the array (suffix
 * scans); they are the adjoints of the forward SUM scans:
 *   d(inclusive)/dx applied to g = reverse inclusive scan of g,
 *   d(exclusive)/dx applied to g = reverse exclusive scan of g. */
typedef enum skel_scan_kind {
    SKEL_INCLUSIVE = 0,
    SKEL_EXCLUSIVE = 1,
    SKEL_REVERSE_INCLUSIVE = 2,
    SKEL_REVERSE_EXCLUSIVE = 3
} skel_scan_kind;

/* associative and commutative combining operator of Reduce / Scan */
typedef enum skel_reduce_op { SKEL_SUM = 0, SKEL_MIN = 1, SKEL_MAX = 2 } skel_reduce_op;

/* Built-in user functions f(x, y; p0, p1) of Map / MapReduce (a skeleton
 * instance is a skeleton plus its user function, Section III).  Parameters
 * are rounded to binary32, the type the kernels compute in. */
typedef enum skel_map_op {
    SKEL_MAP_IDENTITY = 0,    /* x               (1 input,  0 params) */
    SKEL_MAP_AXPY = 1,        /* p0*x + y        (2 inputs, 1 param, fused multiply-add) */
    SKEL_MAP_AFFINE = 2,      /* p0*x + p1       (1 input,  2 params) */
    SKEL_MAP_TANH = 3,        /* tanh(x)         (1 input,  0 params) */
    SKEL_MAP_AFFINE_TANH = 4, /* tanh(p0*x + p1) (1 input,  2 params) */
    SKEL_MAP_MUL = 5,         /* x*y             (2 inputs, 0 params) */
    SKEL_MAP_SQUARE = 6       /* x*x             (1 input,  0 params) */
} skel_map_op;

/* skeleton ids for the variant registry */
typedef enum skel_skeleton {
    SKEL_SK_MAP = 0,
    SKEL_SK_REDUCE = 1,
    SKEL_SK_MAPREDUCE = 2,
    SKEL_SK_MAPOVERLAP1D = 3,
    SKEL_SK_MAPOVERLAP2D = 4,
    SKEL_SK_SCAN = 5,
    SKEL_SK_REDUCE_SEGMENTS = 6,
    SKEL_SK_MAPOVERLAP1D_BACKWARD = 7,
    SKEL_SK_MAPOVERLAP2D_BACKWARD = 8,
    SKEL_SK_SCAN_ROWS = 9,
    SKEL_SK_MAP_OVERLAP2D_REDUCE = 10,
    SKEL_SK_COUNT = 11
} skel_skeleton;

#define SKEL_VARIANT_AUTO (-1)
#define SKEL_MAX_RADIUS_1D 64
#define SKEL_MAX_RADIUS_2D 8

/* Opaque smart container (Section IV): a Vector (rows = 1) or a row-major
 * Matrix, owned by the library. */
typedef struct skel_container skel_container;

/* Device-memory provider.  alloc returns a device pointer aligned to at least
 * 256 bytes (NULL on failure); free releases it, stream-ordered on `stream`.
 * Both are called from the thread that makes the library call. */
typedef struct skel_allocator {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} skel_allocator;

/* Transfer accounting of one container (Section IV, lazy copying).
 *   h2d / d2h          copies the coherence protocol actually issued
 *   h2d_bytes/d2h_bytes their sizes
 *   eager_equiv        copies an eager scheme would have issued: one host-to-
 *                      device copy per skeleton call that reads the container
 *                      and one device-to-host copy per call that writes it
 *   acquires           successful acquire calls (host or device)          */
typedef struct skel_xfer_stats {
    uint64_t h2d, d2h, h2d_bytes, d2h_bytes, eager_equiv, acquires;
} skel_xfer_stats;

/* ------------------------------------------------------------ runtime --- */

/* Bind the library to HIP device `device` (it becomes the current device of
 * the calling thread) and set the device-memory provider (NULL = hipMalloc /
 * hipFree).  May be called again with the same device to change the
 * provider; containers keep the provider they were created under. */
skel_status skel_init(int device, const skel_allocator *alloc);

/* Release the library's per-stream workspaces (not containers).  Blocks until
 * the device is idle.  skel_init may be called again afterwards. */
skel_status skel_finalize(void);

/* Wait for all work on `stream`, then report any error a kernel flagged (a
 * bounded wait that expired gives SKEL_E_TIMEOUT). */
skel_status skel_sync(void *stream);

const char *skel_last_error(void);

/* ---------------------------------------------------------- containers --- */

/* Create a smart container (Section IV: the operand data is wrapped in a
 * container that owns it and tracks where valid copies are) of rows x cols
 * elements of `dtype` (rows >= 1, cols >= 0).  If
 * host_src is non-NULL, rows*cols elements are copied from it (the caller may
 * free it on return) and the host copy is the valid one; otherwise the
 * container is uninitialised and must be written before it is read. */
skel_status skel_container_create(skel_dtype dtype, int64_t rows, int64_t cols,
                                  const void *host_src, skel_container **out);

/* Wrap caller-owned device memory as a container (for frameworks that hold
 * their tensors themselves).  dev_ptr holds rows*cols elements of `dtype`,
 * 16-byte aligned (the kernels use 16-byte vectors; SKEL_E_INVAL otherwise),
 * and is the container's valid device copy; its contents count as written on
 * `stream`, so a later access on another stream waits for that stream's work
 * enqueued before the wrap.  The library never frees dev_ptr, and a host copy
 * is allocated only if the host acquires the container.  The memory must
 * stay allocated until skel_container_destroy returns. */
skel_status skel_container_wrap_device(skel_dtype dtype, int64_t rows, int64_t cols,
                                       void *dev_ptr, void *stream,
                                       skel_container **out);

/* Destroy a container (Section IV: the container owns its copies, so it
 * frees them) with no outstanding acquire; device memory is released
 * stream-ordered after the last device access (wrapped device memory is left
 * to its owner).  Destroying waits for the container's pending device work
 * (unless it wraps device memory and has no host copy) and frees its pinned
 * host copy, so it must not run while a stream is being captured into a
 * graph: those calls would invalidate the capture. */
skel_status skel_container_destroy(skel_container *c);

/* Section IV coherence protocol.  Make the copy at `place` usable for
 * `access` and return its address in *ptr_out (valid until release):
 *   READ  copies from the other place iff this copy is stale;
 *   WRITE copies nothing and invalidates the other copy (whole overwrite);
 *   RW    both.
 * A device acquire enqueues its copy on `stream` and orders the access after
 * the conflicting device accesses on other streams (Section V dependences): a
 * WRITE/RW acquire, or a READ that copies stale data, after every other
 * stream's last access; a READ only after other streams' writes, so reads of
 * one container on several streams may run concurrently.  A host acquire
 * waits for the container's device work to finish.  Errors: SKEL_E_STATE when a
 * WRITE/RW acquire is outstanding, when WRITE/RW meets outstanding readers,
 * or when READ/RW finds no valid copy. */
skel_status skel_container_acquire(skel_container *c, skel_place place,
                                   skel_access access, void *stream,
                                   void **ptr_out);

/* Range-granular form of skel_container_acquire (Section IV: partial copies).
 * Validity is tracked per element range of each copy, so the protocol above
 * applies to elements [first, first + count) only: READ copies just the parts
 * of the range that are stale at `place` (one transfer per stale run), WRITE
 * makes the range current at `place` and stale at the other place and copies
 * nothing.  *ptr_out receives the address of element `first` of the copy.
 * Whole-container acquires (and the skeletons' operands) are the range
 * [0, n), so a container of which the host rewrote a few elements sends only
 * those elements to the device at its next device read.  Errors as for
 * skel_container_acquire, plus SKEL_E_INVAL for a range outside [0, n). */
skel_status skel_container_acquire_range(skel_container *c, skel_place place,
                                         skel_access access, int64_t first,
                                         int64_t count, void *stream, void **ptr_out);

/* The current element ranges of the copy at `place`: *count receives their
 * number and pairs[2k], pairs[2k+1] (for k < max_pairs) the k-th range
 * [first, last), in increasing order.  pairs may be NULL. */
skel_status skel_container_valid_ranges(const skel_container *c, skel_place place,
                                        int64_t *pairs, int64_t max_pairs, int64_t *count);

/* End the access begun by the matching acquire at `place` (Section IV
 * coherence protocol; Section V: a device release records the container's
 * last-access event on `stream`, the dependence later calls order after). */
skel_status skel_container_release(skel_container *c, skel_place place,
                                   void *stream);

skel_status skel_container_stats(const skel_container *c, skel_xfer_stats *out);

/* rows, cols and dtype of a container (any output pointer may be NULL) */
skel_status skel_container_info(const skel_container *c, skel_dtype *dtype,
                                int64_t *rows, int64_t *cols);

/* ----------------------------------------------------------- skeletons --- */

/* Map (Section III): out[i] = f(in[0][i], in[1][i]) for every element i.
 * nin is 1 or 2 as the op requires; all containers are F32 with the same
 * element count.  `out` may be one of the inputs (in-place). */
skel_status skel_map(skel_map_op op, const double *params, int nparams,
                     skel_container *const *in, int nin, skel_container *out,
                     int variant, void *stream);

/* Reduce (Section III): out1[0] = in[0] op in[1] op ... op in[n-1].
 * Type pairs (in -> out1): F32 -> F32 (binary32 accumulation),
 * BF16 -> F32, I32 -> I32 (wraps mod 2^32), I32 -> I64, I64 -> I64.  out1
 * holds one element.  n = 0 gives the identity (0, +inf / INT_MAX,
 * -inf / INT_MIN). */
skel_status skel_reduce(skel_reduce_op op, skel_container *in,
                        skel_container *out1, int variant, void *stream);

/* MapReduce: out1[0] = op over i of f(in[0][i], in[1][i]) with no stored
 * intermediate.  The paper names MapReduce only as another framework's
 * programming model (Section II); the reading taken here is the map-then-
 * reduce composition of the Section III map and reduce skeletons, fused.  Inputs F32 (or BF16 for IDENTITY/MUL/SQUARE), out1 F32. */
skel_status skel_mapreduce(skel_map_op map_op, const double *params,
                           int nparams, skel_container *const *in, int nin,
                           skel_reduce_op op, skel_container *out1,
                           int variant, void *stream);

/* MapOverlap 1D (Section III names mapoverlap among SkePU's data-parallel
 * skeletons; the linear neighbourhood weighting is the reading taken here):
 * out[i] = sum_{k=0}^{2r} w[k] * in[e(i + k - r)] over a
 * vector of n F32 elements (correlation orientation: w[0] weighs the lowest
 * index).  e() applies `edge` (pad is the CONST value).  w holds 2r+1 floats
 * (copied at call time); 0 <= r <= SKEL_MAX_RADIUS_1D.  out != in. */
skel_status skel_mapoverlap1d(skel_container *in, skel_container *out,
                              const float *w, int radius, skel_edge edge,
                              float pad, int variant, void *stream);

/* MapOverlap 2D (Section III, as MapOverlap 1D) on a rows x cols F32 matrix:
 *   out[i][j] = sum_{a=0}^{2ry} sum_{b=0}^{2rx} W[a][b] * in[e(i+a-ry)][e(j+b-rx)]
 * W is w2d ((2ry+1) x (2rx+1) row-major) when non-NULL, else the separable
 * outer product wy[a] * wx[b].  0 <= ry, rx <= SKEL_MAX_RADIUS_2D.  Weights
 * are copied at call time.  out != in. */
skel_status skel_mapoverlap2d(skel_container *in, skel_container *out,
                              const float *w2d, const float *wy,
                              const float *wx, int ry, int rx, skel_edge edge,
                              float pad, int variant, void *stream);

/* MapOverlap 2D over a batch of equally shaped images (fields) stored back to
 * back: in and out are (fields * H) x W containers, and every H x W field is
 * mapped on its own, exactly as skel_mapoverlap2d maps one image (its own
 * borders; no field reads another).  fields must divide the row count
 * (SKEL_E_SHAPE otherwise).  One launch covers many fields, which keeps the
 * device full for small fields.  skel_mapoverlap2d is the case fields = 1. */
skel_status skel_mapoverlap2d_fields(skel_container *in, skel_container *out,
                                     int64_t fields, const float *w2d,
                                     const float *wy, const float *wx, int ry,
                                     int rx, skel_edge edge, float pad,
                                     int variant, void *stream);

/* Scan (Section III): inclusive out[i] = in[0] op ... op in[i]; exclusive
 * out[0] = identity, out[i] = in[0] op ... op in[i-1]; reverse inclusive
 * out[i] = in[i] op ... op in[n-1]; reverse exclusive out[n-1] = identity,
 * out[i] = in[i+1] op ... op in[n-1].  Type pairs: I32 -> I32 (wraps), I32 ->
 * I64, I64 -> I64 (exact, wrapping), F32 -> F32.  out may equal in when the
 * types agree.  The reverse kinds run in the single-pass variants only (S2,
 * S3, S4 -- the single pass with small tiles -- and S5, the flat look-back
 * over those tiles; a forced S0 or S1 gives SKEL_E_UNSUPPORTED).  S5 takes at
 * most 1024 tiles: 2^22 elements, 2^21 for I64 inputs (SKEL_E_UNSUPPORTED
 * beyond). */
skel_status skel_scan(skel_container *in, skel_container *out,
                      skel_scan_kind kind, skel_reduce_op op, int variant,
                      void *stream);

/* Row-wise Scan: the Scan skeleton applied to every row of a rows x cols
 * matrix on its own (a batch of Scan instances of one length, Section III),
 *     out[r][c] = in[r][0] op ... op in[r][c]        (inclusive; the other
 * kinds as skel_scan, within each row).  in and out have the same shape; type
 * pairs, kinds, ops and in-place use as skel_scan.  Variants
 * (SKEL_SK_SCAN_ROWS): 0 runs one flat single-pass Scan per row (the plan's
 * choice for the row length; selectable only when every row starts 16-byte
 * aligned, i.e. cols * element size is a multiple of 16 for both types); 1
 * runs one wavefront per row in a single launch, with 16-byte accesses when
 * the rows are so aligned and element accesses otherwise.  The static rule
 * takes 0 for fewer than 64 aligned rows of at least 2^20 elements, else 1
 * (a few long rows that are not 16-byte aligned therefore run at one
 * wavefront per row, far below the device's bandwidth). */
skel_status skel_scan_rows(skel_container *in, skel_container *out,
                           skel_scan_kind kind, skel_reduce_op op, int variant,
                           void *stream);

/* The call chain Map -> MapOverlap 2D -> Reduce SUM as one skeleton call
 * (Section V: a chain of skeleton calls composed, here optimised as a whole;
 * Section III: the three skeletons):
 *     out1[0] = sum over fields f, pixels (i, j) of
 *               sum_{a,b} W[a][b] * t_f[e(i+a-ry)][e(j+b-rx)],   t = f(in)
 * in is a (fields * H) x W F32 container of `fields` images stored back to
 * back, each mapped with its own borders exactly as skel_mapoverlap2d_fields
 * maps it; map_op is a one-input element function (IDENTITY, AFFINE, TANH,
 * AFFINE_TANH or SQUARE; others give SKEL_E_INVAL) with its parameters;
 * weights, radii, edge and pad as skel_mapoverlap2d; out1 is one F32 element.
 * Variants (SKEL_SK_MAP_OVERLAP2D_REDUCE): 0 composed, the three skeletons'
 * kernels in turn with the mapped fields and the stencil output stored in the
 * stream's scratch memory; 1 fused, one pass that reads `in` once, weighing
 * f(in) by how often the neighbourhood map reads each element (the sum of a
 * linear map's outputs), plus the pad reads for CONST.  Both sum in binary32 in
 * a fixed order (deterministic).  fields must divide the row count
 * (SKEL_E_SHAPE).  n = 0 gives 0. */
skel_status skel_map_overlap2d_reduce(skel_map_op map_op, const double *params, int nparams,
                                      skel_container *in, int64_t fields, const float *w2d,
                                      const float *wy, const float *wx, int ry, int rx,
                                      skel_edge edge, float pad, skel_container *out1,
                                      int variant, void *stream);

/* Reverse mode through that chain, given g1 = dL/d(out1[0]) (one F32 element
 * on the device):
 *     grad_in = g1 * f'(in) * A^T 1   (A^T 1: how often, weighted, each
 *               element is read by the neighbourhood map of its field;
 *               CLAMP reads past an edge count on the edge element, CONST
 *               pad reads on none)
 *     grad_params[k] = g1 * sum_i (A^T 1)_i * df/dp_k(in_i)
 * grad_in: F32, shaped like in, overwritten; grad_params: 2 F32 elements for
 * AFFINE and AFFINE_TANH (NULL to skip), summed in a fixed order.  Same
 * variants as the forward: 0 composes the Reduce adjoint (broadcast of g1),
 * the MapOverlap adjoint and the Map adjoint through stored intermediates; 1
 * reads in once and writes grad_in once. */
skel_status skel_map_overlap2d_reduce_backward(skel_map_op map_op, const double *params,
                                               int nparams, skel_container *in, int64_t fields,
                                               const float *w2d, const float *wy,
                                               const float *wx, int ry, int rx, skel_edge edge,
                                               skel_container *g1, skel_container *grad_in,
                                               skel_container *grad_params, int variant,
                                               void *stream);

/* Segmented Reduce: the Reduce skeleton applied to many vectors of uneven
 * length at once (a batch of operands of one skeleton instance, Section III),
 *     out[s] = op over in[offsets[s]] .. in[offsets[s+1] - 1],  0 <= s < nseg
 * in: F32 with n elements (the vectors back to back); offsets: I64 with
 * nseg + 1 nondecreasing entries in [0, n]; out: F32 with nseg elements.
 * Empty segments give the identity.  The plain variant issues one Reduce per
 * segment; the persistent variant reduces every segment in one launch over
 * (segment, chunk) work items and combines each segment's partials in a fixed
 * order (deterministic).  The persistent variant checks the offsets on the
 * device: if they decrease or leave [0, n] it computes nothing and
 * skel_sync reports SKEL_E_TIMEOUT with flag 4; the per-segment variant
 * reads the offsets on the host and returns SKEL_E_INVAL.  No offsets can
 * make either variant access memory outside the containers. */
skel_status skel_reduce_segments(skel_reduce_op op, skel_container *in,
                                 skel_container *offsets, skel_container *out,
                                 int variant, void *stream);

/* Allocation-free Scan, for callers that cannot allocate device memory:
 * code being captured into a HIP graph, tight serving loops, harnesses that
 * forbid hipMalloc.  It computes exactly what skel_scan computes for the
 * forward kinds (SKEL_INCLUSIVE, SKEL_EXCLUSIVE; the reverse kinds give
 * SKEL_E_UNSUPPORTED), with the same type pairs and ops, on plain device
 * pointers instead of containers: in holds n elements of din, out receives n
 * elements of dout; both are device memory owned by the caller, 16-byte
 * aligned; out equals in (same types) or does not overlap it.  The work is
 * enqueued on `stream` and runs the reduce-then-scan variant S1, whose
 * per-tile totals live in a library array of 256 KiB in device memory, one
 * per GPU, held until the process ends; nothing is allocated or freed by the
 * call, and nothing needs clearing between calls (every total is written
 * before it is read).  Limit: n <= 2^30 elements for 4-byte inputs (I32,
 * F32) and 2^29 for I64 inputs (32768 tiles); larger n gives SKEL_E_SHAPE
 * before anything is enqueued.  Every call on one GPU shares that GPU's
 * array: calls that may run at the same time on one GPU (on different
 * streams without an ordering between them) race and give wrong results;
 * calls on one stream are ordered and safe.  Requires skel_init. */
skel_status skel_scan_noalloc(const void *in, skel_dtype din, void *out, skel_dtype dout,
                              int64_t n, skel_scan_kind kind, skel_reduce_op op,
                              void *stream);

/* --------------------------------------------------------- adjoints ---- */
/* Reverse-mode derivatives for a scalar loss L, given the upstream gradient
 * g = dL/d(out) of a forward call.  All operands are F32 containers; outputs
 * are overwritten (not accumulated into).  They back the torch.autograd
 * functions of the Python binding.  Reduce SUM backward is
 * skel_map_backward(IDENTITY) with a one-element g; MapReduce SUM backward is
 * skel_map_backward of its element function with a one-element g; Scan SUM
 * backward is skel_scan with the reverse kind. */

/* Map backward (chain rule of the element function, Section III map):
 *   grad_in[0][i] = g[i] * df/dx(x[i], y[i]),
 *   grad_in[1][i] = g[i] * df/dy(x[i], y[i])      (two-input ops only),
 *   grad_params[k] = sum_i g[i] * df/dp_k          (if grad_params != NULL)
 * in: the forward inputs (nin as the op requires); g: n elements, or one
 * element broadcast to every i; grad_in: nin containers of n elements, none
 * of them an input or g; grad_params: nparams elements (f32), summed over i
 * deterministically.  Tanh-based ops recompute tanh from x. */
skel_status skel_map_backward(skel_map_op op, const double *params, int nparams,
                              skel_container *const *in, int nin, skel_container *g,
                              skel_container *const *grad_in, skel_container *grad_params,
                              void *stream);

/* MapOverlap 1D backward: the transpose of in -> out applied to g,
 *   grad_in[j] = sum over (i, k) with e(i + k - r) = j of w[k] * g[i];
 * reads of the CONST pad send nothing back; with CLAMP the reads past either
 * end accumulate onto the end elements.  Same w, radius and edge as the
 * forward call; grad_in != g.  Variants (skeleton id
 * SKEL_SK_MAPOVERLAP1D_BACKWARD): 0 gathers the transpose directly for every
 * element; 1 runs the forward stencil kernel on g with the weights reversed
 * (the transpose of a correlation inside the array) and a zero pad or the
 * cyclic rule, then recomputes the two end elements for CLAMP. */
skel_status skel_mapoverlap1d_backward(skel_container *g, skel_container *grad_in,
                                       const float *w, int radius, skel_edge edge,
                                       int variant, void *stream);

/* MapOverlap 2D backward: the transpose of the 2D neighbourhood map,
 *   grad_in[s][t] = sum over (i, j, a, b) with e(i+a-ry) = s, e(j+b-rx) = t
 *                   of W[a][b] * g[i][j]
 * with the forward call's weights (w2d, or the factors wy, wx), radii and
 * edge rule; grad_in != g.  Variants (skeleton id
 * SKEL_SK_MAPOVERLAP2D_BACKWARD): 0 gathers directly for every pixel; 1 runs
 * the forward stencil kernels on g with the weights reversed along both axes
 * and a zero pad or the cyclic rule, then recomputes the first and last rows
 * and columns for CLAMP. */
skel_status skel_mapoverlap2d_backward(skel_container *g, skel_container *grad_in,
                                       const float *w2d, const float *wy,
                                       const float *wx, int ry, int rx, skel_edge edge,
                                       int variant, void *stream);

/* MapOverlap 2D backward over a batch of fields, as skel_mapoverlap2d_fields:
 * every field's transpose on its own.  skel_mapoverlap2d_backward is the case
 * fields = 1. */
skel_status skel_mapoverlap2d_fields_backward(skel_container *g,
                                              skel_container *grad_in,
                                              int64_t fields, const float *w2d,
                                              const float *wy, const float *wx,
                                              int ry, int rx, skel_edge edge,
                                              int variant, void *stream);

/* ------------------------------------------- variants and selection ---- */

int skel_variant_count(int skeleton);
const char *skel_variant_name(int skeleton, int variant); /* NULL if out of range */

/* The execution plan's choice (Section III) for a call context, without
 * running anything: returns the variant index, or -1 if none is selectable.
 * n is the element count (rows*cols for 2D); dtype is the input element type;
 * `aux` is the radius for SKEL_SK_MAPOVERLAP1D(_BACKWARD); for
 * SKEL_SK_MAPOVERLAP2D(_BACKWARD), separable + 2 * max(ry, rx), where separable
 * is 1 when the weights are given as factors wy, wx; 1 for the reverse kinds of SKEL_SK_SCAN and SKEL_SK_SCAN_ROWS, and ignored
 * otherwise (for SKEL_SK_SCAN_ROWS, rows and cols give the matrix shape and
 * dtype serves as both types). */
int skel_select_variant(int skeleton, skel_dtype dtype, int64_t n,
                        int64_t rows, int64_t cols, int aux);

/* Load a size-keyed dispatch table produced by off-line tuning (Section II:
 * a precomputed dispatch structure for fast run-time lookup; Section III:
 * execution plans built off-line per target system).  Text, one entry per
 * line, '#' starts a comment:
 *     <SKELETON> <dtype> <log2 n> <variant name or index> [<class>]
 * e.g. "REDUCE f32 20 R2_ticket".  MapOverlap entries (and only they) end with
 * the stencil class they were tuned on, as skel_select_variant's aux encodes
 * it (the radius in 1D; separable + 2 * max(ry, rx) in 2D, e.g.
 * "MAPOVERLAP2D f32 22 O2c_lds_separable 9" for 9 x 9 factors), and apply
 * only to calls of that class; other classes use the static rules.  A call of
 * size n uses the entry with the largest log2 n <= ceil(log2 n) for its
 * skeleton, input dtype (and class) (sizes beyond the table extrapolate from
 * its last entry, sizes below use its first).  An entry that is not selectable for a call falls back to the
 * static rules.  The whole file is validated before it replaces the current
 * table; on error the old table stays.  SKEL_VARIANT_<SKELETON>=<name> in the
 * environment overrides both. */
skel_status skel_load_plan(const char *path);
skel_status skel_clear_plan(void);

#ifdef __cplusplus
}
#endif
#endif /* SKEL_H */
