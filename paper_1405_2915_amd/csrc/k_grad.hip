// Reverse-mode kernels: the adjoints of Map and MapOverlap for a scalar loss
// (the scan adjoint is the reverse scan in k_scan.hip, the Reduce adjoint is
// the Map adjoint of the identity with a broadcast gradient).
//
//   map_grad       dx = g * df/dx, dy = g * df/dy, and per-workgroup partial
//                  sums of g * df/dp_k combined in order by map_grad_finish;
//                  16-byte vectors, the gradient optionally one broadcast
//                  value (Reduce / MapReduce backward)
//   ov1_adjoint    transpose of the 1D neighbourhood map as a gather: element
//                  j collects w[k] * g[j - k + r] (wrapping for CYCLIC), and
//                  with CLAMP the two end elements also collect every read
//                  that fell past their end
//   ov2_adjoint    the same per axis for the 2D map: for each tap (a, b) the
//                  rows i that read row s form a contiguous range (one row
//                  inside the image, up to ry + 1 rows at a clamped edge)
//
// All are HBM streams (map_grad: 12 to 20 bytes per element; adjoints: 8
// bytes per element plus the cached neighbourhood reads).
#include "kcommon.hpp"
#include "kelem.hpp"
#include "dispatch.hpp"
#include "launch.hpp"

namespace skel {
namespace {

using dev::f32x4;

constexpr int kBlock = 256;

template <int OP>
constexpr bool grad_two_inputs() { return dev::two_inputs<OP>(); }
template <int OP>
constexpr int grad_nparams() { return dev::map_nparams<OP>(); }
using dev::elem_grad;

template <int OP, bool BCAST>
__global__ __launch_bounds__(kBlock) void map_grad(const float* x, const float* y,
                                                   const float* g, float* dx, float* dy,
                                                   int64_t n, float p0, float p1,
                                                   float* partials) {
    constexpr bool TWO = grad_two_inputs<OP>();
    constexpr int NP = grad_nparams<OP>();
    constexpr int U = 4;  // vectors in flight per lane and input
    const float gb = BCAST ? g[0] : 0.0f;
    float a0 = 0.0f, a1 = 0.0f;
    const int64_t nv = n / 4;
    const f32x4* xv = reinterpret_cast<const f32x4*>(x);
    const f32x4* yv = reinterpret_cast<const f32x4*>(y);
    const f32x4* gv = reinterpret_cast<const f32x4*>(g);
    // chunks of U * kBlock vectors, every load of a chunk issued before the
    // arithmetic; single-use inputs and outputs are streamed non-temporally
    for (int64_t c = (int64_t)blockIdx.x * U * kBlock; c < nv; c += (int64_t)gridDim.x * U * kBlock) {
        f32x4 xa[U], ya[U], ga[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = c + u * kBlock + threadIdx.x;
            const bool in = i < nv;
            xa[u] = in ? __builtin_nontemporal_load(&xv[i]) : f32x4{0.f, 0.f, 0.f, 0.f};
            // y enters the derivatives of MUL only (AXPY's are 1 and p0)
            ya[u] = (OP == SKEL_MAP_MUL && in) ? __builtin_nontemporal_load(&yv[i])
                                               : f32x4{0.f, 0.f, 0.f, 0.f};
            ga[u] = BCAST ? f32x4{gb, gb, gb, gb}
                          : (in ? __builtin_nontemporal_load(&gv[i]) : f32x4{0.f, 0.f, 0.f, 0.f});
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = c + u * kBlock + threadIdx.x;
            if (i >= nv) break;
            f32x4 ox, oy;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float ddx, ddy, s0, s1;
                elem_grad<OP>(xa[u][e], ya[u][e], ga[u][e], p0, p1, ddx, ddy, s0, s1);
                ox[e] = ddx;
                oy[e] = ddy;
                a0 += s0;
                a1 += s1;
            }
            dev::store_vec_nt(ox, reinterpret_cast<f32x4*>(dx) + i);
            if constexpr (TWO) dev::store_vec_nt(oy, reinterpret_cast<f32x4*>(dy) + i);
        }
    }
    // the n % 4 tail, one element per low lane of the first workgroup
    const int64_t t = nv * 4 + (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x == 0 && t < n) {
        float ddx, ddy, s0, s1;
        elem_grad<OP>(x[t], OP == SKEL_MAP_MUL ? y[t] : 0.0f, BCAST ? gb : g[t], p0, p1, ddx,
                      ddy, s0, s1);
        dx[t] = ddx;
        if constexpr (TWO) dy[t] = ddy;
        a0 += s0;
        a1 += s1;
    }
    if constexpr (NP > 0) {
        __shared__ float l0[kBlock / dev::kWave], l1[kBlock / dev::kWave];
        using C = dev::Comb<float, SKEL_SUM>;
        a0 = dev::block_reduce<C>(a0, l0);
        a1 = dev::block_reduce<C>(a1, l1);
        if (threadIdx.x == 0) {
            partials[2 * blockIdx.x] = a0;
            partials[2 * blockIdx.x + 1] = a1;
        }
    }
}

// parameter gradients: the workgroups' partials summed in workgroup order
__global__ __launch_bounds__(kBlock) void map_grad_finish(const float* partials, int groups,
                                                          int nparams, float* out) {
    __shared__ float l0[kBlock / dev::kWave], l1[kBlock / dev::kWave];
    using C = dev::Comb<float, SKEL_SUM>;
    float a0 = 0.0f, a1 = 0.0f;
    for (int b = threadIdx.x; b < groups; b += kBlock) {
        a0 += partials[2 * b];
        a1 += partials[2 * b + 1];
    }
    a0 = dev::block_reduce<C>(a0, l0);
    a1 = dev::block_reduce<C>(a1, l1);
    if (threadIdx.x == 0) {
        out[0] = a0;
        if (nparams > 1) out[1] = a1;
    }
}

// --------------------------------------------------------- MapOverlap 1D ---
struct WA1 {
    float w[2 * SKEL_MAX_RADIUS_1D + 1];
};

__device__ __forceinline__ int64_t wrap_index(int64_t i, int64_t n) {
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

// the transpose at element j, gathered: the outputs i whose tap k read x[j]
__device__ __forceinline__ float adj1_at(const float* g, int64_t n, const WA1& w, int r, int edge,
                                         int64_t j) {
    float acc = 0.0f;
    if (edge == SKEL_EDGE_CYCLIC) {
        for (int k = 0; k <= 2 * r; ++k)
            acc = __builtin_fmaf(w.w[k], g[wrap_index(j - k + r, n)], acc);
        return acc;
    }
    for (int k = 0; k <= 2 * r; ++k) {
        const int64_t i = j - k + r;
        if (i >= 0 && i < n) acc = __builtin_fmaf(w.w[k], g[i], acc);
    }
    if (edge == SKEL_EDGE_CLAMP) {
        // reads below index 0 (i + k - r < 0) land on element 0, reads above
        // n - 1 on element n - 1
        if (j == 0)
            for (int k = 0; k < r; ++k)
                for (int64_t i = 0; i < n && i < r - k; ++i) acc = __builtin_fmaf(w.w[k], g[i], acc);
        if (j == n - 1)
            for (int k = r + 1; k <= 2 * r; ++k)
                for (int64_t i = n - 1; i >= 0 && i > n - 1 + r - k; --i)
                    acc = __builtin_fmaf(w.w[k], g[i], acc);
    }
    return acc;
}

__global__ __launch_bounds__(kBlock) void ov1_adjoint(const float* g, float* dx, int64_t n,
                                                      WA1 w, int r, int edge) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride)
        dx[j] = adj1_at(g, n, w, r, edge, j);
}

// elements 0 and n - 1 only (where clamped reads land)
__global__ void ov1_adjoint_ends(const float* g, float* dx, int64_t n, WA1 w, int r, int edge) {
    const int64_t j = threadIdx.x == 0 ? 0 : n - 1;
    if (threadIdx.x < 2) dx[j] = adj1_at(g, n, w, r, edge, j);
}

// --------------------------------------------------------- MapOverlap 2D ---
struct WA2 {
    float w[(2 * SKEL_MAX_RADIUS_2D + 1) * (2 * SKEL_MAX_RADIUS_2D + 1)];
};

// rows i of a length-len axis whose tap a (radius r) reads row s: the range
// [*lo, *hi] (empty if lo > hi).  Inside the axis it is the single row
// s - a + r; a clamped end also collects every read that fell past it; with
// CYCLIC the single row wraps.
__device__ __forceinline__ void tap_range(int64_t s, int a, int r, int64_t len, int edge,
                                          int64_t* lo, int64_t* hi) {
    const int64_t i = s - a + r;
    if (edge == SKEL_EDGE_CYCLIC) {
        *lo = *hi = wrap_index(i, len);
        return;
    }
    *lo = i;
    *hi = i;
    if (edge == SKEL_EDGE_CLAMP) {
        if (s == 0) *lo = -((int64_t)1 << 40);     // reads at or below 0
        if (s == len - 1) *hi = (int64_t)1 << 40;  // reads at or above len - 1
    }
    if (*lo < 0) *lo = 0;
    if (*hi > len - 1) *hi = len - 1;
}

// the transpose at pixel (s, t), gathered
__device__ __forceinline__ float adj2_at(const float* g, int64_t rows, int64_t cols, const WA2& w,
                                         int ry, int rx, int edge, int64_t s, int64_t t) {
    const int nx = 2 * rx + 1;
    float acc = 0.0f;
    for (int a = 0; a <= 2 * ry; ++a) {
        int64_t ilo, ihi;
        tap_range(s, a, ry, rows, edge, &ilo, &ihi);
        for (int b = 0; b <= 2 * rx; ++b) {
            int64_t jlo, jhi;
            tap_range(t, b, rx, cols, edge, &jlo, &jhi);
            const float wab = w.w[a * nx + b];
            for (int64_t i = ilo; i <= ihi; ++i)
                for (int64_t j = jlo; j <= jhi; ++j) acc = __builtin_fmaf(wab, g[i * cols + j], acc);
        }
    }
    return acc;
}

__global__ __launch_bounds__(kBlock) void ov2_adjoint(const float* g, float* dx, int64_t rows,
                                                      int64_t cols, WA2 w, int ry, int rx,
                                                      int edge) {
    // blockIdx.y: one of several equally shaped images stored back to back
    g += (int64_t)blockIdx.y * rows * cols;
    dx += (int64_t)blockIdx.y * rows * cols;
    const int64_t total = rows * cols;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < total; p += stride) {
        const int64_t s = p / cols;
        dx[p] = adj2_at(g, rows, cols, w, ry, rx, edge, s, p - s * cols);
    }
}

// the first and last rows and columns only (the pixels that clamped reads
// land on), in order: row 0, row rows-1, then column 0 and column cols-1 of
// the rows in between.  A group of G lanes per pixel (a power of two chosen by
// the launcher from the tap count: 4 for 3 x 3 weights, 32 for 9 x 9) shares
// the taps (a, b), each lane gathering its taps' row and column ranges, and
// the lane sums are combined by a fixed butterfly within the group.
__global__ __launch_bounds__(kBlock) void ov2_adjoint_border(const float* g, float* dx,
                                                             int64_t rows, int64_t cols, WA2 w,
                                                             int ry, int rx, int edge, int G) {
    // blockIdx.y: one of several equally shaped images stored back to back
    g += (int64_t)blockIdx.y * rows * cols;
    dx += (int64_t)blockIdx.y * rows * cols;
    const int64_t nrow = rows > 1 ? 2 : 1;
    const int64_t ncol = cols > 1 ? 2 : 1;
    const int64_t mid = rows > 2 ? rows - 2 : 0;
    const int64_t total = nrow * cols + ncol * mid;
    const int lg = (int)threadIdx.x % G;  // lane within the pixel's group
    const int nx = 2 * rx + 1, taps = (2 * ry + 1) * nx;
    const int64_t groups = (int64_t)gridDim.x * (kBlock / G);
    // every lane runs the same number of iterations (the butterfly below needs
    // whole wavefronts): pixels past the end are computed on pixel 0 and not
    // stored
    const int64_t iters = (total + groups - 1) / groups;
    for (int64_t it = 0; it < iters; ++it) {
        const int64_t p = it * groups + (int64_t)blockIdx.x * (kBlock / G) + threadIdx.x / G;
        const bool live = p < total;
        const int64_t pp = live ? p : 0;
        int64_t s, t;
        if (pp < nrow * cols) {
            s = pp < cols ? 0 : rows - 1;
            t = pp < cols ? pp : pp - cols;
        } else {
            const int64_t q = pp - nrow * cols;
            s = 1 + q / ncol;
            t = (q % ncol) == 0 ? 0 : cols - 1;
        }
        float acc = 0.0f;
        for (int q = lg; q < taps; q += G) {
            const int a = q / nx, b = q - a * nx;
            int64_t ilo, ihi, jlo, jhi;
            tap_range(s, a, ry, rows, edge, &ilo, &ihi);
            tap_range(t, b, rx, cols, edge, &jlo, &jhi);
            const float wab = w.w[q];
            for (int64_t i = ilo; i <= ihi; ++i)
                for (int64_t j = jlo; j <= jhi; ++j) acc = __builtin_fmaf(wab, g[i * cols + j], acc);
        }
        for (int o = G >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (live && lg == 0) dx[s * cols + t] = acc;
    }
}

int grid_for(int64_t units, const DevInfo& d) {
    int64_t g = (units + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)d.cus * 8;
    if (g > cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

template <int OP>
skel_status map_grad_op(float p0, float p1, const float* x, const float* y, const float* g,
                        bool bcast, float* dx, float* dy, int64_t n, float* dparams,
                        LaunchCtx& lc) {
    constexpr int NP = grad_nparams<OP>();
    const int groups = grid_for((n + 15) / 16, *lc.dev);  // 4 vectors of 4 per lane
    float* partials = nullptr;
    if (NP > 0 && dparams) {
        void* mem = nullptr;
        skel_status e = ws_scratch(lc, (size_t)groups * 2 * sizeof(float), &mem);
        if (e != SKEL_OK) return e;
        partials = static_cast<float*>(mem);
    }
    if (bcast)
        map_grad<OP, true><<<groups, kBlock, 0, lc.stream>>>(x, y, g, dx, dy, n, p0, p1, partials);
    else
        map_grad<OP, false><<<groups, kBlock, 0, lc.stream>>>(x, y, g, dx, dy, n, p0, p1, partials);
    skel_status e = launch_check("map_grad");
    if (e != SKEL_OK || !partials) return e;
    map_grad_finish<<<1, kBlock, 0, lc.stream>>>(partials, groups, NP, dparams);
    return launch_check("map_grad_finish");
}

}  // namespace

skel_status launch_map_backward(int op, float p0, float p1, const float* x, const float* y,
                                const float* g, bool g_broadcast, float* dx, float* dy,
                                int64_t n, float* dparams, LaunchCtx& lc) {
    switch (op) {
    case SKEL_MAP_IDENTITY:
        return map_grad_op<SKEL_MAP_IDENTITY>(p0, p1, x, y, g, g_broadcast, dx, dy, n, dparams, lc);
    case SKEL_MAP_AXPY:
        return map_grad_op<SKEL_MAP_AXPY>(p0, p1, x, y, g, g_broadcast, dx, dy, n, dparams, lc);
    case SKEL_MAP_AFFINE:
        return map_grad_op<SKEL_MAP_AFFINE>(p0, p1, x, y, g, g_broadcast, dx, dy, n, dparams, lc);
    case SKEL_MAP_TANH:
        return map_grad_op<SKEL_MAP_TANH>(p0, p1, x, y, g, g_broadcast, dx, dy, n, dparams, lc);
    case SKEL_MAP_AFFINE_TANH:
        return map_grad_op<SKEL_MAP_AFFINE_TANH>(p0, p1, x, y, g, g_broadcast, dx, dy, n,
                                                 dparams, lc);
    case SKEL_MAP_MUL:
        return map_grad_op<SKEL_MAP_MUL>(p0, p1, x, y, g, g_broadcast, dx, dy, n, dparams, lc);
    default:
        return map_grad_op<SKEL_MAP_SQUARE>(p0, p1, x, y, g, g_broadcast, dx, dy, n, dparams, lc);
    }
}

// A1 (both dimensions): the transpose of a correlation with weights w inside
// the array is the correlation with the reversed weights, so the forward
// kernels compute it with a zero pad (CONST edges send nothing back, and for
// CLAMP this is every element but the ends) or with the cyclic rule (exact);
// for CLAMP the elements that clamped reads land on are then recomputed by
// the gather.
skel_status launch_overlap1d_adjoint(int v, const float* g, float* dx, int64_t n,
                                     const float* w, int r, int edge, LaunchCtx& lc) {
    WA1 wk{};
    for (int k = 0; k <= 2 * r; ++k) wk.w[k] = w[k];
    if (v == A0_GATHER) {
        ov1_adjoint<<<grid_for(n, *lc.dev), kBlock, 0, lc.stream>>>(g, dx, n, wk, r, edge);
        return launch_check("ov1_adjoint");
    }
    float wf[2 * SKEL_MAX_RADIUS_1D + 1];
    for (int k = 0; k <= 2 * r; ++k) wf[k] = w[2 * r - k];
    const int fwd = r <= 4 ? O1C_SHUFFLE : O1B_LDS_TILE;
    skel_status e = launch_overlap1d(fwd, g, dx, n, wf, r,
                                     edge == SKEL_EDGE_CYCLIC ? SKEL_EDGE_CYCLIC : SKEL_EDGE_CONST,
                                     0.0f, lc);
    if (e != SKEL_OK || edge != SKEL_EDGE_CLAMP) return e;
    ov1_adjoint_ends<<<1, dev::kWave, 0, lc.stream>>>(g, dx, n, wk, r, edge);
    return launch_check("ov1_adjoint_ends");
}

skel_status launch_overlap2d_adjoint(int v, const float* g, float* dx, int64_t rows,
                                     int64_t cols, int64_t fields, const float* w2d,
                                     const float* wy, const float* wx, int ry, int rx, int edge,
                                     LaunchCtx& lc) {
    WA2 wk{};
    const int ny = 2 * ry + 1, nx = 2 * rx + 1;
    for (int a = 0; a < ny; ++a)
        for (int b = 0; b < nx; ++b) wk.w[a * nx + b] = w2d ? w2d[a * nx + b] : wy[a] * wx[b];
    const int64_t img = rows * cols;
    if (v == A0_GATHER) {
        for (int64_t f0 = 0; f0 < fields; f0 += kMaxFieldsPerLaunch) {
            const unsigned nf = (unsigned)std::min<int64_t>(fields - f0, kMaxFieldsPerLaunch);
            ov2_adjoint<<<dim3(grid_for(img, *lc.dev), nf), kBlock, 0, lc.stream>>>(
                g + f0 * img, dx + f0 * img, rows, cols, wk, ry, rx, edge);
            const skel_status e = launch_check("ov2_adjoint");
            if (e != SKEL_OK) return e;
        }
        return SKEL_OK;
    }
    const int fe = edge == SKEL_EDGE_CYCLIC ? SKEL_EDGE_CYCLIC : SKEL_EDGE_CONST;
    skel_status e;
    if (w2d) {
        float wf[(2 * SKEL_MAX_RADIUS_2D + 1) * (2 * SKEL_MAX_RADIUS_2D + 1)];
        for (int a = 0; a < ny; ++a)
            for (int b = 0; b < nx; ++b) wf[a * nx + b] = w2d[(ny - 1 - a) * nx + (nx - 1 - b)];
        e = launch_overlap2d(overlap2d_dense_variant(fields * img, ry > rx ? ry : rx), g, dx,
                             rows, cols, fields, wf, nullptr, nullptr, ry, rx, fe, 0.0f, lc);
    } else {
        float fy[2 * SKEL_MAX_RADIUS_2D + 1], fx[2 * SKEL_MAX_RADIUS_2D + 1];
        for (int a = 0; a < ny; ++a) fy[a] = wy[ny - 1 - a];
        for (int b = 0; b < nx; ++b) fx[b] = wx[nx - 1 - b];
        e = launch_overlap2d(overlap2d_separable_variant(fields * img, ry > rx ? ry : rx), g, dx,
                             rows, cols, fields, nullptr, fy, fx, ry, rx, fe, 0.0f, lc);
    }
    if (e != SKEL_OK || edge != SKEL_EDGE_CLAMP) return e;
    const int taps = ny * nx;
    // lanes per border pixel: the power of two that gives each lane about four
    // taps (measured against one tap per lane: 9x9 transpose on 4096^2 47 ->
    // 42 us, the 64-field 3x3 transpose 500 -> 470 us; eight per lane: same)
    constexpr int kTapsPerLane = 4;
    int G = 1;
    while (G * kTapsPerLane < taps && G < dev::kWave) G *= 2;
    const int64_t border = 2 * cols + 2 * rows;
    for (int64_t f0 = 0; f0 < fields; f0 += kMaxFieldsPerLaunch) {
        const unsigned nf = (unsigned)std::min<int64_t>(fields - f0, kMaxFieldsPerLaunch);
        ov2_adjoint_border<<<dim3(grid_for(border * G, *lc.dev), nf), kBlock, 0, lc.stream>>>(
            g + f0 * img, dx + f0 * img, rows, cols, wk, ry, rx, edge, G);
        e = launch_check("ov2_adjoint_border");
        if (e != SKEL_OK) return e;
    }
    return SKEL_OK;
}

}  // namespace skel
