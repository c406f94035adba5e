// The call chain Map -> MapOverlap 2D -> Reduce SUM over a batch of fields
// (composition of skeleton calls, Section V; the three skeletons, Section III):
//
//     loss = sum over fields f and pixels (i, j) of (A_f f(x))[i][j]
//
// where f is a one-input element function and A_f the 2D neighbourhood map of
// field f with its own borders.  Variants:
//   C0  composed: the three skeletons' kernels in turn, with the mapped field
//       and the stencil output stored in between (the plain form: 20 bytes
//       per element moved forward, 24 backward)
//   C1  fused: the sum of a linear map's outputs is the input weighted by the
//       map's column sums, sum(A t) = sum_k t_k (A^T 1)_k (plus the constant
//       pad reads for CONST borders).  (A^T 1) at an element depends only on
//       its distance to the field's borders -- it is the weight sum inside,
//       and differs only within the radius of an edge -- so the host tabulates
//       it per row class x column class (at most 17 x 17 values) and the chain
//       becomes one reduction that reads x once (4 bytes per element).  The
//       backward pass is one more stream: dx = g1 * f'(x) * (A^T 1), with the
//       parameter sums g1 * sum (A^T 1) df/dp in the same pass (8 bytes per
//       element).
// Both C1 kernels write one partial per workgroup and a one-workgroup finish
// combines them in order, so results are deterministic.
#include "chain_table.hpp"
#include "kcommon.hpp"
#include "kelem.hpp"
#include "dispatch.hpp"
#include "launch.hpp"

namespace skel {
namespace {

using namespace dev;

constexpr int kBlock = 256;
constexpr int kUnroll = 4;
constexpr int kMaxClasses = kChainMaxClasses;

// Unsigned division by a divisor fixed for the whole launch, as a multiply-high
// and shifts (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994, unsigned case): l = ceil(log2 d),
// m = floor(2^64 (2^l - d) / d) + 1, q = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0)
// with t = mulhi(m, n).  Exact for every 64-bit n and 1 <= d < 2^63.
struct DivU64 {
    uint64_t m;
    int s1, s2;
    __device__ __forceinline__ uint64_t div(uint64_t n) const {
        const uint64_t t = __umul64hi(m, n);
        return (t + ((n - t) >> s1)) >> s2;
    }
};

DivU64 make_div(uint64_t d) {
    int l = 0;
    while (l < 63 && (UINT64_C(1) << l) < d) ++l;
    const unsigned __int128 num = (unsigned __int128)((UINT64_C(1) << l) - d) << 64;
    DivU64 r;
    r.m = (uint64_t)(num / d) + 1;
    r.s1 = l < 1 ? l : 1;
    r.s2 = l > 1 ? l - 1 : 0;
    return r;
}

// What the kernels need to weigh an element: the field shape, the dividers
// that locate a flat index in its field, and the (A^T 1) table of
// chain_table.hpp (row classes, column classes, the interior entry).
struct ChainGeom {
    int64_t rows, cols;
    DivU64 by_cols, by_rows;  // element index -> row; row -> field
    int ry, rx;
    int small_r, small_c;     // fewer than 2r + 1 rows / columns
    int ncc;                  // column classes (table row length)
    float interior;           // the table's interior entry (the weight sum)
    float tab[kMaxClasses * kMaxClasses];
};

__device__ __forceinline__ int row_class(const ChainGeom& g, int64_t r) {
    if (g.small_r) return (int)r;
    if (r < g.ry) return (int)r;
    if (r >= g.rows - g.ry) return 2 * g.ry - (int)(g.rows - 1 - r);
    return g.ry;
}
__device__ __forceinline__ int col_class(const ChainGeom& g, int64_t c) {
    if (g.small_c) return (int)c;
    if (c < g.rx) return (int)c;
    if (c >= g.cols - g.rx) return 2 * g.rx - (int)(g.cols - 1 - c);
    return g.rx;
}

// (A^T 1) of the four consecutive elements from flat index e0 (they may
// straddle row and field ends); tab is the workgroup's LDS copy of the table
__device__ __forceinline__ void coef4(const ChainGeom& g, const float* tab, int64_t e0,
                                      float (&c)[4]) {
    const uint64_t row = g.by_cols.div((uint64_t)e0);
    int64_t col = e0 - (int64_t)row * g.cols;
    int64_t rl = (int64_t)(row - g.by_rows.div(row) * (uint64_t)g.rows);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const bool in_r = !g.small_r && rl >= g.ry && rl < g.rows - g.ry;
        const bool in_c = !g.small_c && col >= g.rx && col < g.cols - g.rx;
        c[e] = (in_r && in_c) ? g.interior : tab[row_class(g, rl) * g.ncc + col_class(g, col)];
        if (++col == g.cols) {
            col = 0;
            if (++rl == g.rows) rl = 0;
        }
    }
}

__device__ __forceinline__ void load_table(const ChainGeom& g, float* tab) {
    for (int k = threadIdx.x; k < kMaxClasses * kMaxClasses; k += kBlock) tab[k] = g.tab[k];
    __syncthreads();
}

// C1 forward: per-workgroup partial sums of f(x) * (A^T 1); every lane keeps
// kUnroll 16-byte loads in flight, workgroups sweep consecutive chunks
template <int MOP>
__global__ __launch_bounds__(kBlock) void chain_fwd(const float* x, int64_t n, ChainGeom g,
                                                    float p0, float p1, float* partials) {
    __shared__ float tab[kMaxClasses * kMaxClasses];
    __shared__ float lds[kBlock / kWave];
    load_table(g, tab);
    float acc[kUnroll] = {0.0f, 0.0f, 0.0f, 0.0f};
    const f32x4* xv = reinterpret_cast<const f32x4*>(x);
    const int64_t nv = n / 4;
    constexpr int64_t CH = (int64_t)kBlock * kUnroll;
    for (int64_t base = (int64_t)blockIdx.x * CH; base < nv; base += (int64_t)gridDim.x * CH) {
        f32x4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = base + u * kBlock + threadIdx.x;
            v[u] = i < nv ? __builtin_nontemporal_load(&xv[i]) : f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = base + u * kBlock + threadIdx.x;
            if (i >= nv) break;
            float c[4];
            coef4(g, tab, 4 * i, c);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[u] = __builtin_fmaf(fmap<MOP>(v[u][e], 0.0f, p0, p1), c[e], acc[u]);
        }
    }
    // the n % 4 tail: one element per low lane of workgroup 0
    const int64_t t = nv * 4 + threadIdx.x;
    if (blockIdx.x == 0 && t < n) {
        float c[4];
        coef4(g, tab, t, c);
        acc[0] = __builtin_fmaf(fmap<MOP>(x[t], 0.0f, p0, p1), c[0], acc[0]);
    }
    float a = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    a = block_reduce<Comb<float, SKEL_SUM>>(a, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = a;
}

// the partials of `np` sums (np arrays of `groups` values), each combined in
// workgroup order; out[k] = sum of array k, plus add0 for k = 0
__global__ __launch_bounds__(kBlock) void chain_finish(const float* partials, int groups, int np,
                                                       float add0, float* out) {
    __shared__ float lds[kBlock / kWave];
    for (int k = 0; k < np; ++k) {
        float a = 0.0f;
        for (int i = threadIdx.x; i < groups; i += kBlock) a += partials[(int64_t)k * groups + i];
        a = block_reduce<Comb<float, SKEL_SUM>>(a, lds);
        if (threadIdx.x == 0) out[k] = k == 0 ? a + add0 : a;
        __syncthreads();  // lds is reused by the next sum
    }
}

// C1 backward: dx = g1 * (A^T 1) * df/dx, and per-workgroup partials of
// g1 * (A^T 1) * df/dp_k (NP arrays of gridDim.x values)
template <int MOP>
__global__ __launch_bounds__(kBlock) void chain_bwd(const float* x, int64_t n, ChainGeom g,
                                                    float p0, float p1, const float* g1,
                                                    float* dx, float* partials) {
    constexpr int NP = map_nparams<MOP>();
    __shared__ float tab[kMaxClasses * kMaxClasses];
    __shared__ float lds[kBlock / kWave];
    load_table(g, tab);
    const float gv = g1[0];
    float a0 = 0.0f, a1 = 0.0f;
    const f32x4* xv = reinterpret_cast<const f32x4*>(x);
    f32x4* dv = reinterpret_cast<f32x4*>(dx);
    const int64_t nv = n / 4;
    constexpr int64_t CH = (int64_t)kBlock * kUnroll;
    for (int64_t base = (int64_t)blockIdx.x * CH; base < nv; base += (int64_t)gridDim.x * CH) {
        f32x4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = base + u * kBlock + threadIdx.x;
            v[u] = i < nv ? __builtin_nontemporal_load(&xv[i]) : f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = base + u * kBlock + threadIdx.x;
            if (i >= nv) break;
            float c[4];
            coef4(g, tab, 4 * i, c);
            f32x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float ddx, ddy, s0, s1;
                elem_grad<MOP>(v[u][e], 0.0f, gv * c[e], p0, p1, ddx, ddy, s0, s1);
                o[e] = ddx;
                a0 += s0;
                a1 += s1;
            }
            store_vec_nt(o, &dv[i]);
        }
    }
    const int64_t t = nv * 4 + threadIdx.x;
    if (blockIdx.x == 0 && t < n) {
        float c[4];
        coef4(g, tab, t, c);
        float ddx, ddy, s0, s1;
        elem_grad<MOP>(x[t], 0.0f, gv * c[0], p0, p1, ddx, ddy, s0, s1);
        dx[t] = ddx;
        a0 += s0;
        a1 += s1;
    }
    if constexpr (NP > 0) {
        a0 = block_reduce<Comb<float, SKEL_SUM>>(a0, lds);
        if (threadIdx.x == 0) partials[blockIdx.x] = a0;
        __syncthreads();
        if constexpr (NP > 1) {
            a1 = block_reduce<Comb<float, SKEL_SUM>>(a1, lds);
            if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = a1;
        }
    }
}

int grid_for(int64_t n, const DevInfo& d) {
    int64_t g = (n / 4 + (int64_t)kBlock * kUnroll - 1) / ((int64_t)kBlock * kUnroll);
    const int64_t cap = (int64_t)d.cus * 4;
    if (g > cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

ChainGeom geometry(const ChainTable& t) {
    ChainGeom g;
    g.rows = t.rows;
    g.cols = t.cols;
    g.by_cols = make_div((uint64_t)t.cols);
    g.by_rows = make_div((uint64_t)t.rows);
    g.ry = t.ry;
    g.rx = t.rx;
    g.small_r = t.small_r;
    g.small_c = t.small_c;
    g.ncc = t.ncc;
    g.interior = t.interior;
    for (int k = 0; k < kMaxClasses * kMaxClasses; ++k) g.tab[k] = t.tab[k];
    return g;
}

template <int MOP>
skel_status fused_forward(const float* x, int64_t n, const ChainGeom& g, float p0, float p1,
                          float add, float* out, LaunchCtx& lc) {
    const int groups = grid_for(n, *lc.dev);
    void* mem = nullptr;
    skel_status e = ws_scratch(lc, (size_t)groups * sizeof(float), &mem);
    if (e != SKEL_OK) return e;
    float* part = static_cast<float*>(mem);
    chain_fwd<MOP><<<groups, kBlock, 0, lc.stream>>>(x, n, g, p0, p1, part);
    if ((e = launch_check("chain_fwd")) != SKEL_OK) return e;
    chain_finish<<<1, kBlock, 0, lc.stream>>>(part, groups, 1, add, out);
    return launch_check("chain_finish");
}

template <int MOP>
skel_status fused_backward(const float* x, int64_t n, const ChainGeom& g, float p0, float p1,
                           const float* g1, float* dx, float* dparams, LaunchCtx& lc) {
    constexpr int NP = map_nparams<MOP>();
    const int groups = grid_for(n, *lc.dev);
    void* mem = nullptr;
    skel_status e = ws_scratch(lc, (size_t)groups * 2 * sizeof(float), &mem);
    if (e != SKEL_OK) return e;
    float* part = static_cast<float*>(mem);
    chain_bwd<MOP><<<groups, kBlock, 0, lc.stream>>>(x, n, g, p0, p1, g1, dx, part);
    if ((e = launch_check("chain_bwd")) != SKEL_OK) return e;
    if (NP == 0 || !dparams) return SKEL_OK;
    chain_finish<<<1, kBlock, 0, lc.stream>>>(part, groups, NP, 0.0f, dparams);
    return launch_check("chain_finish");
}

// The composed form keeps its two intermediates in the stream's scratch
// buffer past this offset; the skeleton launchers it calls take their own
// partials (at most a few tens of KiB) from the buffer's start.
constexpr size_t kComposedOffset = size_t(1) << 20;

int plan_variant(CallContext c, skel_status* st) { return choose_variant(SKEL_VARIANT_AUTO, c, st); }

}  // namespace

skel_status launch_chain(int variant, int map_op, float p0, float p1, const float* x,
                         int64_t rows, int64_t cols, int64_t fields, const float* w2d,
                         const float* wy, const float* wx, int ry, int rx, int edge, float pad,
                         float* out, LaunchCtx& lc) {
    const int64_t n = fields * rows * cols;
    if (variant == C1_FUSED) {
        ChainTable tb;
        chain_table(rows, cols, fields, w2d, wy, wx, ry, rx, edge, pad, &tb);
        const ChainGeom g = geometry(tb);
        const float add = (float)tb.pad_total;
        switch (map_op) {
        case SKEL_MAP_IDENTITY:
            return fused_forward<SKEL_MAP_IDENTITY>(x, n, g, p0, p1, add, out, lc);
        case SKEL_MAP_AFFINE: return fused_forward<SKEL_MAP_AFFINE>(x, n, g, p0, p1, add, out, lc);
        case SKEL_MAP_TANH: return fused_forward<SKEL_MAP_TANH>(x, n, g, p0, p1, add, out, lc);
        case SKEL_MAP_AFFINE_TANH:
            return fused_forward<SKEL_MAP_AFFINE_TANH>(x, n, g, p0, p1, add, out, lc);
        default: return fused_forward<SKEL_MAP_SQUARE>(x, n, g, p0, p1, add, out, lc);
        }
    }
    // C0: Map into t, the neighbourhood map of every field into s, Reduce s,
    // each step by the variant the plan picks for it alone
    void* mem = nullptr;
    skel_status e = ws_scratch(lc, kComposedOffset + (size_t)n * 2 * sizeof(float), &mem);
    if (e != SKEL_OK) return e;
    float* t = reinterpret_cast<float*>(static_cast<char*>(mem) + kComposedOffset);
    float* s = t + n;
    CallContext cm;
    cm.skeleton = SKEL_SK_MAP;
    cm.n = n;
    cm.op = map_op;
    CallContext co;
    co.skeleton = SKEL_SK_MAPOVERLAP2D;
    co.n = n;
    co.rows = rows;
    co.cols = cols;
    co.separable = w2d ? 0 : 1;
    co.radius = ry > rx ? ry : rx;
    CallContext cr;
    cr.skeleton = SKEL_SK_REDUCE;
    cr.n = n;
    cr.op = SKEL_SUM;
    const int vm = plan_variant(cm, &e);
    if (vm < 0) return e;
    const int vo = plan_variant(co, &e);
    if (vo < 0) return e;
    const int vr = plan_variant(cr, &e);
    if (vr < 0) return e;
    if ((e = launch_map(vm, map_op, p0, p1, x, nullptr, t, n, lc)) != SKEL_OK) return e;
    if ((e = launch_overlap2d(vo, t, s, rows, cols, fields, w2d, w2d ? nullptr : wy,
                              w2d ? nullptr : wx, ry, rx, edge, pad, lc)) != SKEL_OK)
        return e;
    return launch_reduce(vr, SKEL_SUM, SKEL_F32, SKEL_F32, s, n, out, lc);
}

skel_status launch_chain_backward(int variant, int map_op, float p0, float p1, const float* x,
                                  int64_t rows, int64_t cols, int64_t fields, const float* w2d,
                                  const float* wy, const float* wx, int ry, int rx, int edge,
                                  const float* g1, float* dx, float* dparams, LaunchCtx& lc) {
    const int64_t n = fields * rows * cols;
    if (variant == C1_FUSED) {
        ChainTable tb;
        chain_table(rows, cols, fields, w2d, wy, wx, ry, rx, edge, 0.0f, &tb);
        const ChainGeom g = geometry(tb);
        switch (map_op) {
        case SKEL_MAP_IDENTITY:
            return fused_backward<SKEL_MAP_IDENTITY>(x, n, g, p0, p1, g1, dx, dparams, lc);
        case SKEL_MAP_AFFINE:
            return fused_backward<SKEL_MAP_AFFINE>(x, n, g, p0, p1, g1, dx, dparams, lc);
        case SKEL_MAP_TANH:
            return fused_backward<SKEL_MAP_TANH>(x, n, g, p0, p1, g1, dx, dparams, lc);
        case SKEL_MAP_AFFINE_TANH:
            return fused_backward<SKEL_MAP_AFFINE_TANH>(x, n, g, p0, p1, g1, dx, dparams, lc);
        default: return fused_backward<SKEL_MAP_SQUARE>(x, n, g, p0, p1, g1, dx, dparams, lc);
        }
    }
    // C0: the Reduce adjoint (g1 broadcast, as the Map adjoint of the identity),
    // the transposed neighbourhood map, the Map adjoint
    void* mem = nullptr;
    skel_status e = ws_scratch(lc, kComposedOffset + (size_t)n * 2 * sizeof(float), &mem);
    if (e != SKEL_OK) return e;
    float* gs = reinterpret_cast<float*>(static_cast<char*>(mem) + kComposedOffset);
    float* gt = gs + n;
    CallContext ca;
    ca.skeleton = SKEL_SK_MAPOVERLAP2D_BACKWARD;
    ca.n = n;
    ca.rows = rows;
    ca.cols = cols;
    ca.separable = w2d ? 0 : 1;
    ca.radius = ry > rx ? ry : rx;
    const int va = plan_variant(ca, &e);
    if (va < 0) return e;
    if ((e = launch_map_backward(SKEL_MAP_IDENTITY, 0.0f, 0.0f, x, nullptr, g1, true, gs, nullptr,
                                 n, nullptr, lc)) != SKEL_OK)
        return e;
    if ((e = launch_overlap2d_adjoint(va, gs, gt, rows, cols, fields, w2d, w2d ? nullptr : wy,
                                      w2d ? nullptr : wx, ry, rx, edge, lc)) != SKEL_OK)
        return e;
    return launch_map_backward(map_op, p0, p1, x, nullptr, gt, false, dx, nullptr, n, dparams,
                               lc);
}

}  // namespace skel
