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
#ifndef SKEL_CHAIN_UNROLL
#define SKEL_CHAIN_UNROLL 4
#endif
constexpr int kUnroll = SKEL_CHAIN_UNROLL;  // 16-byte loads in flight per lane and chunk
constexpr int kMaxClasses = kChainMaxClasses;

// Unsigned division by a divisor fixed for the whole launch, as a multiply-high
// and shifts (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994, unsigned case): l = ceil(log2 d),
// m = floor(2^W (2^l - d) / d) + 1, q = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0)
// with t = mulhi(m, n).  Exact for every W-bit n and 1 <= d < 2^(W-1).
template <class T>
struct DivU {
    T m;
    int s1, s2;
    __device__ __forceinline__ T div(T n) const {
        T t;
        if constexpr (sizeof(T) == 4) t = __umulhi(m, n);
        else t = __umul64hi(m, n);
        return (t + ((n - t) >> s1)) >> s2;
    }
};

template <class T>
DivU<T> make_div(uint64_t d) {
    constexpr int W = 8 * sizeof(T);
    int l = 0;
    while (l < W - 1 && (UINT64_C(1) << l) < d) ++l;
    const unsigned __int128 num = (unsigned __int128)((UINT64_C(1) << l) - d) << W;
    DivU<T> r;
    r.m = (T)(num / d + 1);
    r.s1 = l < 1 ? l : 1;
    r.s2 = l > 1 ? l - 1 : 0;
    return r;
}

// What the kernels need to weigh an element: the field shape, the dividers
// that locate a flat index in its field (T: 32-bit indices when the array
// has fewer than 2^32 elements, else 64-bit), and the (A^T 1) table of
// chain_table.hpp (row classes, column classes, the interior entry).
template <class T>
struct ChainGeom {
    T rows, cols;
    DivU<T> by_cols, by_rows;  // element index -> row; row -> field
    // a lane's position moves by kBlock * 4 elements from one vector of a
    // chunk to the next, and by the grid's stride from one chunk to the next:
    // each step as (columns mod cols, rows mod rows) -- see advance()
    T vec_c, vec_r, chunk_c, chunk_r;
    int ry, rx;
    int inner_ok;              // the field has interior rows and columns
    int small_r, small_c;      // fewer than 2r + 1 rows / columns
    int ncc;                   // column classes (table row length)
    float interior;            // the table's interior entry (the weight sum)
    float tab[kMaxClasses * kMaxClasses];
};

template <class T>
__device__ __forceinline__ int row_class(const ChainGeom<T>& g, T r) {
    if (g.small_r || r < (T)g.ry) return (int)r;
    if (r >= g.rows - g.ry) return 2 * g.ry - (int)(g.rows - 1 - r);
    return g.ry;
}
template <class T>
__device__ __forceinline__ int col_class(const ChainGeom<T>& g, T c) {
    if (g.small_c || c < (T)g.rx) return (int)c;
    if (c >= g.cols - g.rx) return 2 * g.rx - (int)(g.cols - 1 - c);
    return g.rx;
}

// (row within its field, column) of flat element index e: two divisions by
// invariant integers (each a multiply-high, a quarter-rate instruction)
template <class T>
__device__ __forceinline__ void locate(const ChainGeom<T>& g, T e, T& rl, T& col) {
    const T row = g.by_cols.div(e);
    col = e - row * g.cols;
    rl = row - g.by_rows.div(row) * g.rows;
}

// Move (rl, col) forward by a fixed number of elements given as (dc, dr) =
// (that number mod cols, (that number div cols) mod rows).  col + dc < 2 cols
// and rl + dr + 1 < 2 rows, so one conditional subtraction wraps each: adds,
// compares and selects instead of the divisions of locate().
template <class T>
__device__ __forceinline__ void advance(const ChainGeom<T>& g, T dc, T dr, T& rl, T& col) {
    col += dc;
    const bool wrap = col >= g.cols;
    col = wrap ? col - g.cols : col;
    rl += dr + (wrap ? (T)1 : (T)0);
    rl = rl >= g.rows ? rl - g.rows : rl;
}

// (A^T 1) of the four consecutive elements from (rl, col).  Inside a field
// (the common case) all four take the interior entry; a vector that touches a
// border band, or straddles a row or field end, looks each element up in the
// workgroup's LDS copy of the table.
template <class T>
__device__ __forceinline__ void coef4(const ChainGeom<T>& g, const float (&tab)[kMaxClasses * kMaxClasses],
                                      T rl, T col, float (&c)[4]) {
    const bool inner = g.inner_ok && rl >= (T)g.ry && rl < g.rows - g.ry && col >= (T)g.rx &&
                       col + 3 + g.rx < g.cols;
    if (inner) {
#pragma unroll
        for (int e = 0; e < 4; ++e) c[e] = g.interior;
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        c[e] = tab[row_class(g, rl) * g.ncc + col_class(g, col)];
        if (++col == g.cols) {
            col = 0;
            if (++rl == g.rows) rl = 0;
        }
    }
}

template <class T>
__device__ __forceinline__ void load_table(const ChainGeom<T>& g,
                                           float (&tab)[kMaxClasses * kMaxClasses]) {
    for (int k = threadIdx.x; k < kMaxClasses * kMaxClasses; k += kBlock) tab[k] = g.tab[k];
    __syncthreads();
}

// tanh from the identity tanh(a) = (1 - e^-2a) / (1 + e^-2a) for a = |y| with
// the hardware base-2 exponential and reciprocal, and the odd Taylor series
// y - y^3/3 + 2y^5/15 below |y| = 1/16 (truncation under 2^-27 relative
// there, where the quotient would lose digits to cancellation); absolute
// error about 1e-7 everywhere, saturating to +-1 without overflow
__device__ __forceinline__ float tanh_fast(float y) {
    const float a = __builtin_fabsf(y);
    const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * a);  // e^-2a, 2 log2(e) a
    const float q = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
    const float y2 = y * y;
    const float p = y * __builtin_fmaf(y2, __builtin_fmaf(y2, 0.13333333333f, -0.33333333333f), 1.0f);
    return a < 0.0625f ? p : __builtin_copysignf(q, y);
}

// the chain's element function (one input), tanh by tanh_fast
template <int MOP>
__device__ __forceinline__ float chain_f(float x, float p0, float p1) {
    if constexpr (MOP == SKEL_MAP_TANH) return tanh_fast(x);
    else if constexpr (MOP == SKEL_MAP_AFFINE_TANH) return tanh_fast(__builtin_fmaf(p0, x, p1));
    else return fmap<MOP>(x, 0.0f, p0, p1);
}

// g * (df/dx, df/dp0, df/dp1) of the chain's element function
template <int MOP>
__device__ __forceinline__ void chain_grad(float x, float g, float p0, float p1, float& dx,
                                           float& s0, float& s1) {
    s0 = 0.0f;
    s1 = 0.0f;
    if constexpr (MOP == SKEL_MAP_TANH) {
        const float t = tanh_fast(x);
        dx = g * (1.0f - t * t);
    } else if constexpr (MOP == SKEL_MAP_AFFINE_TANH) {
        const float t = tanh_fast(__builtin_fmaf(p0, x, p1));
        const float gd = g * (1.0f - t * t);
        dx = gd * p0;
        s0 = gd * x;
        s1 = gd;
    } else {
        float dy;
        elem_grad<MOP>(x, 0.0f, g, p0, p1, dx, dy, s0, s1);
    }
}

// the kUnroll vectors of one lane in the chunk at vector index `base`
template <class T>
__device__ __forceinline__ void load_chunk(const f32x4* xv, T nv, T base, f32x4 (&v)[kUnroll]) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const T i = base + u * kBlock + threadIdx.x;
        v[u] = i < nv ? __builtin_nontemporal_load(&xv[i]) : f32x4{0.f, 0.f, 0.f, 0.f};
    }
}

// C1 forward: per-workgroup partial sums of f(x) * (A^T 1); every lane keeps
// kUnroll 16-byte loads in flight, workgroups sweep consecutive chunks
template <int MOP, class T>
__global__ __launch_bounds__(kBlock) void chain_fwd(const float* x, T n, ChainGeom<T> g,
                                                    float p0, float p1, float* partials) {
    __shared__ float tab[kMaxClasses * kMaxClasses];
    __shared__ float lds[kBlock / kWave];
    load_table(g, tab);
    float acc[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc[u] = 0.0f;
    const f32x4* xv = reinterpret_cast<const f32x4*>(x);
    const T nv = n / 4;
    constexpr T CH = (T)kBlock * kUnroll;
    const T stride = (T)gridDim.x * CH;
    // the next chunk's loads are issued before this chunk's arithmetic, so
    // the memory system stays busy while the lanes compute
    f32x4 v[kUnroll];
    load_chunk(xv, nv, (T)blockIdx.x * CH, v);
    // the lane's position at its first vector of each chunk
    T rl0 = 0, col0 = 0;
    if ((T)blockIdx.x * CH + threadIdx.x < nv)
        locate(g, 4 * ((T)blockIdx.x * CH + threadIdx.x), rl0, col0);
    for (T base = (T)blockIdx.x * CH; base < nv; base += stride) {
        f32x4 cur[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) cur[u] = v[u];
        if (base + stride < nv) load_chunk(xv, nv, base + stride, v);
        T rl = rl0, col = col0;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const T i = base + u * kBlock + threadIdx.x;
            if (i >= nv) break;
            float c[4];
            coef4(g, tab, rl, col, c);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc[u] = __builtin_fmaf(chain_f<MOP>(cur[u][e], p0, p1), c[e], acc[u]);
            advance(g, g.vec_c, g.vec_r, rl, col);
        }
        advance(g, g.chunk_c, g.chunk_r, rl0, col0);
    }
    // the n % 4 tail: one element per low lane of workgroup 0
    const T t = nv * 4 + threadIdx.x;
    if (blockIdx.x == 0 && t < n) {
        float c[4];
        T rl, col;
        locate(g, t, rl, col);
        coef4(g, tab, rl, col, c);
        acc[0] = __builtin_fmaf(chain_f<MOP>(x[t], p0, p1), c[0], acc[0]);
    }
    float a = 0.0f;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) a += acc[u];
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
template <int MOP, class T>
__global__ __launch_bounds__(kBlock) void chain_bwd(const float* x, T n, ChainGeom<T> g,
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
    const T nv = n / 4;
    constexpr T CH = (T)kBlock * kUnroll;
    const T stride = (T)gridDim.x * CH;
    f32x4 v[kUnroll];
    load_chunk(xv, nv, (T)blockIdx.x * CH, v);
    T rl0 = 0, col0 = 0;
    if ((T)blockIdx.x * CH + threadIdx.x < nv)
        locate(g, 4 * ((T)blockIdx.x * CH + threadIdx.x), rl0, col0);
    for (T base = (T)blockIdx.x * CH; base < nv; base += stride) {
        f32x4 cur[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) cur[u] = v[u];
        if (base + stride < nv) load_chunk(xv, nv, base + stride, v);
        T rl = rl0, col = col0;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const T i = base + u * kBlock + threadIdx.x;
            if (i >= nv) break;
            float c[4];
            coef4(g, tab, rl, col, c);
            advance(g, g.vec_c, g.vec_r, rl, col);
            f32x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float d, s0, s1;
                chain_grad<MOP>(cur[u][e], gv * c[e], p0, p1, d, s0, s1);
                o[e] = d;
                a0 += s0;
                a1 += s1;
            }
            store_vec_nt(o, &dv[i]);
        }
    }
    const T t = nv * 4 + threadIdx.x;
    if (blockIdx.x == 0 && t < n) {
        float c[4];
        T rl, col;
        locate(g, t, rl, col);
        coef4(g, tab, rl, col, c);
        float o, s0, s1;
        chain_grad<MOP>(x[t], gv * c[0], p0, p1, o, s0, s1);
        dx[t] = o;
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

#ifndef SKEL_CHAIN_GROUPS_PER_CU
#define SKEL_CHAIN_GROUPS_PER_CU 16
#endif

// one chunk of kBlock * kUnroll vectors per workgroup at least, at most
// SKEL_CHAIN_GROUPS_PER_CU workgroups per CU (the element function's
// arithmetic needs more waves in flight than a plain reduction)
int grid_for(int64_t n, const DevInfo& d) {
    int64_t g = (n / 4 + (int64_t)kBlock * kUnroll - 1) / ((int64_t)kBlock * kUnroll);
    const int64_t cap = (int64_t)d.cus * SKEL_CHAIN_GROUPS_PER_CU;
    if (g > cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

template <class T>
ChainGeom<T> geometry(const ChainTable& t, int groups) {
    ChainGeom<T> g;
    g.rows = (T)t.rows;
    g.cols = (T)t.cols;
    // element steps between a lane's vectors (kBlock vectors of 4) and
    // between its chunks (the grid's stride), as (mod cols, div cols mod rows)
    const uint64_t vstep = (uint64_t)kBlock * 4;
    const uint64_t cstep = (uint64_t)groups * kBlock * kUnroll * 4;
    g.vec_c = (T)(vstep % t.cols);
    g.vec_r = (T)((vstep / t.cols) % t.rows);
    g.chunk_c = (T)(cstep % t.cols);
    g.chunk_r = (T)((cstep / t.cols) % t.rows);
    g.by_cols = make_div<T>((uint64_t)t.cols);
    g.by_rows = make_div<T>((uint64_t)t.rows);
    g.ry = t.ry;
    g.rx = t.rx;
    g.small_r = t.small_r;
    g.small_c = t.small_c;
    g.inner_ok = !t.small_r && !t.small_c;
    g.ncc = t.ncc;
    g.interior = t.interior;
    for (int k = 0; k < kMaxClasses * kMaxClasses; ++k) g.tab[k] = t.tab[k];
    return g;
}

template <int MOP, class T>
skel_status fused_forward(const float* x, int64_t n, const ChainTable& tb, float p0, float p1,
                          float* out, LaunchCtx& lc) {
    const int groups = grid_for(n, *lc.dev);
    void* mem = nullptr;
    skel_status e = ws_scratch(lc, (size_t)groups * sizeof(float), &mem);
    if (e != SKEL_OK) return e;
    float* part = static_cast<float*>(mem);
    chain_fwd<MOP, T><<<groups, kBlock, 0, lc.stream>>>(x, (T)n, geometry<T>(tb, groups), p0, p1,
                                                       part);
    if ((e = launch_check("chain_fwd")) != SKEL_OK) return e;
    chain_finish<<<1, kBlock, 0, lc.stream>>>(part, groups, 1, (float)tb.pad_total, out);
    return launch_check("chain_finish");
}

template <int MOP, class T>
skel_status fused_backward(const float* x, int64_t n, const ChainTable& tb, float p0, float p1,
                           const float* g1, float* dx, float* dparams, LaunchCtx& lc) {
    constexpr int NP = map_nparams<MOP>();
    const int groups = grid_for(n, *lc.dev);
    void* mem = nullptr;
    skel_status e = ws_scratch(lc, (size_t)groups * 2 * sizeof(float), &mem);
    if (e != SKEL_OK) return e;
    float* part = static_cast<float*>(mem);
    chain_bwd<MOP, T><<<groups, kBlock, 0, lc.stream>>>(x, (T)n, geometry<T>(tb, groups), p0, p1,
                                                       g1, dx, part);
    if ((e = launch_check("chain_bwd")) != SKEL_OK) return e;
    if (NP == 0 || !dparams) return SKEL_OK;
    chain_finish<<<1, kBlock, 0, lc.stream>>>(part, groups, NP, 0.0f, dparams);
    return launch_check("chain_finish");
}

// 32-bit index arithmetic when every flat index fits
template <int MOP>
skel_status fused_forward_any(const float* x, int64_t n, const ChainTable& tb, float p0, float p1,
                              float* out, LaunchCtx& lc) {
    if (n < (INT64_C(1) << 32) - 4)
        return fused_forward<MOP, uint32_t>(x, n, tb, p0, p1, out, lc);
    return fused_forward<MOP, uint64_t>(x, n, tb, p0, p1, out, lc);
}

template <int MOP>
skel_status fused_backward_any(const float* x, int64_t n, const ChainTable& tb, float p0,
                               float p1, const float* g1, float* dx, float* dparams,
                               LaunchCtx& lc) {
    if (n < (INT64_C(1) << 32) - 4)
        return fused_backward<MOP, uint32_t>(x, n, tb, p0, p1, g1, dx, dparams, lc);
    return fused_backward<MOP, uint64_t>(x, n, tb, p0, p1, g1, dx, dparams, lc);
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
        switch (map_op) {
        case SKEL_MAP_IDENTITY:
            return fused_forward_any<SKEL_MAP_IDENTITY>(x, n, tb, p0, p1, out, lc);
        case SKEL_MAP_AFFINE: return fused_forward_any<SKEL_MAP_AFFINE>(x, n, tb, p0, p1, out, lc);
        case SKEL_MAP_TANH: return fused_forward_any<SKEL_MAP_TANH>(x, n, tb, p0, p1, out, lc);
        case SKEL_MAP_AFFINE_TANH:
            return fused_forward_any<SKEL_MAP_AFFINE_TANH>(x, n, tb, p0, p1, out, lc);
        default: return fused_forward_any<SKEL_MAP_SQUARE>(x, n, tb, p0, p1, out, lc);
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
        switch (map_op) {
        case SKEL_MAP_IDENTITY:
            return fused_backward_any<SKEL_MAP_IDENTITY>(x, n, tb, p0, p1, g1, dx, dparams, lc);
        case SKEL_MAP_AFFINE:
            return fused_backward_any<SKEL_MAP_AFFINE>(x, n, tb, p0, p1, g1, dx, dparams, lc);
        case SKEL_MAP_TANH:
            return fused_backward_any<SKEL_MAP_TANH>(x, n, tb, p0, p1, g1, dx, dparams, lc);
        case SKEL_MAP_AFFINE_TANH:
            return fused_backward_any<SKEL_MAP_AFFINE_TANH>(x, n, tb, p0, p1, g1, dx, dparams, lc);
        default:
            return fused_backward_any<SKEL_MAP_SQUARE>(x, n, tb, p0, p1, g1, dx, dparams, lc);
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
