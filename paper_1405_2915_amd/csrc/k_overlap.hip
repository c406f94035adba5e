// MapOverlap skeleton kernels: a map whose element function sees a
// neighbourhood (Section III lists mapoverlap among the data-parallel
// skeletons).  Here the neighbourhood function is a linear weighting in
// correlation orientation:
//   1D  out[i]    = sum_k w[k] * x[e(i + k - r)]
//   2D  out[i][j] = sum_a sum_b W[a][b] * x[e(i + a - ry)][e(j + b - rx)]
// with e() the border rule (clamp, constant pad, cyclic).
//
// Variants:
//   O1a  1D direct: one output per lane, taps read through the caches
//   O1b  1D LDS tile: a workgroup stages 1024 + 2r inputs once, each lane
//        computes four outputs from registers
//   O1c  1D cross-lane: r <= 4 neighbours come from adjacent lanes by
//        shuffles; no LDS, no barrier
//   O2a  2D direct: one output per lane, (2ry+1)(2rx+1) taps from global
//   O2b  2D LDS tile: a 64x64 output tile plus halo staged in LDS with 16-byte
//        loads; each lane computes a 4x4 output block, reusing every loaded
//        row segment for up to four output rows
//   O2c  2D separable (W = wy (x) wx): the staged tile is filtered along rows
//        into a second LDS buffer, then along columns; 2(2r+1) instead of
//        (2r+1)^2 multiply-adds per output
//   O2d  2D separable with the row pass read from global memory through L1
//        and only its result staged in LDS (64x32 tiles, full occupancy)
//   O2e  2D marching window (ry, rx <= 4): each wavefront walks down a strip
//        of 256 columns, loading every input row once; horizontal neighbours
//        come from the adjacent lanes by DPP moves and the 2ry+1 output rows
//        a loaded row feeds are kept in a ring of registers.  No LDS, no
//        barrier.
// 2D tiles are visited in an XCD-aware order: consecutive workgroups go to
// different XCDs round-robin, so tile ids are remapped to give each XCD a
// contiguous band of tiles whose shared halo rows stay in that XCD's L2.
#include "kcommon.hpp"
#include "dispatch.hpp"
#include "launch.hpp"

namespace skel {
namespace {

using dev::f32x4;

struct W1 {
    float w[2 * SKEL_MAX_RADIUS_1D + 1];
};
struct W2 {
    float w[(2 * SKEL_MAX_RADIUS_2D + 1) * (2 * SKEL_MAX_RADIUS_2D + 1)];
    float wy[2 * SKEL_MAX_RADIUS_2D + 1];
    float wx[2 * SKEL_MAX_RADIUS_2D + 1];
};

// border rule: true and the index to read, or false for the constant pad
__device__ __forceinline__ bool border(int64_t j, int64_t n, int edge, int64_t& k) {
    if (j >= 0 && j < n) {
        k = j;
        return true;
    }
    if (edge == SKEL_EDGE_CLAMP) {
        k = j < 0 ? 0 : n - 1;
        return true;
    }
    if (edge == SKEL_EDGE_CYCLIC) {
        int64_t m = j % n;
        k = m < 0 ? m + n : m;
        return true;
    }
    return false;
}

__device__ __forceinline__ float fetch1(const float* x, int64_t n, int64_t j, int edge,
                                        float pad) {
    int64_t k;
    return border(j, n, edge, k) ? x[k] : pad;
}

__device__ __forceinline__ float fetch2(const float* x, int64_t rows, int64_t cols, int64_t i,
                                        int64_t j, int edge, float pad) {
    int64_t a, b;
    if (!border(i, rows, edge, a) || !border(j, cols, edge, b)) return pad;
    return x[a * cols + b];
}

constexpr int kBlock = 256;

// ------------------------------------------------------------------- 1D
template <int RT>
__global__ __launch_bounds__(kBlock) void ov1_direct(const float* x, float* out, int64_t n,
                                                     W1 w, int r_, int edge, float pad) {
    const int r = RT >= 0 ? RT : r_;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float acc = 0.0f;
    if (i - r >= 0 && i + r < n) {
#pragma unroll
        for (int k = 0; k <= 2 * (RT >= 0 ? RT : SKEL_MAX_RADIUS_1D); ++k) {
            if (k > 2 * r) break;
            acc = __builtin_fmaf(w.w[k], x[i + k - r], acc);
        }
    } else {
        for (int k = 0; k <= 2 * r; ++k)
            acc = __builtin_fmaf(w.w[k], fetch1(x, n, i + k - r, edge, pad), acc);
    }
    out[i] = acc;
}

constexpr int kT1 = kBlock * 4;  // outputs per workgroup

template <int RT>
__global__ __launch_bounds__(kBlock) void ov1_lds(const float* x, float* out, int64_t n, W1 w,
                                                  int r_, int edge, float pad) {
    constexpr int MR = RT >= 0 ? RT : SKEL_MAX_RADIUS_1D;
    const int r = RT >= 0 ? RT : r_;
    __shared__ float s[kT1 + 2 * MR];
    const int64_t base = (int64_t)blockIdx.x * kT1;
    for (int k = threadIdx.x; k < kT1 + 2 * r; k += kBlock) {
        const int64_t j = base - r + k;
        s[k] = (j >= 0 && j < n) ? x[j] : fetch1(x, n, j, edge, pad);
    }
    __syncthreads();
    const int o = threadIdx.x * 4;
    float win[4 + 2 * MR];
#pragma unroll
    for (int k = 0; k < 4 + 2 * MR; ++k)
        if (k < 4 + 2 * r) win[k] = s[o + k];
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k <= 2 * MR; ++k) {
        if (k > 2 * r) break;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_fmaf(w.w[k], win[c + k], acc[c]);
    }
    const int64_t i = base + o;
    if (i + 4 <= n && (n & 3) == 0) {
        *reinterpret_cast<f32x4*>(out + i) = f32x4{acc[0], acc[1], acc[2], acc[3]};
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (i + c < n) out[i + c] = acc[c];
    }
}

// O1c: no LDS and no barrier.  Each wavefront owns kShflRows consecutive rows
// of 256 outputs (one 16-byte vector per lane per row, every row's load
// issued before any arithmetic); the r <= 4 neighbours on either side of a
// lane's vector come from the adjacent lanes by cross-lane shuffles, a row's
// end lanes take theirs from the adjacent row's end lane, and the first and
// last lanes of the group read one extra vector each (from cache).  Groups
// that touch the array ends take the scalar path.
// rows of 64 vectors per wavefront: one measured fastest in the bench step
// (5-point stencil on 2^26 floats: 103 us with one row, 112 with two or four,
// 123 with eight); more rows mean fewer, longer-lived wavefronts
#ifndef SKEL_O1C_ROWS
#define SKEL_O1C_ROWS 1
#endif
constexpr int kShflRows = SKEL_O1C_ROWS;

template <int RT>
__global__ __launch_bounds__(kBlock) void ov1_shfl(const float* x, float* out, int64_t n, W1 w,
                                                   int r_, int edge, float pad) {
    constexpr int MR = RT >= 0 ? RT : 4;
    constexpr int U = kShflRows;
    const int r = RT >= 0 ? RT : r_;
    const int l = dev::lane();
    // this wavefront's U consecutive rows of 64 x 4 elements
    const int64_t wb0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x - l) * 4 * U;
    if (wb0 >= n) return;
    const bool interior = wb0 - 4 >= 0 && wb0 + 4 * dev::kWave * U + 4 <= n;
    if (interior) {
        const f32x4* xv = reinterpret_cast<const f32x4*>(x + wb0);
        f32x4 c[U];
#pragma unroll
        for (int k = 0; k < U; ++k) c[k] = xv[k * dev::kWave + l];  // all loads in flight
        f32x4 edge_l = {0.f, 0.f, 0.f, 0.f}, edge_r = {0.f, 0.f, 0.f, 0.f};
        if (l == 0) edge_l = xv[-1];
        if (l == dev::kWave - 1) edge_r = xv[U * dev::kWave];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            // neighbours: adjacent lanes of the same row; at the row ends, the
            // adjacent row's end lane (or the extra halo vectors)
            const f32x4 prev = k > 0 ? c[k - 1] : edge_l;
            const f32x4 next = k + 1 < U ? c[k + 1] : edge_r;
            // register-only moves: lane 0 takes the previous row's last vector
            // (or the halo), lane 63 the next row's first (or the halo)
            const f32x4 lt = dev::wave_shift_up(
                c[k], k > 0 ? dev::lane_value(prev, dev::kWave - 1) : edge_l);
            const f32x4 rt = dev::wave_shift_down(c[k], k + 1 < U ? dev::lane_value(next, 0)
                                                                  : edge_r);
            const float v[12] = {lt.x, lt.y, lt.z, lt.w, c[k].x, c[k].y, c[k].z, c[k].w,
                                 rt.x, rt.y, rt.z, rt.w};
            float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk <= 2 * MR; ++kk) {
                if (kk > 2 * r) break;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[q] = __builtin_fmaf(w.w[kk], v[4 + q + kk - r], acc[q]);
            }
            // plain store: measured faster than non-temporal here (5-point
            // stencil on 2^26 floats: 96 us against 103 us)
            reinterpret_cast<f32x4*>(out + wb0)[k * dev::kWave + l] =
                f32x4{acc[0], acc[1], acc[2], acc[3]};
        }
    } else {
        for (int k = 0; k < U; ++k) {
            const int64_t wb = wb0 + (int64_t)k * 4 * dev::kWave;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t i = wb + 4 * l + q;
                if (i >= n) break;
                float acc = 0.0f;
                for (int kk = 0; kk <= 2 * r; ++kk)
                    acc = __builtin_fmaf(w.w[kk], fetch1(x, n, i + kk - r, edge, pad), acc);
                out[i] = acc;
            }
        }
    }
}

// ------------------------------------------------------------------- 2D
constexpr int kTX = 64, kTY = 64;  // output tile of the LDS variants

// compile-time radii, or (-1, -1) for any radius up to the maximum
template <int RY, int RX>
struct Rad {
    static constexpr bool dyn = RY < 0;
    static constexpr int MY = dyn ? SKEL_MAX_RADIUS_2D : RY;
    static constexpr int MX = dyn ? SKEL_MAX_RADIUS_2D : RX;
    static constexpr int HX = (MX + 3) / 4 * 4;  // column halo rounded to 16 bytes
    static constexpr int LW = kTX + 2 * HX;      // LDS row width of the input tile
    static constexpr int LH = kTY + 2 * MY;      // LDS rows of the input tile
};

// tile id -> (tile x, tile y) with an XCD-contiguous order
__device__ __forceinline__ void tile_coords(int64_t nbx, int64_t nb, int64_t& bx, int64_t& by) {
    int64_t b = blockIdx.x, L = b;
    if ((nb & 7) == 0) L = (b & 7) * (nb >> 3) + (b >> 3);
    bx = L % nbx;
    by = L / nbx;
}

// Stage rows [y0 - ry, y0 + kTY + ry) and columns [x0 - HX, x0 + kTX + HX) of
// the input into LDS (row stride Rad::LW).
template <class RD>
__device__ __forceinline__ void stage_tile(const float* x, int64_t rows, int64_t cols,
                                           int64_t y0, int64_t x0, int ry, int edge, float pad,
                                           float* tin) {
    constexpr int LW = RD::LW, HX = RD::HX, V = LW / 4;
    const int nrows = kTY + 2 * ry;
    const bool interior = y0 - ry >= 0 && y0 + kTY + ry <= rows && x0 - HX >= 0 &&
                          x0 + kTX + HX <= cols && (cols & 3) == 0;
    if (interior) {
        const float* src = x + (y0 - ry) * cols + (x0 - HX);
        for (int k = threadIdx.x; k < nrows * V; k += kBlock) {
            const int rr = k / V, cc = k - rr * V;
            f32x4 v = *reinterpret_cast<const f32x4*>(src + (int64_t)rr * cols + 4 * cc);
            *reinterpret_cast<f32x4*>(tin + rr * LW + 4 * cc) = v;
        }
    } else {
        for (int k = threadIdx.x; k < nrows * LW; k += kBlock) {
            const int rr = k / LW, cc = k - rr * LW;
            tin[rr * LW + cc] = fetch2(x, rows, cols, y0 - ry + rr, x0 - HX + cc, edge, pad);
        }
    }
}

template <int RY, int RX>
__global__ __launch_bounds__(kBlock) void ov2_direct(const float* x, float* out, int64_t rows,
                                                     int64_t cols, W2 w, int ry_, int rx_,
                                                     int edge, float pad, int64_t nbx) {
    // blockIdx.y: one of several equally shaped images stored back to back
    x += (int64_t)blockIdx.y * rows * cols;
    out += (int64_t)blockIdx.y * rows * cols;
    using RD = Rad<RY, RX>;
    const int ry = RD::dyn ? ry_ : RY, rx = RD::dyn ? rx_ : RX;
    const int wx = 2 * rx + 1;
    const int64_t j = (blockIdx.x % nbx) * 64 + threadIdx.x % 64;
    const int64_t i = (blockIdx.x / nbx) * 4 + threadIdx.x / 64;
    if (i >= rows || j >= cols) return;
    float acc = 0.0f;
    const bool interior = i - ry >= 0 && i + ry < rows && j - rx >= 0 && j + rx < cols;
#pragma unroll
    for (int a = 0; a <= 2 * RD::MY; ++a) {
        if (a > 2 * ry) break;
#pragma unroll
        for (int b = 0; b <= 2 * RD::MX; ++b) {
            if (b > 2 * rx) break;
            const float v = interior ? x[(i + a - ry) * cols + (j + b - rx)]
                                     : fetch2(x, rows, cols, i + a - ry, j + b - rx, edge, pad);
            acc = __builtin_fmaf(w.w[a * wx + b], v, acc);
        }
    }
    out[i * cols + j] = acc;
}

// store one 4-wide output segment of row i starting at column j
__device__ __forceinline__ void store4(float* out, int64_t rows, int64_t cols, int64_t i,
                                       int64_t j, const float (&v)[4]) {
    if (i >= rows) return;
    if (j + 4 <= cols && (cols & 3) == 0) {
        // non-temporal: measured faster than plain stores for the 2D tiles
        // (9x9 separable on 4096^2: 42 us against 46 us)
        dev::store_vec_nt(f32x4{v[0], v[1], v[2], v[3]},
                          reinterpret_cast<f32x4*>(out + i * cols + j));
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (j + c < cols) out[i * cols + j + c] = v[c];
    }
}

template <int RY, int RX>
__global__ __launch_bounds__(kBlock) void ov2_lds(const float* x, float* out, int64_t rows,
                                                  int64_t cols, W2 w, int ry_, int rx_, int edge,
                                                  float pad, int64_t nbx, int64_t nb) {
    // blockIdx.y: one of several equally shaped images stored back to back
    x += (int64_t)blockIdx.y * rows * cols;
    out += (int64_t)blockIdx.y * rows * cols;
    using RD = Rad<RY, RX>;
    constexpr int LW = RD::LW, HX = RD::HX, MY = RD::MY, MX = RD::MX;
    const int ry = RD::dyn ? ry_ : RY, rx = RD::dyn ? rx_ : RX;
    const int wx = 2 * rx + 1;
    __shared__ __attribute__((aligned(16))) float tin[RD::LH * LW];
    int64_t bx, by;
    tile_coords(nbx, nb, bx, by);
    const int64_t y0 = by * kTY, x0 = bx * kTX;
    stage_tile<RD>(x, rows, cols, y0, x0, ry, edge, pad, tin);
    __syncthreads();
    const int cg = threadIdx.x % 16, rg = threadIdx.x / 16;
    float acc[4][4];
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[o][c] = 0.0f;
    const int c0 = 4 * cg + HX - rx;  // LDS column of tap b = 0 for output column 0
    // input row k of the block's window contributes to output row o with a = k - o
#pragma unroll
    for (int k = 0; k < 4 + 2 * MY; ++k) {
        if (k >= 4 + 2 * ry) break;
        float seg[4 + 2 * MX];
        const float* row = tin + (4 * rg + k) * LW + c0;
#pragma unroll
        for (int t = 0; t < 4 + 2 * MX; ++t)
            if (t < 4 + 2 * rx) seg[t] = row[t];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int a = k - o;
            if (a < 0 || a > 2 * ry) continue;
#pragma unroll
            for (int b = 0; b <= 2 * MX; ++b) {
                if (b > 2 * rx) break;
                const float wab = w.w[a * wx + b];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[o][c] = __builtin_fmaf(wab, seg[c + b], acc[o][c]);
            }
        }
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) store4(out, rows, cols, y0 + 4 * rg + o, x0 + 4 * cg, acc[o]);
}

template <int RY, int RX>
__global__ __launch_bounds__(kBlock) void ov2_sep(const float* x, float* out, int64_t rows,
                                                  int64_t cols, W2 w, int ry_, int rx_, int edge,
                                                  float pad, int64_t nbx, int64_t nb) {
    // blockIdx.y: one of several equally shaped images stored back to back
    x += (int64_t)blockIdx.y * rows * cols;
    out += (int64_t)blockIdx.y * rows * cols;
    using RD = Rad<RY, RX>;
    constexpr int LW = RD::LW, HX = RD::HX, MY = RD::MY, MX = RD::MX;
    constexpr int HW = kTX + 4;  // row-pass buffer stride (padded)
    const int ry = RD::dyn ? ry_ : RY, rx = RD::dyn ? rx_ : RX;
    __shared__ __attribute__((aligned(16))) float tin[RD::LH * LW];
    __shared__ __attribute__((aligned(16))) float th[RD::LH * HW];
    int64_t bx, by;
    tile_coords(nbx, nb, bx, by);
    const int64_t y0 = by * kTY, x0 = bx * kTX;
    stage_tile<RD>(x, rows, cols, y0, x0, ry, edge, pad, tin);
    __syncthreads();
    const int cg = threadIdx.x % 16, rg = threadIdx.x / 16;
    // row pass: th[y][x] = sum_b wx[b] * in[y][x + b - rx] for all staged rows
    const int nrows = kTY + 2 * ry;
    for (int y = rg; y < nrows; y += 16) {
        const float* row = tin + y * LW + 4 * cg + HX - rx;
        float seg[4 + 2 * MX];
#pragma unroll
        for (int t = 0; t < 4 + 2 * MX; ++t)
            if (t < 4 + 2 * rx) seg[t] = row[t];
        float h[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b <= 2 * MX; ++b) {
            if (b > 2 * rx) break;
#pragma unroll
            for (int c = 0; c < 4; ++c) h[c] = __builtin_fmaf(w.wx[b], seg[c + b], h[c]);
        }
        *reinterpret_cast<f32x4*>(th + y * HW + 4 * cg) = f32x4{h[0], h[1], h[2], h[3]};
    }
    __syncthreads();
    // column pass: out[y][x] = sum_a wy[a] * th[y + a][x]
    float acc[4][4];
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[o][c] = 0.0f;
#pragma unroll
    for (int k = 0; k < 4 + 2 * MY; ++k) {
        if (k >= 4 + 2 * ry) break;
        const f32x4 v = *reinterpret_cast<const f32x4*>(th + (4 * rg + k) * HW + 4 * cg);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int a = k - o;
            if (a < 0 || a > 2 * ry) continue;
            const float wa = w.wy[a];
            acc[o][0] = __builtin_fmaf(wa, v.x, acc[o][0]);
            acc[o][1] = __builtin_fmaf(wa, v.y, acc[o][1]);
            acc[o][2] = __builtin_fmaf(wa, v.z, acc[o][2]);
            acc[o][3] = __builtin_fmaf(wa, v.w, acc[o][3]);
        }
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) store4(out, rows, cols, y0 + 4 * rg + o, x0 + 4 * cg, acc[o]);
}

// O2d: separable, with the row pass read straight from global memory through
// the L1 cache (each lane loads its 4 + 2*HX aligned inputs as 16-byte
// vectors; neighbouring lanes' overlaps hit L1), so LDS holds only the
// row-pass result of a 64 x 32 tile.  The small LDS footprint allows full
// occupancy, and the 32-row tile keeps 4x more workgroups in flight than the
// 64 x 64 tile.
#ifndef SKEL_O2D_TY
#define SKEL_O2D_TY 32
#endif
constexpr int kTY2 = SKEL_O2D_TY;

template <int RY, int RX>
__global__ __launch_bounds__(kBlock) void ov2_sep_l1(const float* x, float* out, int64_t rows,
                                                     int64_t cols, W2 w, int ry_, int rx_,
                                                     int edge, float pad, int64_t nbx,
                                                     int64_t nb) {
    // blockIdx.y: one of several equally shaped images stored back to back
    x += (int64_t)blockIdx.y * rows * cols;
    out += (int64_t)blockIdx.y * rows * cols;
    using RD = Rad<RY, RX>;
    constexpr int MY = RD::MY, MX = RD::MX, HX = RD::HX;
    constexpr int HW = kTX + 4;              // row-pass buffer stride (padded)
    constexpr int LH = kTY2 + 2 * MY;        // row-pass rows
    constexpr int NV = (4 + 2 * HX) / 4;     // 16-byte vectors per lane and row
    constexpr int RO = kTY2 / 16;            // output rows per lane
    const int ry = RD::dyn ? ry_ : RY, rx = RD::dyn ? rx_ : RX;
    __shared__ __attribute__((aligned(16))) float th[LH * HW];
    int64_t bx, by;
    tile_coords(nbx, nb, bx, by);
    const int64_t y0 = by * kTY2, x0 = bx * kTX;
    const bool interior = y0 - ry >= 0 && y0 + kTY2 + ry <= rows && x0 - HX >= 0 &&
                          x0 + kTX + HX <= cols && (cols & 3) == 0;
    const int cg = threadIdx.x % 16, rg = threadIdx.x / 16;
    const int nrows = kTY2 + 2 * ry;
    // row pass: every row this lane handles is loaded before any arithmetic
    // (kIt rows of NV 16-byte vectors in flight per lane)
    constexpr int kIt = (LH + 15) / 16;
    float seg[kIt][4 + 2 * HX];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int y = rg + 16 * it;
        if (y >= nrows) continue;
        const int64_t gy = y0 - ry + y;
        if (interior) {
            const float* src = x + gy * cols + (x0 - HX + 4 * cg);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const f32x4 t = *reinterpret_cast<const f32x4*>(src + 4 * v);
                seg[it][4 * v] = t.x;
                seg[it][4 * v + 1] = t.y;
                seg[it][4 * v + 2] = t.z;
                seg[it][4 * v + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int t = 0; t < 4 + 2 * HX; ++t)
                seg[it][t] = fetch2(x, rows, cols, gy, x0 - HX + 4 * cg + t, edge, pad);
        }
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int y = rg + 16 * it;
        if (y >= nrows) continue;
        float h[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b <= 2 * MX; ++b) {
            if (b > 2 * rx) break;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                h[c] = __builtin_fmaf(w.wx[b], seg[it][c + b + HX - rx], h[c]);
        }
        *reinterpret_cast<f32x4*>(th + y * HW + 4 * cg) = f32x4{h[0], h[1], h[2], h[3]};
    }
    __syncthreads();
    float acc[RO][4];
#pragma unroll
    for (int o = 0; o < RO; ++o)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[o][c] = 0.0f;
#pragma unroll
    for (int k = 0; k < RO + 2 * MY; ++k) {
        if (k >= RO + 2 * ry) break;
        const f32x4 v = *reinterpret_cast<const f32x4*>(th + (RO * rg + k) * HW + 4 * cg);
#pragma unroll
        for (int o = 0; o < RO; ++o) {
            const int a = k - o;
            if (a < 0 || a > 2 * ry) continue;
            const float wa = w.wy[a];
            acc[o][0] = __builtin_fmaf(wa, v.x, acc[o][0]);
            acc[o][1] = __builtin_fmaf(wa, v.y, acc[o][1]);
            acc[o][2] = __builtin_fmaf(wa, v.z, acc[o][2]);
            acc[o][3] = __builtin_fmaf(wa, v.w, acc[o][3]);
        }
    }
#pragma unroll
    for (int o = 0; o < RO; ++o) store4(out, rows, cols, y0 + RO * rg + o, x0 + 4 * cg, acc[o]);
}

// O2e.  A workgroup's four wavefronts take four vertically stacked strips,
// so the ry halo rows that one strip shares with the next are read from
// cache.  Input row m of a strip (row i0 - ry + m of the image) feeds output
// rows m - a of the strip with weight row a; output row o accumulates in ring
// slot o mod (2ry+1), which is stored and cleared once row o + 2ry is in.
// What bounds it is how many rows a wavefront has in flight: all rows of a
// chunk are loaded before the first is used.  Measured (5-point stencil on
// 64 fields of 2048^2; strip rows / chunk rows): 32/9 394 us, 16/9 378,
// 64/9 397, 32/18 433, 16/18 (the whole strip) 358, O2b 428.  A dense 9 x 9
// needs 24 rows for a 16-row strip, more than the registers hold: 64-row
// strips in chunks of 18 rows are used there (on 4096^2, back to back with
// the image in the Infinity Cache: 67 us, 16-row strips 90; evicted, all of
// them lose to O2b, which the plan therefore keeps for radii above 2).
constexpr int kMarchCols = 4 * dev::kWave;    // columns per strip
constexpr int kMarchMaxR = 4;                 // radius reach of one neighbour lane
// With a run-time column radius (radii other than 1, 2 or 4 in both
// directions) the tap loop is longer, and whole-strip chunks spill; those
// instances load about eight rows at a time (one ring of 7 for radius 3,
// where two rings spill).
template <int RY, bool DYN>
struct March {
    static constexpr int NW = 2 * RY + 1;                       // ring slots
    static constexpr int rows = RY <= 2 ? 16 : 64;              // output rows per strip
    static constexpr int chunk = DYN ? (RY == 3 ? NW : NW * ((8 + NW - 1) / NW))
                               : RY <= 2 ? rows + 2 * RY : 2 * NW;  // rows loaded at once
    static_assert(chunk % NW == 0 && (rows + 2 * RY) % chunk == 0, "whole chunks per strip");
};

// four consecutive columns starting at j of row rp, through the column rule
__device__ __forceinline__ f32x4 fetch_row4(const float* rp, int64_t cols, int64_t j,
                                            bool aligned, int edge, float pad) {
    if (aligned && j >= 0 && j + 4 <= cols) return *reinterpret_cast<const f32x4*>(rp + j);
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int64_t c;
        v[q] = border(j + q, cols, edge, c) ? rp[c] : pad;
    }
    return f32x4{v[0], v[1], v[2], v[3]};
}

// Add loaded row m of a strip (held in ring position t = m mod (2ry+1)) into
// the output rows it feeds, then store output row m - 2ry, now complete, and
// clear its slot for row m + 1.  c: this lane's four columns; e: the chunk
// beyond the strip's end read by lanes 0 (left) and 63 (right).  SEP: the
// weights are factors, so the row is filtered once with wx and the result
// added with wy[a] (the LDS separable variants' order of operations).
template <int RY, int MX, bool SEP>
__device__ __forceinline__ void march_row(float (&acc)[2 * RY + 1][4], int t, int m, f32x4 c,
                                          f32x4 e, const W2& w, int rx, float* out,
                                          int64_t i0, int64_t j, int64_t cols, bool vec_store) {
    constexpr int NW = 2 * RY + 1;
    const int nx = 2 * rx + 1;
    const f32x4 lt = dev::wave_shift_up(c, e), rt = dev::wave_shift_down(c, e);
    const float v[12] = {lt.x, lt.y, lt.z, lt.w, c.x, c.y, c.z, c.w, rt.x, rt.y, rt.z, rt.w};
    if constexpr (SEP) {
        float h[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int d = -MX; d <= MX; ++d) {
            if (d < -rx || d > rx) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) h[q] = __builtin_fmaf(w.wx[d + rx], v[4 + q + d], h[q]);
        }
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            const int s = ((t - a) % NW + NW) % NW;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[s][q] = __builtin_fmaf(w.wy[a], h[q], acc[s][q]);
        }
    } else {
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            const int s = ((t - a) % NW + NW) % NW;
#pragma unroll
            for (int d = -MX; d <= MX; ++d) {
                if (d < -rx || d > rx) continue;
                const float wab = w.w[a * nx + d + rx];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[s][q] = __builtin_fmaf(wab, v[4 + q + d], acc[s][q]);
            }
        }
    }
    const int sd = (t + 1) % NW;
    if (m >= 2 * RY) {
        float* op = out + (i0 + m - 2 * RY) * cols;
        if (vec_store) {
            dev::store_vec_nt(f32x4{acc[sd][0], acc[sd][1], acc[sd][2], acc[sd][3]},
                              reinterpret_cast<f32x4*>(op + j));
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (j + q < cols) op[j + q] = acc[sd][q];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[sd][q] = 0.0f;
}

template <int RY, int RX, bool SEP>
__global__ __launch_bounds__(kBlock) void ov2_march(const float* x, float* out, int64_t rows,
                                                    int64_t cols, W2 w, int rx_, int edge,
                                                    float pad, int64_t nbx, int64_t nb) {
    // blockIdx.y: one of several equally shaped images stored back to back
    x += (int64_t)blockIdx.y * rows * cols;
    out += (int64_t)blockIdx.y * rows * cols;
    using M = March<RY, (RX < 0)>;
    constexpr int NW = M::NW, CH = M::chunk, kMarchRows = M::rows;
    constexpr int MX = RX >= 0 ? RX : kMarchMaxR;
    const int rx = RX >= 0 ? RX : rx_;
    const int l = dev::lane();
    const int64_t bx = (int64_t)blockIdx.x % nbx, by = (int64_t)blockIdx.x / nbx;
    const int64_t j0 = bx * kMarchCols;
    const int64_t i0 = (by * (kBlock / dev::kWave) + threadIdx.x / dev::kWave) * kMarchRows;
    if (i0 >= rows) return;  // whole wavefronts; no barrier follows
    const int64_t j = j0 + 4 * l;
    const bool aligned = (cols & 3) == 0;
    const int nout = (int)(rows - i0 < kMarchRows ? rows - i0 : kMarchRows);
    const int nin = nout + 2 * RY;
    // the chunk the edge lanes read beyond the strip: left of it for lane 0,
    // right of it for lane 63 (other lanes re-read their own chunk)
    const int64_t je = l == 0 ? j0 - 4 : l == dev::kWave - 1 ? j0 + kMarchCols : j;
    float acc[NW][4];
#pragma unroll
    for (int s = 0; s < NW; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[s][q] = 0.0f;
    int m0 = 0;
    // fast path: the strip lies inside the row, so every row is two
    // unconditional 16-byte loads per lane.  Rows beyond the image ends (at
    // most ry <= rows away) and the edge chunks beyond the row ends map by the
    // edge rule without branches: cyclic reads the chunk at the other end,
    // clamp repeats the row's end value, const takes the pad.
    if (aligned && j0 + kMarchCols <= cols && rows >= kMarchMaxR) {
        const bool lo = l == 0 && j0 == 0, hi = l == dev::kWave - 1 && j0 + kMarchCols == cols;
        const bool efix = (lo || hi) && edge != SKEL_EDGE_CYCLIC;
        const int64_t jf = lo ? cols - 4 : hi ? 0 : je;
        const int64_t jr = efix ? j : jf;
        for (; m0 + CH <= nin; m0 += CH) {
            f32x4 c[CH], e[CH];
            bool in[CH];
#pragma unroll
            for (int t = 0; t < CH; ++t) {
                const int64_t k = i0 - RY + m0 + t;
                in[t] = k >= 0 && k < rows;
                const int64_t kk = in[t] ? k
                                 : edge == SKEL_EDGE_CYCLIC ? (k < 0 ? k + rows : k - rows)
                                 : (k < 0 ? 0 : rows - 1);
                c[t] = *reinterpret_cast<const f32x4*>(x + kk * cols + j);
                e[t] = *reinterpret_cast<const f32x4*>(x + kk * cols + jr);
            }
#pragma unroll
            for (int t = 0; t < CH; ++t) {
                if (edge == SKEL_EDGE_CONST && !in[t]) {
                    c[t] = f32x4{pad, pad, pad, pad};
                    e[t] = c[t];
                }
                if (efix) {
                    const float b = edge == SKEL_EDGE_CONST ? pad : lo ? c[t].x : c[t].w;
                    e[t] = f32x4{b, b, b, b};
                }
                march_row<RY, MX, SEP>(acc, t % NW, m0 + t, c[t], e[t], w, rx, out, i0, j, cols,
                                  true);
            }
        }
    } else if (rows >= kMarchMaxR) {
        // a strip past a ragged row end, or rows not 16-byte aligned: the
        // column rule is the same for every row, so each lane maps its four
        // columns and the edge chunk once; rows are then straight-line element
        // loads from valid addresses, with the pad selected afterwards
        int64_t ci[4], ei[4];
        bool cp[4], ep[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int64_t cc;
            cp[q] = !border(j + q, cols, edge, cc);
            ci[q] = cp[q] ? 0 : cc;
            ep[q] = !border(je + q, cols, edge, cc);
            ei[q] = ep[q] ? 0 : cc;
        }
        const bool vec_store = aligned && j + 4 <= cols;
        for (; m0 + CH <= nin; m0 += CH) {
            float cv[CH][4], ev[CH][4];
            bool in[CH];
#pragma unroll
            for (int t = 0; t < CH; ++t) {
                const int64_t k = i0 - RY + m0 + t;
                in[t] = k >= 0 && k < rows;
                const int64_t kk = in[t] ? k
                                 : edge == SKEL_EDGE_CYCLIC ? (k < 0 ? k + rows : k - rows)
                                 : (k < 0 ? 0 : rows - 1);
                const float* rp = x + kk * cols;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    cv[t][q] = rp[ci[q]];
                    ev[t][q] = rp[ei[q]];
                }
            }
#pragma unroll
            for (int t = 0; t < CH; ++t) {
                const bool padrow = edge == SKEL_EDGE_CONST && !in[t];
                float c[4], e[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    c[q] = padrow || cp[q] ? pad : cv[t][q];
                    e[q] = padrow || ep[q] ? pad : ev[t][q];
                }
                march_row<RY, MX, SEP>(acc, t % NW, m0 + t, f32x4{c[0], c[1], c[2], c[3]},
                                       f32x4{e[0], e[1], e[2], e[3]}, w, rx, out, i0, j, cols,
                                       vec_store);
            }
        }
    }
    // general path: the last strip of an image whose height is not a whole
    // number of strips, and images of fewer than four rows
    for (; m0 < nin; m0 += NW) {
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            const int m = m0 + t;
            if (m >= nin) break;
            int64_t kk;
            f32x4 c = {pad, pad, pad, pad}, e = {pad, pad, pad, pad};
            if (border(i0 - RY + m, rows, edge, kk)) {
                const float* rp = x + kk * cols;
                c = fetch_row4(rp, cols, j, aligned, edge, pad);
                if (l == 0 || l == dev::kWave - 1) e = fetch_row4(rp, cols, je, aligned, edge, pad);
            }
            march_row<RY, MX, SEP>(acc, t, m, c, e, w, rx, out, i0, j, cols, aligned && j + 4 <= cols);
        }
    }
}

// --------------------------------------------------------------- launchers
int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <int RT>
skel_status run1d(int v, const float* x, float* out, int64_t n, const W1& w, int r, int edge,
                  float pad, hipStream_t st) {
    if (v == O1A_DIRECT) {
        ov1_direct<RT><<<(unsigned)div_up(n, kBlock), kBlock, 0, st>>>(x, out, n, w, r, edge, pad);
        return launch_check("overlap1d_direct");
    }
    if (v == O1C_SHUFFLE) {  // selectable for r <= 4 only
        ov1_shfl<RT><<<(unsigned)div_up(n, 4 * kBlock * kShflRows), kBlock, 0, st>>>(
            x, out, n, w, r, edge, pad);
        return launch_check("overlap1d_shuffle");
    }
    ov1_lds<RT><<<(unsigned)div_up(n, kT1), kBlock, 0, st>>>(x, out, n, w, r, edge, pad);
    return launch_check("overlap1d_lds");
}

template <int RY, int RX, bool SEP>
skel_status run2d_march(const float* x, float* out, int64_t rows, int64_t cols, unsigned fields,
                        const W2& w, int ry, int rx, int edge, float pad, hipStream_t st) {
    const int64_t nbx = div_up(cols, kMarchCols);
    constexpr int64_t kWaves = kBlock / dev::kWave;
    if constexpr (RY >= 0) {
        const int64_t nb = nbx * div_up(rows, March<RY, (RX < 0)>::rows * kWaves);
        ov2_march<RY, RX, SEP><<<dim3((unsigned)nb, fields), kBlock, 0, st>>>(
            x, out, rows, cols, w, rx, edge, pad, nbx, nb);
    } else {
        switch (ry) {
#define SKEL_O2E_CASE(R)                                                                       \
    case R: {                                                                                  \
        const int64_t nb = nbx * div_up(rows, March<R, true>::rows * kWaves);                  \
        ov2_march<R, -1, SEP><<<dim3((unsigned)nb, fields), kBlock, 0, st>>>(                  \
            x, out, rows, cols, w, rx, edge, pad, nbx, nb);                                    \
        break;                                                                                 \
    }
            SKEL_O2E_CASE(0)
            SKEL_O2E_CASE(1)
            SKEL_O2E_CASE(2)
            SKEL_O2E_CASE(3)
            SKEL_O2E_CASE(4)
#undef SKEL_O2E_CASE
        default: return SKEL_E_UNSUPPORTED;
        }
    }
    return launch_check("overlap2d_march");
}

template <int RY, int RX>
skel_status run2d(int v, const float* x, float* out, int64_t rows, int64_t cols,
                  unsigned fields, const W2& w, bool sep, int ry, int rx, int edge, float pad,
                  hipStream_t st) {
    if (v == O2A_DIRECT) {
        const int64_t nbx = div_up(cols, 64), nby = div_up(rows, 4);
        ov2_direct<RY, RX><<<dim3((unsigned)(nbx * nby), fields), kBlock, 0, st>>>(
            x, out, rows, cols, w, ry, rx, edge, pad, nbx);
        return launch_check("overlap2d_direct");
    }
    if (v == O2E_MARCH)  // selectable for ry, rx <= 4 only
        return sep ? run2d_march<RY, RX, true>(x, out, rows, cols, fields, w, ry, rx, edge, pad, st)
                   : run2d_march<RY, RX, false>(x, out, rows, cols, fields, w, ry, rx, edge, pad,
                                                st);
    if (v == O2D_SEPARABLE_L1) {
        const int64_t nbx = div_up(cols, kTX), nb = nbx * div_up(rows, kTY2);
        ov2_sep_l1<RY, RX><<<dim3((unsigned)nb, fields), kBlock, 0, st>>>(
            x, out, rows, cols, w, ry, rx, edge, pad, nbx, nb);
        return launch_check("overlap2d_separable_l1");
    }
    const int64_t nbx = div_up(cols, kTX), nby = div_up(rows, kTY), nb = nbx * nby;
    if (v == O2B_LDS_TILE) {
        ov2_lds<RY, RX><<<dim3((unsigned)nb, fields), kBlock, 0, st>>>(
            x, out, rows, cols, w, ry, rx, edge, pad, nbx, nb);
        return launch_check("overlap2d_lds");
    }
    ov2_sep<RY, RX><<<dim3((unsigned)nb, fields), kBlock, 0, st>>>(x, out, rows, cols, w, ry,
                                                                   rx, edge, pad, nbx, nb);
    return launch_check("overlap2d_separable");
}

template <int RY, int RX>
skel_status run2d_fields(int v, const float* x, float* out, int64_t rows, int64_t cols,
                         int64_t fields, const W2& w, bool sep, int ry, int rx, int edge,
                         float pad, hipStream_t st) {
    const int64_t img = rows * cols;
    for (int64_t f0 = 0; f0 < fields; f0 += kMaxFieldsPerLaunch) {
        const unsigned nf = (unsigned)std::min<int64_t>(fields - f0, kMaxFieldsPerLaunch);
        const skel_status e = run2d<RY, RX>(v, x + f0 * img, out + f0 * img, rows, cols, nf, w,
                                            sep, ry, rx, edge, pad, st);
        if (e != SKEL_OK) return e;
    }
    return SKEL_OK;
}

}  // namespace

skel_status launch_overlap1d(int v, const float* x, float* out, int64_t n, const float* w,
                             int r, int edge, float pad, LaunchCtx& lc) {
    W1 wk{};
    for (int k = 0; k <= 2 * r; ++k) wk.w[k] = w[k];
    switch (r) {
    case 1: return run1d<1>(v, x, out, n, wk, r, edge, pad, lc.stream);
    case 2: return run1d<2>(v, x, out, n, wk, r, edge, pad, lc.stream);
    case 4: return run1d<4>(v, x, out, n, wk, r, edge, pad, lc.stream);
    default: return run1d<-1>(v, x, out, n, wk, r, edge, pad, lc.stream);
    }
}

skel_status launch_overlap2d(int v, const float* x, float* out, int64_t rows, int64_t cols,
                             int64_t fields, const float* w2d, const float* wy, const float* wx,
                             int ry, int rx, int edge, float pad, LaunchCtx& lc) {
    W2 wk{};
    const int ny = 2 * ry + 1, nx = 2 * rx + 1;
    for (int a = 0; a < ny; ++a)
        for (int b = 0; b < nx; ++b)
            wk.w[a * nx + b] = w2d ? w2d[a * nx + b] : wy[a] * wx[b];
    if (!w2d) {
        for (int a = 0; a < ny; ++a) wk.wy[a] = wy[a];
        for (int b = 0; b < nx; ++b) wk.wx[b] = wx[b];
    }
    if (ry == 4 && rx == 4)
        return run2d_fields<4, 4>(v, x, out, rows, cols, fields, wk, !w2d, ry, rx, edge, pad, lc.stream);
    if (ry == 1 && rx == 1)
        return run2d_fields<1, 1>(v, x, out, rows, cols, fields, wk, !w2d, ry, rx, edge, pad, lc.stream);
    if (ry == 2 && rx == 2)
        return run2d_fields<2, 2>(v, x, out, rows, cols, fields, wk, !w2d, ry, rx, edge, pad, lc.stream);
    return run2d_fields<-1, -1>(v, x, out, rows, cols, fields, wk, !w2d, ry, rx, edge, pad, lc.stream);
}

}  // namespace skel
