// Map skeleton kernels: out[i] = f(x[i], y[i]) (Section III, map).
//
// Three variants of one computation (Section III: multiple implementations
// per skeleton):
//   M0  scalar grid-stride loop, one element per lane per step (the plain
//       form every GPU port starts from);
//   M1  16-byte vector loads/stores (4 floats per lane per step), grid-stride;
//   M2  each lane moves four 16-byte vectors of one 4096-element chunk per
//       workgroup (all loads issued before any arithmetic), with
//       non-temporal loads and stores (measured in the bench step, saxpy on
//       2^26 floats: 128 us, against 145-161 us with plain loads or stores).
// All three are HBM-bound streams: 8 or 12 bytes per element, 1-2 flops.
#include "kcommon.hpp"
#include "kelem.hpp"
#include "launch.hpp"

namespace skel {
namespace {

using dev::f32x4;

using dev::fmap;
using dev::two_inputs;

template <int OP>
__device__ __forceinline__ f32x4 fmap4(f32x4 a, f32x4 b, float p0, float p1) {
    f32x4 r;
    r.x = fmap<OP>(a.x, b.x, p0, p1);
    r.y = fmap<OP>(a.y, b.y, p0, p1);
    r.z = fmap<OP>(a.z, b.z, p0, p1);
    r.w = fmap<OP>(a.w, b.w, p0, p1);
    return r;
}

constexpr int kBlock = 256;

template <int OP>
__global__ __launch_bounds__(kBlock) void map_m0(const float* x, const float* y, float* out,
                                                 int64_t n, float p0, float p1) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        out[i] = fmap<OP>(x[i], two_inputs<OP>() ? y[i] : 0.0f, p0, p1);
}

template <int OP>
__global__ __launch_bounds__(kBlock) void map_m1(const float* x, const float* y, float* out,
                                                 int64_t n, float p0, float p1) {
    const int64_t nv = n >> 2;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const f32x4* xv = reinterpret_cast<const f32x4*>(x);
    const f32x4* yv = reinterpret_cast<const f32x4*>(y);
    f32x4* ov = reinterpret_cast<f32x4*>(out);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nv; i += stride) {
        f32x4 a = xv[i];
        f32x4 b = two_inputs<OP>() ? yv[i] : f32x4{0.f, 0.f, 0.f, 0.f};
        ov[i] = fmap4<OP>(a, b, p0, p1);
    }
    // the last n % 4 elements
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        int64_t k = (nv << 2) + threadIdx.x;
        out[k] = fmap<OP>(x[k], two_inputs<OP>() ? y[k] : 0.0f, p0, p1);
    }
}

constexpr int kM2Unroll = 4;
constexpr int kM2Chunk = kBlock * 4 * kM2Unroll;  // elements per workgroup

template <int OP>
__global__ __launch_bounds__(kBlock) void map_m2(const float* x, const float* y, float* out,
                                                 int64_t n, float p0, float p1) {
    const int64_t base = (int64_t)blockIdx.x * kM2Chunk;
    if (base + kM2Chunk <= n) {
        const f32x4* xv = reinterpret_cast<const f32x4*>(x + base);
        const f32x4* yv = reinterpret_cast<const f32x4*>(y + base);
        f32x4* ov = reinterpret_cast<f32x4*>(out + base);
        f32x4 a[kM2Unroll], b[kM2Unroll];
#pragma unroll
        for (int u = 0; u < kM2Unroll; ++u) {
            a[u] = __builtin_nontemporal_load(&xv[u * kBlock + threadIdx.x]);
            b[u] = two_inputs<OP>() ? __builtin_nontemporal_load(&yv[u * kBlock + threadIdx.x])
                                    : f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < kM2Unroll; ++u)
            dev::store_vec_nt(fmap4<OP>(a[u], b[u], p0, p1), &ov[u * kBlock + threadIdx.x]);
    } else {
        for (int64_t i = base + threadIdx.x; i < n; i += kBlock)
            out[i] = fmap<OP>(x[i], two_inputs<OP>() ? y[i] : 0.0f, p0, p1);
    }
}

template <int OP>
skel_status launch_op(int variant, float p0, float p1, const float* x, const float* y,
                      float* out, int64_t n, LaunchCtx& lc) {
    const int64_t cap = (int64_t)lc.dev->cus * 16;
    switch (variant) {
    case 0: {
        int64_t g = (n + kBlock - 1) / kBlock;
        if (g > cap) g = cap;
        map_m0<OP><<<dim3((unsigned)g), dim3(kBlock), 0, lc.stream>>>(x, y, out, n, p0, p1);
        return launch_check("map_m0");
    }
    case 1: {
        int64_t g = ((n >> 2) + kBlock - 1) / kBlock;
        if (g < 1) g = 1;
        if (g > cap) g = cap;
        map_m1<OP><<<dim3((unsigned)g), dim3(kBlock), 0, lc.stream>>>(x, y, out, n, p0, p1);
        return launch_check("map_m1");
    }
    default: {
        int64_t g = (n + kM2Chunk - 1) / kM2Chunk;
        map_m2<OP><<<dim3((unsigned)g), dim3(kBlock), 0, lc.stream>>>(x, y, out, n, p0, p1);
        return launch_check("map_m2");
    }
    }
}

}  // namespace

skel_status launch_map(int variant, int op, float p0, float p1, const float* x,
                       const float* y, float* out, int64_t n, LaunchCtx& lc) {
    switch (op) {
    case SKEL_MAP_IDENTITY: return launch_op<SKEL_MAP_IDENTITY>(variant, p0, p1, x, y, out, n, lc);
    case SKEL_MAP_AXPY: return launch_op<SKEL_MAP_AXPY>(variant, p0, p1, x, y, out, n, lc);
    case SKEL_MAP_AFFINE: return launch_op<SKEL_MAP_AFFINE>(variant, p0, p1, x, y, out, n, lc);
    case SKEL_MAP_TANH: return launch_op<SKEL_MAP_TANH>(variant, p0, p1, x, y, out, n, lc);
    case SKEL_MAP_AFFINE_TANH:
        return launch_op<SKEL_MAP_AFFINE_TANH>(variant, p0, p1, x, y, out, n, lc);
    case SKEL_MAP_MUL: return launch_op<SKEL_MAP_MUL>(variant, p0, p1, x, y, out, n, lc);
    case SKEL_MAP_SQUARE: return launch_op<SKEL_MAP_SQUARE>(variant, p0, p1, x, y, out, n, lc);
    }
    return fail(SKEL_E_INVAL, "unknown map op %d", op);
}

}  // namespace skel
