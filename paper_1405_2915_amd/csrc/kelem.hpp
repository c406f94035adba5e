// Element functions f(x, y; p0, p1) of the built-in Map / MapReduce user
// functions (a skeleton instance is a skeleton plus its user function,
// Section III), and their partial derivatives for the reverse-mode kernels.
// Computed in binary32; tanh is recomputed from x where a derivative needs it.
#pragma once

#include <hip/hip_runtime.h>

#include "skel.h"

namespace skel {
namespace dev {

template <int OP>
__device__ __forceinline__ float fmap(float x, float y, float p0, float p1) {
    if constexpr (OP == SKEL_MAP_IDENTITY) return x;
    else if constexpr (OP == SKEL_MAP_AXPY) return __builtin_fmaf(p0, x, y);
    else if constexpr (OP == SKEL_MAP_AFFINE) return __builtin_fmaf(p0, x, p1);
    else if constexpr (OP == SKEL_MAP_TANH) return tanhf(x);
    else if constexpr (OP == SKEL_MAP_AFFINE_TANH) return tanhf(__builtin_fmaf(p0, x, p1));
    else if constexpr (OP == SKEL_MAP_MUL) return x * y;
    else return x * x;
}

template <int OP>
constexpr bool two_inputs() { return OP == SKEL_MAP_AXPY || OP == SKEL_MAP_MUL; }

template <int OP>
constexpr int map_nparams() {
    return OP == SKEL_MAP_AXPY ? 1 : (OP == SKEL_MAP_AFFINE || OP == SKEL_MAP_AFFINE_TANH) ? 2 : 0;
}

// g times the partial derivatives of f at (x, y): dx, dy and the parameter
// terms s0 = g df/dp0, s1 = g df/dp1
template <int OP>
__device__ __forceinline__ void elem_grad(float x, float y, float g, float p0, float p1,
                                          float& dx, float& dy, float& s0, float& s1) {
    dy = 0.0f;
    s0 = 0.0f;
    s1 = 0.0f;
    if constexpr (OP == SKEL_MAP_IDENTITY) {
        dx = g;
    } else if constexpr (OP == SKEL_MAP_AXPY) {
        dx = p0 * g;
        dy = g;
        s0 = g * x;
    } else if constexpr (OP == SKEL_MAP_AFFINE) {
        dx = p0 * g;
        s0 = g * x;
        s1 = g;
    } else if constexpr (OP == SKEL_MAP_TANH) {
        const float t = tanhf(x);
        dx = g * (1.0f - t * t);
    } else if constexpr (OP == SKEL_MAP_AFFINE_TANH) {
        const float t = tanhf(__builtin_fmaf(p0, x, p1));
        const float gd = g * (1.0f - t * t);  // g * tanh' at the pre-activation
        dx = gd * p0;
        s0 = gd * x;
        s1 = gd;
    } else if constexpr (OP == SKEL_MAP_MUL) {
        dx = g * y;
        dy = g * x;
    } else {  // SQUARE
        dx = 2.0f * g * x;
    }
}

}  // namespace dev
}  // namespace skel
