// Device-side building blocks shared by the skeleton kernels: combining
// operators, element-type policies, 64-lane wavefront reductions and scans,
// and 16-byte vector access.  gfx950 only: wavefronts are 64 lanes wide.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "skel.h"

namespace skel {
namespace dev {

constexpr int kWave = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// ------------------------------------------------------------ operators --

template <class T, int OP>
struct Comb;

template <class T>
struct Comb<T, SKEL_SUM> {
    static __device__ __forceinline__ T id() { return T(0); }
    static __device__ __forceinline__ T op(T a, T b) { return a + b; }
};

template <class T>
struct Lim;
template <>
struct Lim<float> {
    static __device__ __forceinline__ float hi() { return __builtin_inff(); }
    static __device__ __forceinline__ float lo() { return -__builtin_inff(); }
};
template <>
struct Lim<int32_t> {
    static __device__ __forceinline__ int32_t hi() { return INT32_MAX; }
    static __device__ __forceinline__ int32_t lo() { return INT32_MIN; }
};
template <>
struct Lim<int64_t> {
    static __device__ __forceinline__ int64_t hi() { return INT64_MAX; }
    static __device__ __forceinline__ int64_t lo() { return INT64_MIN; }
};

template <class T>
struct Comb<T, SKEL_MIN> {
    static __device__ __forceinline__ T id() { return Lim<T>::hi(); }
    static __device__ __forceinline__ T op(T a, T b) { return b < a ? b : a; }
};
template <class T>
struct Comb<T, SKEL_MAX> {
    static __device__ __forceinline__ T id() { return Lim<T>::lo(); }
    static __device__ __forceinline__ T op(T a, T b) { return b > a ? b : a; }
};

// --------------------------------------------------------- element types --
// Storage types by dtype; bf16 is stored as its 16-bit pattern.
template <int DT>
struct Stored;
template <> struct Stored<SKEL_F32> { using type = float; };
template <> struct Stored<SKEL_BF16> { using type = uint16_t; };
template <> struct Stored<SKEL_I32> { using type = int32_t; };
template <> struct Stored<SKEL_I64> { using type = int64_t; };

// Accumulator of a (input, output, op) triple.  Integer sums use unsigned
// arithmetic of the output width, which is the two's-complement wrap the
// contract asks for without signed-overflow undefined behaviour.
template <int DIN, int DOUT, int OP>
struct Acc {
    using type = typename Stored<DOUT>::type;
};
template <int DIN>
struct Acc<DIN, SKEL_F32, SKEL_SUM> { using type = float; };
template <>
struct Acc<SKEL_I32, SKEL_I32, SKEL_SUM> { using type = uint32_t; };
template <int DIN>
struct Acc<DIN, SKEL_I64, SKEL_SUM> { using type = uint64_t; };

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

// Widen a stored input element to the accumulator type.
template <class A, class S>
__device__ __forceinline__ A widen(S v) {
    return (A)v;  // int32 -> uint64 / int64 sign-extends; float -> float
}
template <>
__device__ __forceinline__ float widen<float, uint16_t>(uint16_t v) {
    return bf16_to_f32(v);
}
template <>
__device__ __forceinline__ uint64_t widen<uint64_t, int32_t>(int32_t v) {
    return (uint64_t)(int64_t)v;
}

// ------------------------------------------------------- wave primitives --
// lane exchange; accumulator types made of several words provide their own
// overload, found by argument-dependent lookup
template <class T>
__device__ __forceinline__ T xshfl(T v, int o) {
    return __shfl_xor(v, o);
}

// 64-lane butterfly reduction: every lane ends with the full result, combined
// in a fixed order (deterministic for a fixed launch shape).
template <class C, class T>
__device__ __forceinline__ T wave_reduce(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = C::op(v, xshfl(v, o));
    return v;
}

// Inclusive scan over the 64 lanes (Hillis-Steele with lane shifts).
template <class C, class T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int l = lane();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_up(v, d);
        if (l >= d) v = C::op(u, v);
    }
    return v;
}

// Inclusive suffix scan over the 64 lanes: lane l ends with v[l] op ... op
// v[63] (lane shifts downwards).
template <class C, class T>
__device__ __forceinline__ T wave_inclusive_suffix_scan(T v) {
    const int l = lane();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_down(v, d);
        if (l + d < kWave) v = C::op(v, u);
    }
    return v;
}

// Block reduction for blocks of up to 1024 threads.  `lds` holds one T per
// wavefront.  The result is valid in every lane of wavefront 0.
template <class C, class T>
__device__ __forceinline__ T block_reduce(T v, T* lds) {
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    v = wave_reduce<C>(v);
    if (lane() == 0) lds[w] = v;
    __syncthreads();
    if (w == 0) {
        v = lane() < nw ? lds[lane()] : C::id();
        v = wave_reduce<C>(v);
    }
    return v;
}

// ------------------------------------------------ self-validating words --
// Inter-workgroup hand-off words [state:2 | epoch:30 | payload:32], written
// and read with device-scope relaxed atomics.  A word is valid only if its
// epoch matches the reader's, so the array never needs clearing (the host
// gives each call a fresh epoch), and because state and payload travel in one
// single-copy-atomic word, no release/acquire fence (an L2 write-back on this
// multi-XCD part) is needed.  64-bit payloads use two words whose tags must
// agree.
typedef unsigned long long u64;

__device__ __forceinline__ void tag_store(u64* w, int state, uint32_t epoch, uint32_t payload) {
    const u64 v = ((u64)state << 62) | ((u64)epoch << 32) | payload;
    __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ u64 tag_load(u64* w) {
    return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class A>
__device__ __forceinline__ void tagged_put(u64* w2, int state, uint32_t epoch, A v) {
    if constexpr (sizeof(A) == 4) {
        uint32_t b;
        __builtin_memcpy(&b, &v, 4);
        tag_store(w2, state, epoch, b);
    } else {
        u64 b;
        __builtin_memcpy(&b, &v, 8);
        tag_store(w2, state, epoch, (uint32_t)b);
        tag_store(w2 + 1, state, epoch, (uint32_t)(b >> 32));
    }
}

// Returns the state (0 when the word is stale, i.e. of another epoch, or when
// the two halves of a 64-bit payload carry different tags) and the payload.
template <class A>
__device__ __forceinline__ int tagged_get(u64* w2, uint32_t epoch, A& v) {
    const u64 lo = tag_load(w2);
    if (((lo >> 32) & 0x3fffffffull) != epoch) return 0;
    if constexpr (sizeof(A) == 4) {
        const uint32_t b = (uint32_t)lo;
        __builtin_memcpy(&v, &b, 4);
    } else {
        const u64 hi = tag_load(w2 + 1);
        if ((hi >> 32) != (lo >> 32)) return 0;
        const u64 b = (lo & 0xffffffffull) | (hi << 32);
        __builtin_memcpy(&v, &b, 8);
    }
    return (int)(lo >> 62);
}

// ---------------------------------------------------------- vector access --
template <class T>
__device__ __forceinline__ void load16(const T* p, T (&v)[16 / sizeof(T)]) {
    u32x4 raw = *reinterpret_cast<const u32x4*>(p);
    __builtin_memcpy(&v, &raw, 16);
}

// streaming read of data used once (non-temporal: does not displace cache
// lines that other accesses reuse)
template <class T>
__device__ __forceinline__ void load16_nt(const T* p, T (&v)[16 / sizeof(T)]) {
    u32x4 raw = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    __builtin_memcpy(&v, &raw, 16);
}

// Output stores.  Which kind streams an output to HBM faster depends on the
// access pattern and was measured per kernel on MI355X: plain vector stores
// win where a lane keeps many stores outstanding (the scan's widening rows,
// the 1D stencil), non-temporal ones where each lane writes a few vectors of
// a dense chunk (Map M2, the 2D tiles).
template <class V>
__device__ __forceinline__ void store_vec_nt(V v, V* p) {
    __builtin_nontemporal_store(v, p);
}

// E elements as whole 16-byte vectors, plain stores
template <class T, int E>
__device__ __forceinline__ void store_vecs(T* p, const T (&v)[E]) {
    static_assert((sizeof(T) * E) % 16 == 0, "whole 16-byte vectors only");
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) * E / 16); ++k) {
        u32x4 raw;
        __builtin_memcpy(&raw, reinterpret_cast<const char*>(&v) + 16 * k, 16);
        reinterpret_cast<u32x4*>(p)[k] = raw;
    }
}

}  // namespace dev
}  // namespace skel
