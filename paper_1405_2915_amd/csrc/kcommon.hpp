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

// ------------------------------------------- register-only cross-lane moves
// DPP (data-parallel primitive) moves and v_readlane pass values between the
// lanes of a wavefront inside the register file; __shfl* go through the LDS
// crossbar (ds_bpermute), which costs LDS bandwidth and a round trip per
// move.  Controls (gfx9 encoding): row_shl:k 0x100+k and row_shr:k 0x110+k
// move within rows of 16 lanes; wave_shl:1 0x130 and wave_shr:1 0x138 move
// across the whole wavefront.  "shr" moves data to higher lanes (lane i reads
// lane i - k).
enum : int {
    kDppRowShl = 0x100,
    kDppRowShr = 0x110,
    kDppWaveShl1 = 0x130,
    kDppWaveShr1 = 0x138
};

// dpp<CTRL>(fill, v): every lane receives v of the lane CTRL names; a lane
// whose source lies outside its row (row controls) or outside the wavefront
// (wave controls) receives its own `fill`.
template <int CTRL, class T>
__device__ __forceinline__ T dpp(T fill, T v) {
    static_assert(sizeof(T) % 4 == 0, "DPP moves 32-bit words");
    constexpr int W = sizeof(T) / 4;
    int f[W], x[W], r[W];
    __builtin_memcpy(f, &fill, sizeof(T));
    __builtin_memcpy(x, &v, sizeof(T));
#pragma unroll
    for (int k = 0; k < W; ++k)
        r[k] = __builtin_amdgcn_update_dpp(f[k], x[k], CTRL, 0xf, 0xf, false);
    T out;
    __builtin_memcpy(&out, r, sizeof(T));
    return out;
}

// v of lane `src` (a constant), in every lane
template <class T>
__device__ __forceinline__ T lane_value(T v, int src) {
    static_assert(sizeof(T) % 4 == 0, "v_readlane moves 32-bit words");
    constexpr int W = sizeof(T) / 4;
    int x[W], r[W];
    __builtin_memcpy(x, &v, sizeof(T));
#pragma unroll
    for (int k = 0; k < W; ++k) r[k] = __builtin_amdgcn_readlane(x[k], src);
    T out;
    __builtin_memcpy(&out, r, sizeof(T));
    return out;
}

// lane l receives v of lane l - 1; lane 0 receives its own fill
template <class T>
__device__ __forceinline__ T wave_shift_up(T v, T fill) {
    return dpp<kDppWaveShr1>(fill, v);
}

// lane l receives v of lane l + 1; lane 63 receives its own fill
template <class T>
__device__ __forceinline__ T wave_shift_down(T v, T fill) {
    return dpp<kDppWaveShl1>(fill, v);
}

// Inclusive scan over the 64 lanes: Hillis-Steele steps of 1, 2, 4 and 8
// lanes inside each row of 16 (DPP row shifts, the identity entering at the
// row start), then each row adds the totals of the rows before it, read from
// lanes 15, 31 and 47.  Needs every lane of the wavefront active.
template <class C, class T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const T id = C::id();
    v = C::op(dpp<kDppRowShr + 1>(id, v), v);
    v = C::op(dpp<kDppRowShr + 2>(id, v), v);
    v = C::op(dpp<kDppRowShr + 4>(id, v), v);
    v = C::op(dpp<kDppRowShr + 8>(id, v), v);
    const T t0 = lane_value(v, 15), t1 = lane_value(v, 31), t2 = lane_value(v, 47);
    const T b2 = C::op(t0, t1), b3 = C::op(b2, t2);
    const int row = lane() >> 4;
    const T before = row == 0 ? id : row == 1 ? t0 : row == 2 ? b2 : b3;
    return C::op(before, v);
}

// Inclusive suffix scan over the 64 lanes: lane l ends with v[l] op ... op
// v[63] (DPP row shifts downwards, then the totals of the rows after, read
// from lanes 16, 32 and 48).  Needs every lane of the wavefront active.
template <class C, class T>
__device__ __forceinline__ T wave_inclusive_suffix_scan(T v) {
    const T id = C::id();
    v = C::op(v, dpp<kDppRowShl + 1>(id, v));
    v = C::op(v, dpp<kDppRowShl + 2>(id, v));
    v = C::op(v, dpp<kDppRowShl + 4>(id, v));
    v = C::op(v, dpp<kDppRowShl + 8>(id, v));
    const T t1 = lane_value(v, 16), t2 = lane_value(v, 32), t3 = lane_value(v, 48);
    const T a1 = C::op(t2, t3), a0 = C::op(t1, a1);
    const int row = lane() >> 4;
    const T after = row == 3 ? id : row == 2 ? t3 : row == 1 ? a1 : a0;
    return C::op(v, after);
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
//
// Both words of a 64-bit payload are loaded before either is examined, so a
// read costs one round trip to the device-coherent level, not two (a load
// issued only after the first word's tag checked out waits for that word).
// Which order the two words are observed in does not matter: a pair is taken
// only when both carry the same state and epoch, and a writer publishes each
// state's pair with one tag.
template <class A>
__device__ __forceinline__ int tagged_get(u64* w2, uint32_t epoch, A& v) {
    if constexpr (sizeof(A) == 4) {
        const u64 lo = tag_load(w2);
        if (((lo >> 32) & 0x3fffffffull) != epoch) return 0;
        const uint32_t b = (uint32_t)lo;
        __builtin_memcpy(&v, &b, 4);
        return (int)(lo >> 62);
    } else {
        const u64 lo = tag_load(w2);
        const u64 hi = tag_load(w2 + 1);
        if (((lo >> 32) & 0x3fffffffull) != epoch || (hi >> 32) != (lo >> 32)) return 0;
        const u64 b = (lo & 0xffffffffull) | (hi << 32);
        __builtin_memcpy(&v, &b, 8);
        return (int)(lo >> 62);
    }
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
