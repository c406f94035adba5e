// Reduce and MapReduce skeleton kernels.
//
// Reduce (Section III): r = x[0] op x[1] op ... op x[n-1].  MapReduce: the
// same over f(x[i], y[i]) with no stored intermediate.  Variants:
//   R0 / MR3  one workgroup of 1024 lanes (small n: one launch, no partials)
//   R1 / MR1  two passes: a grid of workgroups writes partials, one
//             workgroup combines them (the plain form; R1 runs at a fixed
//             launch shape)
//   R2 / MR2  one pass: each workgroup publishes its partial and takes a
//             ticket; the workgroup that draws the last ticket combines all
//             partials in index order, so the result is deterministic
//   R3        one pass with a hardware atomic finish (order-dependent for
//             floating point)
//   R4 / MR4  the R2 pass with compensated (TwoSum / TwoProduct) binary32
//             accumulation: accuracy of a doubled working precision for the
//             same HBM traffic, for long sums of bf16 or f32 data
//   R5 / MR5  the R2 pass with pairwise (cascade) summation in every lane:
//             each chunk's values are added as a balanced tree, and the chunk
//             sums are folded into a binary counter of partial sums, so a
//             lane's additions form a balanced tree over its whole share
//             (error growing with log n instead of n per lane), for the same
//             HBM traffic
//   R6 / MR6  one pass without tickets: every workgroup but the last
//             publishes its partial; the last workgroup by index gathers all
//             of them in index order (deterministic), skipping R2's two
//             serialised atomics -- the latency that dominates arrays of a few
//             million elements
//   MR0       the composed plain form: Map into a temporary, then R1
// Every lane streams 16-byte vectors with four loads in flight and keeps four
// independent accumulators; partials are combined by 64-lane butterflies and
// one LDS step.  Integer sums wrap in the output width (unsigned arithmetic).
#include <type_traits>

#include "kcommon.hpp"
#include "kelem.hpp"
#include "dispatch.hpp"
#include "kepoch.hpp"
#include "launch.hpp"

namespace skel {
namespace {

using namespace dev;

constexpr int kBlock = 256;
constexpr int kSingleBlock = 1024;
constexpr int kUnroll = 4;

template <int DIN, int DOUT, int OP>
struct RP {
    using in_t = typename Stored<DIN>::type;
    using out_t = typename Stored<DOUT>::type;
    using acc_t = typename Acc<DIN, DOUT, OP>::type;
    using C = Comb<acc_t, OP>;
    static constexpr int E = 16 / sizeof(in_t);
    static constexpr int kOp = OP;
};

// ----------------------------------------------------------- element sources
template <class P>
struct PlainSrc {
    using acc_t = typename P::acc_t;
    using in_t = typename P::in_t;
    static constexpr int E = P::E;
    struct Vec {
        in_t a[E];
    };
    const in_t* x;
    __device__ __forceinline__ void load(int64_t vi, Vec& v) const { load16_nt(x + vi * E, v.a); }
    __device__ __forceinline__ void accum(const Vec& v, acc_t& acc) const {
#pragma unroll
        for (int e = 0; e < E; ++e) acc = P::C::op(acc, widen<acc_t>(v.a[e]));
    }
    __device__ __forceinline__ acc_t at(int64_t i) const { return widen<acc_t>(x[i]); }
};

using dev::fmap;
using dev::two_inputs;

// f(x[i], y[i]) accumulated in binary32; inputs f32 or bf16 bit patterns
template <class P, int MOP>
struct MapSrc {
    using acc_t = float;
    using in_t = typename P::in_t;
    static constexpr int E = P::E;
    struct Vec {
        in_t a[E], b[E];
    };
    const in_t* x;
    const in_t* y;
    float p0, p1;
    __device__ __forceinline__ void load(int64_t vi, Vec& v) const {
        load16_nt(x + vi * E, v.a);
        if constexpr (two_inputs<MOP>()) load16_nt(y + vi * E, v.b);
    }
    __device__ __forceinline__ void accum(const Vec& v, float& acc) const {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            float xv = widen<float>(v.a[e]);
            float yv = two_inputs<MOP>() ? widen<float>(v.b[e]) : 0.0f;
            acc = P::C::op(acc, fmap<MOP>(xv, yv, p0, p1));
        }
    }
    __device__ __forceinline__ float at(int64_t i) const {
        float xv = widen<float>(x[i]);
        float yv = two_inputs<MOP>() ? widen<float>(y[i]) : 0.0f;
        return fmap<MOP>(xv, yv, p0, p1);
    }
};

// ------------------------------------------------------- compensated sums
// R4 / MR4: a running sum carried as s + c in two binary32 numbers.  Every
// addition is split exactly into its rounded sum and its rounding error
// (TwoSum, Knuth), the errors are accumulated in c, and products are split
// exactly with a fused multiply-add (TwoProduct), so the accumulated error
// is that of a sum kept to about twice the working precision; s + c is
// rounded once at the end.
struct Comp {
    float s, c;
    __device__ explicit operator float() const { return s + c; }
};

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

__device__ __forceinline__ Comp comp_add(Comp a, float x) {
    float s, e;
    two_sum(a.s, x, s, e);
    return {s, a.c + e};
}

struct CombComp {
    static __device__ __forceinline__ Comp id() { return {0.0f, 0.0f}; }
    static __device__ __forceinline__ Comp op(Comp a, Comp b) {
        float s, e;
        two_sum(a.s, b.s, s, e);
        return {s, (a.c + b.c) + e};
    }
};

__device__ __forceinline__ Comp xshfl(Comp v, int o) {
    return {__shfl_xor(v.s, o), __shfl_xor(v.c, o)};
}

template <int DIN>
struct RPC {
    using in_t = typename Stored<DIN>::type;
    using out_t = float;
    using acc_t = Comp;
    using C = CombComp;
    static constexpr int E = 16 / sizeof(in_t);
    static constexpr int kOp = SKEL_SUM;
};

template <class P>
struct CompSrc {
    using acc_t = Comp;
    using in_t = typename P::in_t;
    static constexpr int E = P::E;
    struct Vec {
        in_t a[E];
    };
    const in_t* x;
    __device__ __forceinline__ void load(int64_t vi, Vec& v) const { load16_nt(x + vi * E, v.a); }
    __device__ __forceinline__ void accum(const Vec& v, Comp& acc) const {
#pragma unroll
        for (int e = 0; e < E; ++e) acc = comp_add(acc, widen<float>(v.a[e]));
    }
    __device__ __forceinline__ Comp at(int64_t i) const { return {widen<float>(x[i]), 0.0f}; }
};

// f(x, y) added with compensation; products (MUL, SQUARE) add their exact
// rounding error as well
template <int MOP>
__device__ __forceinline__ Comp comp_add_mapped(Comp acc, float xv, float yv, float p0,
                                                float p1) {
#pragma clang fp contract(off)
    if constexpr (MOP == SKEL_MAP_MUL || MOP == SKEL_MAP_SQUARE) {
        const float b = MOP == SKEL_MAP_MUL ? yv : xv;
        const float p = xv * b;
        const float err = __builtin_fmaf(xv, b, -p);  // x*b - p exactly
        acc = comp_add(acc, p);
        acc.c += err;
        return acc;
    } else {
        return comp_add(acc, fmap<MOP>(xv, yv, p0, p1));
    }
}

template <class P, int MOP>
struct CompMapSrc {
    using acc_t = Comp;
    using in_t = typename P::in_t;
    static constexpr int E = P::E;
    struct Vec {
        in_t a[E], b[E];
    };
    const in_t* x;
    const in_t* y;
    float p0, p1;
    __device__ __forceinline__ void load(int64_t vi, Vec& v) const {
        load16_nt(x + vi * E, v.a);
        if constexpr (two_inputs<MOP>()) load16_nt(y + vi * E, v.b);
    }
    __device__ __forceinline__ void accum(const Vec& v, Comp& acc) const {
#pragma unroll
        for (int e = 0; e < E; ++e)
            acc = comp_add_mapped<MOP>(acc, widen<float>(v.a[e]),
                                       two_inputs<MOP>() ? widen<float>(v.b[e]) : 0.0f, p0,
                                       p1);
    }
    __device__ __forceinline__ Comp at(int64_t i) const {
        return comp_add_mapped<MOP>(CombComp::id(), widen<float>(x[i]),
                                    two_inputs<MOP>() ? widen<float>(y[i]) : 0.0f, p0, p1);
    }
};

// ----------------------------------------------------------- pairwise sums
// R5 / MR5 sources: the same loads as PlainSrc / MapSrc, and `vals`, the E
// (mapped) values of one vector for the pairwise tree
template <class P>
struct PairSrc : PlainSrc<P> {
    static constexpr bool kPairwise = true;
    __device__ __forceinline__ void vals(const typename PlainSrc<P>::Vec& v,
                                         float (&o)[P::E]) const {
#pragma unroll
        for (int e = 0; e < P::E; ++e) o[e] = widen<float>(v.a[e]);
    }
};

template <class P, int MOP>
struct PairMapSrc : MapSrc<P, MOP> {
    static constexpr bool kPairwise = true;
    __device__ __forceinline__ void vals(const typename MapSrc<P, MOP>::Vec& v,
                                         float (&o)[P::E]) const {
#pragma unroll
        for (int e = 0; e < P::E; ++e)
            o[e] = fmap<MOP>(widen<float>(v.a[e]), two_inputs<MOP>() ? widen<float>(v.b[e]) : 0.0f,
                             this->p0, this->p1);
    }
};

template <class S, class = void>
struct IsPairwise { static constexpr bool value = false; };
template <class S>
struct IsPairwise<S, decltype((void)S::kPairwise)> { static constexpr bool value = S::kPairwise; };

// balanced tree over K values (K a power of two), in place
template <int K>
__device__ __forceinline__ float tree_sum(float (&v)[K]) {
#pragma unroll
    for (int w = K / 2; w >= 1; w /= 2)
#pragma unroll
        for (int i = 0; i < w; ++i) v[i] = v[i] + v[i + w];
    return v[0];
}

// Insert chunk sum `c` (the k-th of this lane, counting from 0) into the
// binary counter of partial sums: level l holds the sum of 2^l consecutive
// chunks while bit l of k is set.  Adding chunk k carries through the set low
// bits like an increment, so every addition combines two equal-sized sums.
// The top level absorbs whatever would carry beyond it.
constexpr int kPairLevels = 16;
__device__ __forceinline__ void cascade_insert(float (&lvl)[kPairLevels], float c, uint32_t k) {
    bool going = true;
#pragma unroll
    for (int l = 0; l < kPairLevels - 1; ++l) {
        const bool bit = ((k >> l) & 1u) != 0;
        const float merged = lvl[l] + c;
        if (going) {
            if (bit) {
                c = merged;
                lvl[l] = 0.0f;
            } else {
                lvl[l] = c;
                going = false;
            }
        }
    }
    if (going) lvl[kPairLevels - 1] += c;
}

// pairwise form of thread_acc (below): same chunks and tails
template <class P, int NT, class Src>
__device__ __forceinline__ float thread_acc_pairwise(const Src& s, int64_t n, int64_t blk,
                                                     int64_t nblk) {
    constexpr int E = P::E;
    constexpr int64_t CH = (int64_t)NT * kUnroll;
    float lvl[kPairLevels];
#pragma unroll
    for (int l = 0; l < kPairLevels; ++l) lvl[l] = 0.0f;
    const int64_t nv = n / E;
    const int64_t nch = nv / CH;
    uint32_t k = 0;
    for (int64_t c = blk; c < nch; c += nblk, ++k) {
        const int64_t b = c * CH + threadIdx.x;
        typename Src::Vec v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) s.load(b + u * NT, v[u]);
        float t[kUnroll * E];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            float o[E];
            s.vals(v[u], o);
#pragma unroll
            for (int e = 0; e < E; ++e) t[u * E + e] = o[e];
        }
        cascade_insert(lvl, tree_sum<kUnroll * E>(t), k);
    }
    // the levels in increasing order, then the tails (fewer than one chunk)
    float total = 0.0f;
#pragma unroll
    for (int l = 0; l < kPairLevels; ++l) total += lvl[l];
    for (int64_t i = nch * CH + blk * NT + threadIdx.x; i < nv; i += nblk * NT) {
        typename Src::Vec v;
        s.load(i, v);
        float o[E];
        s.vals(v, o);
        total += tree_sum<E>(o);
    }
    const int64_t t = nv * E + blk * NT + threadIdx.x;
    if (t < n) total += s.at(t);
    return total;
}

// One lane's share of workgroup `blk` of `nblk`: the workgroup walks chunks of
// NT * kUnroll consecutive 16-byte vectors (chunk blk, blk + nblk, ...), every
// lane with kUnroll loads in flight; then the vectors after the last whole
// chunk, then the n % E tail elements (one per low lane of workgroup 0).
// Consecutive workgroups read consecutive chunks, so the whole grid sweeps one
// narrow window of memory.
template <class P, int NT, class Src>
__device__ __forceinline__ typename P::acc_t thread_acc(const Src& s, int64_t n, int64_t blk,
                                                        int64_t nblk) {
    using acc_t = typename P::acc_t;
    if constexpr (IsPairwise<Src>::value) return thread_acc_pairwise<P, NT>(s, n, blk, nblk);
    constexpr int E = P::E;
    constexpr int64_t CH = (int64_t)NT * kUnroll;
    acc_t a[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) a[u] = P::C::id();
    const int64_t nv = n / E;
    const int64_t nch = nv / CH;
    for (int64_t c = blk; c < nch; c += nblk) {
        const int64_t b = c * CH + threadIdx.x;
        typename Src::Vec v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) s.load(b + u * NT, v[u]);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) s.accum(v[u], a[u]);
    }
    for (int64_t i = nch * CH + blk * NT + threadIdx.x; i < nv; i += nblk * NT) {
        typename Src::Vec v;
        s.load(i, v);
        s.accum(v, a[0]);
    }
    const int64_t t = nv * E + blk * NT + threadIdx.x;
    if (t < n) a[0] = P::C::op(a[0], s.at(t));
#pragma unroll
    for (int u = 1; u < kUnroll; ++u) a[0] = P::C::op(a[0], a[u]);
    return a[0];
}

constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kSlotReady = 1;  // state of a published partial

// ------------------------------------------------------------------ kernels
template <class P, class Src>
__global__ __launch_bounds__(kSingleBlock) void k_single(Src s, int64_t n,
                                                         typename P::out_t* out) {
    __shared__ typename P::acc_t lds[kSingleBlock / kWave];
    auto a = thread_acc<P, kSingleBlock>(s, n, 0, 1);
    a = block_reduce<typename P::C>(a, lds);
    if (threadIdx.x == 0) *out = (typename P::out_t)a;
}

template <class P, class Src>
__global__ __launch_bounds__(kBlock) void k_partials(Src s, int64_t n,
                                                     typename P::acc_t* partials) {
    __shared__ typename P::acc_t lds[kBlock / kWave];
    auto a = thread_acc<P, kBlock>(s, n, blockIdx.x, gridDim.x);
    a = block_reduce<typename P::C>(a, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = a;
}

template <class P>
__global__ __launch_bounds__(kSingleBlock) void k_finish(const typename P::acc_t* partials,
                                                         int g, typename P::out_t* out) {
    __shared__ typename P::acc_t lds[kSingleBlock / kWave];
    auto a = P::C::id();
    for (int i = threadIdx.x; i < g; i += kSingleBlock) a = P::C::op(a, partials[i]);
    a = block_reduce<typename P::C>(a, lds);
    if (threadIdx.x == 0) *out = (typename P::out_t)a;
}

// Single pass: every workgroup publishes its partial as a self-validating
// tagged word (two words per slot), then draws a ticket; the workgroup with
// the last ticket waits until every slot carries this call's epoch and
// combines them in slot order (deterministic).  No fence is needed because a
// slot is valid exactly when its tag says so.  Tickets are two-level: device-
// scope atomics on one word serialise (about 10 ns each measured on MI355X,
// 10 us for 1024 workgroups), so workgroup b draws from first-level ticket
// b % kSubTickets, and only the last drawer of each draws the top ticket.
template <class P, class Src>
__global__ __launch_bounds__(kBlock) void k_ticket(Src s, int64_t n, u64* slots, u64* sync,
                                                   typename P::out_t* out) {
    using acc_t = typename P::acc_t;
    __shared__ acc_t lds[kBlock / kWave];
    __shared__ int is_last;
    __shared__ uint32_t s_epoch;
    u64* ticket = sync + SYNC_TICKET;
    u64* err = sync + SYNC_ERROR;
    acc_t a = thread_acc<P, kBlock>(s, n, blockIdx.x, gridDim.x);
    a = block_reduce<typename P::C>(a, lds);
    if (threadIdx.x == 0) {
        // the epoch is read before the ticket, and advanced only by the holder
        // of the last ticket after it has read every slot
        const uint32_t epoch = epoch_of_call(sync);
        s_epoch = epoch;
        tagged_put(slots + 2 * blockIdx.x, kSlotReady, epoch, a);
        const unsigned c = blockIdx.x % kSubTickets;
        u64* sub = sync + SYNC_SUB_TICKET + 16 * c;
        const u64 drawers = (gridDim.x - c + kSubTickets - 1) / kSubTickets;
        int last = 0;
        if (atomicAdd(sub, 1ull) == drawers - 1) {
            // every workgroup of this first-level ticket has drawn: reset it
            __hip_atomic_store(sub, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const u64 groups = gridDim.x < (unsigned)kSubTickets ? gridDim.x : kSubTickets;
            last = atomicAdd(ticket, 1ull) == groups - 1;
        }
        is_last = last;
    }
    __syncthreads();
    if (!is_last) return;
    const uint32_t epoch = s_epoch;
    // each lane reads its slots i = base + k * kBlock + lane with all loads in
    // flight at once; a retry re-reads only the slots not yet valid
    acc_t b = P::C::id();
    for (unsigned base = 0; base < gridDim.x; base += 4 * kBlock) {
        acc_t v[4];
        bool ready[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = P::C::id();
            ready[k] = base + k * kBlock + threadIdx.x >= gridDim.x;
        }
        uint32_t spins = 0;
        while (true) {
            bool all = true;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (ready[k]) continue;
                const unsigned i = base + k * kBlock + threadIdx.x;
                ready[k] = tagged_get(slots + 2 * i, epoch, v[k]) == kSlotReady;
                all = all && ready[k];
            }
            if (all) break;
            if (++spins > kSpinLimit) {  // bounded: flag it and finish
                atomicOr(err, 2ull);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) b = P::C::op(b, ready[k] ? v[k] : P::C::id());
    }
    b = block_reduce<typename P::C>(b, lds);
    if (threadIdx.x == 0) {
        *out = (typename P::out_t)b;
        __hip_atomic_store(ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        epoch_advance(sync);
    }
}

// Single pass without tickets (R6 / MR6): every workgroup but the last
// publishes its partial as a tagged word and exits; the last workgroup by
// index -- the last to start, so every other one has started and none of them
// waits on anything -- reads all partials with every lane at once (a retry
// re-reads only the slots not yet valid), combines them in a fixed order
// (deterministic) with its own, and advances the epoch: every other workgroup
// read the epoch before it published.  This saves the two serialised
// device-scope ticket atomics of R2 (a few microseconds on arrays of a few
// million elements, where the whole reduction takes about as long).
template <class P, class Src>
__global__ __launch_bounds__(kBlock) void k_gather(Src s, int64_t n, u64* slots, u64* sync,
                                                   typename P::out_t* out) {
    using acc_t = typename P::acc_t;
    using C = typename P::C;
    __shared__ acc_t lds[kBlock / kWave];
    __shared__ acc_t s_own;
    __shared__ uint32_t s_epoch;
    uint32_t ep = 0;
    if (threadIdx.x == 0) ep = epoch_of_call(sync);  // in flight with the first loads
    acc_t a = thread_acc<P, kBlock>(s, n, blockIdx.x, gridDim.x);
    a = block_reduce<C>(a, lds);
    const unsigned last = gridDim.x - 1;
    if (blockIdx.x != last) {
        if (threadIdx.x == 0) tagged_put(slots + 2 * blockIdx.x, kSlotReady, ep, a);
        return;
    }
    if (threadIdx.x == 0) {
        s_own = a;
        s_epoch = ep;
    }
    __syncthreads();  // also ends block_reduce's reads of lds before its reuse
    const uint32_t epoch = s_epoch;
    acc_t b = C::id();
    for (unsigned base = 0; base < last; base += 4 * kBlock) {
        acc_t v[4];
        bool ready[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = C::id();
            ready[k] = base + k * kBlock + threadIdx.x >= last;
        }
        uint32_t spins = 0;
        while (true) {
            bool all = true;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (ready[k]) continue;
                const unsigned i = base + k * kBlock + threadIdx.x;
                ready[k] = tagged_get(slots + 2 * i, epoch, v[k]) == kSlotReady;
                all = all && ready[k];
            }
            if (all) break;
            if (++spins > kSpinLimit) {  // bounded: flag it and finish
                atomicOr(sync + SYNC_ERROR, 2ull);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) b = C::op(b, ready[k] ? v[k] : C::id());
    }
    b = block_reduce<C>(b, lds);
    if (threadIdx.x == 0) {
        *out = (typename P::out_t)C::op(b, s_own);
        epoch_advance(sync);
    }
}

template <class P>
__global__ void k_set_identity(typename P::out_t* out) {
    *out = (typename P::out_t)P::C::id();
}

template <class P>
__device__ __forceinline__ void atomic_combine(typename P::out_t* out, typename P::acc_t v);

template <class P, class Src>
__global__ __launch_bounds__(kBlock) void k_atomic(Src s, int64_t n, typename P::out_t* out) {
    __shared__ typename P::acc_t lds[kBlock / kWave];
    auto a = thread_acc<P, kBlock>(s, n, blockIdx.x, gridDim.x);
    a = block_reduce<typename P::C>(a, lds);
    if (threadIdx.x == 0) atomic_combine<P>(out, a);
}

template <class P>
__device__ __forceinline__ void atomic_combine(typename P::out_t* out, typename P::acc_t v) {
    using acc_t = typename P::acc_t;
    if constexpr (std::is_same<acc_t, float>::value) {
        unsafeAtomicAdd(out, v);  // SUM only (selectability constraint)
    } else if constexpr (std::is_same<acc_t, uint32_t>::value) {
        atomicAdd(reinterpret_cast<unsigned int*>(out), (unsigned int)v);
    } else if constexpr (std::is_same<acc_t, uint64_t>::value) {
        atomicAdd(reinterpret_cast<unsigned long long*>(out), (unsigned long long)v);
    } else if constexpr (std::is_same<acc_t, int32_t>::value) {
        if (P::kOp == SKEL_MIN) atomicMin(reinterpret_cast<int*>(out), (int)v);
        else atomicMax(reinterpret_cast<int*>(out), (int)v);
    } else {
        if (P::kOp == SKEL_MIN) atomicMin(reinterpret_cast<long long*>(out), (long long)v);
        else atomicMax(reinterpret_cast<long long*>(out), (long long)v);
    }
}

// --------------------------------------------------------------- launchers
int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// grid of the single-pass variants: one chunk of kBlock * kUnroll vectors per
// workgroup at least, at most 4 workgroups per CU (measured best on MI355X)
template <class P>
int grid_for(int64_t n, const DevInfo& d) {
    int64_t g = div_up(n / P::E, (int64_t)kBlock * kUnroll);
    if (g < 1) g = 1;
    int64_t cap = (int64_t)d.cus * 4;
    return (int)(g < cap ? g : cap);
}

// partial buffer bytes for the grid variants: at most 8 groups per CU, 8-byte
// accumulators, rounded to 256 bytes
size_t partial_bytes(const DevInfo& d) { return ((size_t)d.cus * 8 * 8 + 255) & ~size_t(255); }

// single-pass launch without tickets (R6, MR6)
template <class P, class Src>
skel_status launch_gather(const Src& s, int64_t n, typename P::out_t* out, LaunchCtx& lc) {
    int g = grid_for<P>(n, *lc.dev);
    void* slots = nullptr;
    skel_status e = ws_status(lc, (size_t)g * 16, &slots);
    if (e != SKEL_OK) return e;
    k_gather<P, Src><<<(unsigned)g, kBlock, 0, lc.stream>>>(s, n, static_cast<u64*>(slots),
                                                            lc.ws->sync, out);
    return launch_check("reduce_gather");
}

// single-pass ticket launch (R2, MR2 and the compensated forms R4, MR4)
template <class P, class Src>
skel_status launch_ticket(const Src& s, int64_t n, typename P::out_t* out, LaunchCtx& lc) {
    int g = grid_for<P>(n, *lc.dev);
    void* slots = nullptr;
    skel_status e = ws_status(lc, (size_t)g * 16, &slots);
    if (e != SKEL_OK) return e;
    k_ticket<P, Src><<<(unsigned)g, kBlock, 0, lc.stream>>>(s, n, static_cast<u64*>(slots),
                                                            lc.ws->sync, out);
    return launch_check("reduce_ticket");
}

template <class P, class Src>
skel_status run_variant(int v, const Src& s, int64_t n, typename P::out_t* out,
                        LaunchCtx& lc, void* partial_mem) {
    using acc_t = typename P::acc_t;
    hipStream_t st = lc.stream;
    switch (v) {
    case R0_SINGLE_WG:
        k_single<P, Src><<<1, kSingleBlock, 0, st>>>(s, n, out);
        return launch_check("reduce_single");
    case R1_TWO_PASS: {
        // fixed plain launch: 256 lanes, min(ceil(n / 2048), 4 * CUs) groups
        int64_t g = div_up(n, 2048);
        if (g < 1) g = 1;
        if (g > (int64_t)lc.dev->cus * 4) g = (int64_t)lc.dev->cus * 4;
        acc_t* part = static_cast<acc_t*>(partial_mem);
        k_partials<P, Src><<<(unsigned)g, kBlock, 0, st>>>(s, n, part);
        skel_status e = launch_check("reduce_partials");
        if (e != SKEL_OK) return e;
        k_finish<P><<<1, kSingleBlock, 0, st>>>(part, (int)g, out);
        return launch_check("reduce_finish");
    }
    case R2_TICKET: return launch_ticket<P>(s, n, out, lc);
    case R6_GATHER: return launch_gather<P>(s, n, out, lc);
    case R3_ATOMIC: {
        int g = grid_for<P>(n, *lc.dev);
        k_set_identity<P><<<1, 1, 0, st>>>(out);
        skel_status e = launch_check("reduce_set_identity");
        if (e != SKEL_OK) return e;
        k_atomic<P, Src><<<(unsigned)g, kBlock, 0, st>>>(s, n, out);
        return launch_check("reduce_atomic");
    }
    default: return fail(SKEL_E_UNSUPPORTED, "reduce variant %d", v);
    }
}

template <int DIN, int DOUT, int OP>
skel_status reduce_typed(int v, const void* x, int64_t n, void* out, LaunchCtx& lc) {
    using P = RP<DIN, DOUT, OP>;
    if constexpr (DOUT == SKEL_F32 && OP == SKEL_SUM) if (v == R4_COMPENSATED) {
        using PC = RPC<DIN>;
        CompSrc<PC> cs{static_cast<const typename PC::in_t*>(x)};
        return launch_ticket<PC>(cs, n, static_cast<float*>(out), lc);
    }
    if constexpr (DOUT == SKEL_F32 && OP == SKEL_SUM) if (v == R5_PAIRWISE) {
        PairSrc<P> ps;
        ps.x = static_cast<const typename P::in_t*>(x);
        return launch_ticket<P>(ps, n, static_cast<float*>(out), lc);
    }
    void* part = nullptr;
    skel_status e = ws_scratch(lc, partial_bytes(*lc.dev), &part);
    if (e != SKEL_OK) return e;
    PlainSrc<P> s{static_cast<const typename P::in_t*>(x)};
    return run_variant<P>(v, s, n, static_cast<typename P::out_t*>(out), lc, part);
}

template <int DIN, int DOUT>
skel_status reduce_op(int v, int op, const void* x, int64_t n, void* out, LaunchCtx& lc) {
    switch (op) {
    case SKEL_SUM: return reduce_typed<DIN, DOUT, SKEL_SUM>(v, x, n, out, lc);
    case SKEL_MIN: return reduce_typed<DIN, DOUT, SKEL_MIN>(v, x, n, out, lc);
    default: return reduce_typed<DIN, DOUT, SKEL_MAX>(v, x, n, out, lc);
    }
}

template <int DIN, int MOP, int OP>
skel_status mapreduce_typed(int v, float p0, float p1, const void* x, const void* y,
                            int64_t n, float* out, LaunchCtx& lc) {
    using P = RP<DIN, SKEL_F32, OP>;
    using in_t = typename P::in_t;
    MapSrc<P, MOP> s{static_cast<const in_t*>(x), static_cast<const in_t*>(y), p0, p1};
    if constexpr (OP == SKEL_SUM) if (v == MR4_COMPENSATED) {
        using PC = RPC<DIN>;
        CompMapSrc<PC, MOP> cs{static_cast<const in_t*>(x), static_cast<const in_t*>(y), p0, p1};
        return launch_ticket<PC>(cs, n, out, lc);
    }
    if constexpr (OP == SKEL_SUM) if (v == MR5_PAIRWISE) {
        PairMapSrc<P, MOP> ps;
        ps.x = static_cast<const in_t*>(x);
        ps.y = static_cast<const in_t*>(y);
        ps.p0 = p0;
        ps.p1 = p1;
        return launch_ticket<P>(ps, n, out, lc);
    }
    if constexpr (DIN == SKEL_F32) if (v == MR0_UNFUSED) {
        // Map into a temporary with the Map skeleton's vector kernel, then the
        // plain two-pass Reduce over the temporary
        size_t tbytes = ((size_t)n * 4 + 255) & ~size_t(255);
        void* mem = nullptr;
        skel_status e = ws_scratch(lc, tbytes + partial_bytes(*lc.dev), &mem);
        if (e != SKEL_OK) return e;
        float* tmp = static_cast<float*>(mem);
        if (n > 0) {
            e = launch_map(M1_VEC4, MOP, p0, p1, static_cast<const float*>(x),
                           static_cast<const float*>(y), tmp, n, lc);
            if (e != SKEL_OK) return e;
        }
        using PF = RP<SKEL_F32, SKEL_F32, OP>;
        PlainSrc<PF> ps{tmp};
        return run_variant<PF>(R1_TWO_PASS, ps, n, out, lc,
                               static_cast<char*>(mem) + tbytes);
    }
    void* part = nullptr;
    skel_status e = ws_scratch(lc, partial_bytes(*lc.dev), &part);
    if (e != SKEL_OK) return e;
    int rv = v == MR1_FUSED_TWO_PASS ? R1_TWO_PASS
             : v == MR2_FUSED_TICKET ? R2_TICKET
             : v == MR3_FUSED_SINGLE_WG ? R0_SINGLE_WG
             : v == MR6_FUSED_GATHER    ? R6_GATHER
                                        : -1;
    if (rv < 0) return fail(SKEL_E_UNSUPPORTED, "mapreduce variant %d", v);
    return run_variant<P>(rv, s, n, out, lc, part);
}

template <int DIN, int MOP>
skel_status mapreduce_op(int v, int op, float p0, float p1, const void* x, const void* y,
                         int64_t n, float* out, LaunchCtx& lc) {
    switch (op) {
    case SKEL_SUM: return mapreduce_typed<DIN, MOP, SKEL_SUM>(v, p0, p1, x, y, n, out, lc);
    case SKEL_MIN: return mapreduce_typed<DIN, MOP, SKEL_MIN>(v, p0, p1, x, y, n, out, lc);
    default: return mapreduce_typed<DIN, MOP, SKEL_MAX>(v, p0, p1, x, y, n, out, lc);
    }
}

}  // namespace

skel_status launch_reduce(int v, int op, skel_dtype din, skel_dtype dout, const void* x,
                          int64_t n, void* out, LaunchCtx& lc) {
    if (din == SKEL_F32) return reduce_op<SKEL_F32, SKEL_F32>(v, op, x, n, out, lc);
    if (din == SKEL_BF16) return reduce_op<SKEL_BF16, SKEL_F32>(v, op, x, n, out, lc);
    if (din == SKEL_I32 && dout == SKEL_I32)
        return reduce_op<SKEL_I32, SKEL_I32>(v, op, x, n, out, lc);
    if (din == SKEL_I32) return reduce_op<SKEL_I32, SKEL_I64>(v, op, x, n, out, lc);
    return reduce_op<SKEL_I64, SKEL_I64>(v, op, x, n, out, lc);
}

skel_status launch_mapreduce(int v, int map_op, float p0, float p1, skel_dtype din,
                             const void* x, const void* y, int64_t n, int op, float* out,
                             LaunchCtx& lc) {
    if (din == SKEL_BF16) {
        switch (map_op) {
        case SKEL_MAP_IDENTITY:
            return mapreduce_op<SKEL_BF16, SKEL_MAP_IDENTITY>(v, op, p0, p1, x, y, n, out, lc);
        case SKEL_MAP_MUL:
            return mapreduce_op<SKEL_BF16, SKEL_MAP_MUL>(v, op, p0, p1, x, y, n, out, lc);
        default:
            return mapreduce_op<SKEL_BF16, SKEL_MAP_SQUARE>(v, op, p0, p1, x, y, n, out, lc);
        }
    }
    switch (map_op) {
    case SKEL_MAP_IDENTITY:
        return mapreduce_op<SKEL_F32, SKEL_MAP_IDENTITY>(v, op, p0, p1, x, y, n, out, lc);
    case SKEL_MAP_AXPY:
        return mapreduce_op<SKEL_F32, SKEL_MAP_AXPY>(v, op, p0, p1, x, y, n, out, lc);
    case SKEL_MAP_AFFINE:
        return mapreduce_op<SKEL_F32, SKEL_MAP_AFFINE>(v, op, p0, p1, x, y, n, out, lc);
    case SKEL_MAP_TANH:
        return mapreduce_op<SKEL_F32, SKEL_MAP_TANH>(v, op, p0, p1, x, y, n, out, lc);
    case SKEL_MAP_AFFINE_TANH:
        return mapreduce_op<SKEL_F32, SKEL_MAP_AFFINE_TANH>(v, op, p0, p1, x, y, n, out, lc);
    case SKEL_MAP_MUL:
        return mapreduce_op<SKEL_F32, SKEL_MAP_MUL>(v, op, p0, p1, x, y, n, out, lc);
    default:
        return mapreduce_op<SKEL_F32, SKEL_MAP_SQUARE>(v, op, p0, p1, x, y, n, out, lc);
    }
}

}  // namespace skel
