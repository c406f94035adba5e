// Scan skeleton kernels (Section III, scan): inclusive out[i] = x[0] op ...
// op x[i]; exclusive out[0] = identity, out[i] = x[0] op ... op x[i-1].
//
// Tile layout (all variants): a workgroup of 4 wavefronts owns a tile of
// 8192 elements; each wavefront owns a contiguous quarter and walks it in
// rows of 64 lanes x one 16-byte vector, so every load and store instruction
// of a wavefront covers one contiguous 1 KiB span (no LDS transposition).
// Inside a row a lane scans its own vector serially, the wavefront scans the
// 64 lane totals with lane shifts, and rows are chained by a running carry;
// the four wavefront totals meet in LDS.
//
// Variants:
//   S0  one workgroup walks all tiles in order carrying the prefix (small n)
//   S1  reduce-then-scan: tile totals, one workgroup scans the totals, then
//       every tile rescans with its offset (three launches, input read twice)
//   S2  single pass with decoupled look-back: each tile publishes its total
//       as soon as it has it, then wavefront 0 inspects the 64 preceding tile
//       descriptors at once and combines back to the nearest finished prefix.
//       Tiles are numbered by an atomic counter in start order, so every tile
//       waited on is already resident: the wait always ends.
//
// Tile descriptors are 64-bit words [state:2 | epoch:30 | value:32], two per
// tile for 64-bit values.  Each word is written and read with single-copy-
// atomic device-scope accesses and validates itself (state and epoch agree),
// so no fences and no clearing pass are needed; the host gives every call a
// fresh epoch.  The look-back wait is bounded: on expiry the kernel raises a
// flag that skel_sync reports, and finishes (with wrong values) instead of
// hanging.
#include "kcommon.hpp"
#include "dispatch.hpp"
#include "launch.hpp"

namespace skel {
namespace {

using namespace dev;
typedef unsigned long long u64;

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr uint32_t kSpinLimit = 1u << 22;

template <int DIN, int DOUT, int OP>
struct SP {
    using in_t = typename Stored<DIN>::type;
    using out_t = typename Stored<DOUT>::type;
    using acc_t = typename Acc<DIN, DOUT, OP>::type;
    using C = Comb<acc_t, OP>;
    static constexpr int E = 16 / sizeof(in_t);         // elements per lane per row
    static constexpr int R = sizeof(in_t) == 4 ? 8 : 16;  // rows per wavefront
    static constexpr int kWaveElems = kWave * E * R;      // 2048
    static constexpr int kTile = kWaves * kWaveElems;     // 8192
};

template <class P>
struct TileState {
    typename P::acc_t v[P::R][P::E];  // lane-local inclusive scan of each row vector
    typename P::acc_t lex[P::R];      // exclusive prefix of the lane within its row
    typename P::acc_t rtot[P::R];     // row totals
};

// Load the wavefront's quarter of `tile` and scan it locally.  Returns the
// wavefront total.  Elements at or beyond n read as the identity.
template <class P, bool FULL>
__device__ __forceinline__ typename P::acc_t tile_load_scan(const typename P::in_t* in,
                                                            int64_t n, int64_t tile,
                                                            TileState<P>& ts) {
    using acc_t = typename P::acc_t;
    using C = typename P::C;
    constexpr int E = P::E, R = P::R;
    const int w = threadIdx.x / kWave, l = lane();
    const int64_t wbase = tile * P::kTile + (int64_t)w * P::kWaveElems + (int64_t)l * E;
    typename P::in_t raw[R][E];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t idx = wbase + (int64_t)r * kWave * E;
        if (FULL || idx + E <= n) {
            load16(in + idx, raw[r]);
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) raw[r][e] = idx + e < n ? in[idx + e] : 0;
        }
    }
    acc_t wtot = C::id();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t idx = wbase + (int64_t)r * kWave * E;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            acc_t x = (FULL || idx + e < n) ? widen<acc_t>(raw[r][e]) : C::id();
            ts.v[r][e] = e == 0 ? x : C::op(ts.v[r][e - 1], x);
        }
        acc_t incl = wave_inclusive_scan<C>(ts.v[r][E - 1]);
        ts.rtot[r] = __shfl(incl, kWave - 1);
        acc_t ex = __shfl_up(incl, 1);
        ts.lex[r] = l == 0 ? C::id() : ex;
        wtot = C::op(wtot, ts.rtot[r]);
    }
    return wtot;
}

// Write the scanned quarter given the exclusive prefix of the wavefront.
template <class P, bool FULL>
__device__ __forceinline__ void tile_store(typename P::out_t* out, int64_t n, int64_t tile,
                                           const TileState<P>& ts,
                                           typename P::acc_t prefix, bool exclusive) {
    using acc_t = typename P::acc_t;
    using out_t = typename P::out_t;
    using C = typename P::C;
    constexpr int E = P::E, R = P::R;
    const int w = threadIdx.x / kWave, l = lane();
    const int64_t wbase = tile * P::kTile + (int64_t)w * P::kWaveElems + (int64_t)l * E;
    acc_t running = prefix;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t idx = wbase + (int64_t)r * kWave * E;
        const acc_t base = C::op(running, ts.lex[r]);
        out_t o[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            acc_t val;
            if (exclusive) val = e == 0 ? base : C::op(base, ts.v[r][e - 1]);
            else val = C::op(base, ts.v[r][e]);
            o[e] = (out_t)val;
        }
        if (FULL || idx + E <= n) {
            store_nt<out_t, E>(out + idx, o);
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (idx + e < n) out[idx + e] = o[e];
        }
        running = C::op(running, ts.rtot[r]);
    }
}

// --------------------------------------------------------- tile descriptors
enum { ST_INVALID = 0, ST_AGG = 1, ST_PREFIX = 2 };

template <class A>
__device__ __forceinline__ u64 to_bits(A v) {
    if constexpr (sizeof(A) == 4) {
        uint32_t b;
        __builtin_memcpy(&b, &v, 4);
        return b;
    } else {
        u64 b;
        __builtin_memcpy(&b, &v, 8);
        return b;
    }
}
template <class A>
__device__ __forceinline__ A from_bits(u64 b) {
    A v;
    if constexpr (sizeof(A) == 4) {
        uint32_t b32 = (uint32_t)b;
        __builtin_memcpy(&v, &b32, 4);
    } else {
        __builtin_memcpy(&v, &b, 8);
    }
    return v;
}

template <class A>
__device__ __forceinline__ void publish(u64* st, int64_t t, int state, A val, uint32_t epoch) {
    const u64 bits = to_bits(val);
    const u64 tag = ((u64)state << 62) | ((u64)epoch << 32);
    __hip_atomic_store(&st[2 * t], tag | (bits & 0xffffffffull), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    if constexpr (sizeof(A) == 8)
        __hip_atomic_store(&st[2 * t + 1], tag | (bits >> 32), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <class A>
__device__ __forceinline__ int peek(u64* st, int64_t t, uint32_t epoch, A& val) {
    const u64 lo = __hip_atomic_load(&st[2 * t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (((lo >> 32) & 0x3fffffffull) != epoch) return ST_INVALID;
    u64 bits = lo & 0xffffffffull;
    if constexpr (sizeof(A) == 8) {
        const u64 hi = __hip_atomic_load(&st[2 * t + 1], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
        if ((hi >> 32) != (lo >> 32)) return ST_INVALID;  // halves of different states
        bits |= hi << 32;
    }
    val = from_bits<A>(bits);
    return (int)(lo >> 62);
}

// Run by one whole wavefront.  Publishes the tile total, finds the exclusive
// prefix of the tile from its predecessors' descriptors, publishes the
// inclusive prefix, and returns the exclusive prefix (in every lane).
template <class P>
__device__ typename P::acc_t lookback(u64* status, int64_t tile, typename P::acc_t agg,
                                      uint32_t epoch, u64* err) {
    using acc_t = typename P::acc_t;
    using C = typename P::C;
    const int l = lane();
    if (tile == 0) {
        if (l == 0) publish(status, 0, ST_PREFIX, agg, epoch);
        return C::id();
    }
    if (l == 0) publish(status, tile, ST_AGG, agg, epoch);
    acc_t excl = C::id();
    int64_t base = tile - 1;
    uint32_t spins = 0;
    while (true) {
        const int64_t j = base - l;
        acc_t val = C::id();
        const int s = j >= 0 ? peek(status, j, epoch, val) : ST_PREFIX;
        const u64 pre = __ballot(s == ST_PREFIX);
        const u64 inv = __ballot(s == ST_INVALID);
        const int p = pre ? __ffsll((long long)pre) - 1 : kWave;
        const u64 need = p >= kWave - 1 ? ~0ull : ((2ull << p) - 1);
        if (inv & need) {
            if (++spins > kSpinLimit) {
                if (l == 0) atomicOr(err, 1ull);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl = C::op(excl, wave_reduce<C>(l <= p ? val : C::id()));
        if (p < kWave) break;
        base -= kWave;
    }
    if (l == 0) publish(status, tile, ST_PREFIX, C::op(excl, agg), epoch);
    return excl;
}

// ------------------------------------------------------------------ kernels
template <class P>
__device__ __forceinline__ void combine_waves(typename P::acc_t* s_wtot, typename P::acc_t* wex,
                                              typename P::acc_t* agg) {
    using C = typename P::C;
    const int w = threadIdx.x / kWave;
    *wex = C::id();
    *agg = C::id();
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        typename P::acc_t t = s_wtot[k];
        if (k < w) *wex = C::op(*wex, t);
        *agg = C::op(*agg, t);
    }
}

template <class P>
__global__ __launch_bounds__(kBlock) void scan_lookback(const typename P::in_t* in,
                                                        typename P::out_t* out, int64_t n,
                                                        int64_t ntiles, int exclusive,
                                                        u64* status, u64* sync,
                                                        uint32_t epoch) {
    using acc_t = typename P::acc_t;
    __shared__ int64_t s_tile;
    __shared__ acc_t s_wtot[kWaves];
    __shared__ acc_t s_prefix;
    if (threadIdx.x == 0) {
        const u64 t = atomicAdd(&sync[SYNC_TILE_COUNTER], 1ull);
        if (t == (u64)ntiles - 1)  // every other tile id has been taken
            __hip_atomic_store(&sync[SYNC_TILE_COUNTER], 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        s_tile = (int64_t)t;
    }
    __syncthreads();
    const int64_t tile = s_tile;
    const bool full = (tile + 1) * P::kTile <= n;
    TileState<P> ts;
    acc_t wtot = full ? tile_load_scan<P, true>(in, n, tile, ts)
                      : tile_load_scan<P, false>(in, n, tile, ts);
    const int w = threadIdx.x / kWave;
    if (lane() == 0) s_wtot[w] = wtot;
    __syncthreads();
    acc_t wex, agg;
    combine_waves<P>(s_wtot, &wex, &agg);
    if (w == 0) {
        acc_t e = lookback<P>(status, tile, agg, epoch, sync + SYNC_ERROR);
        if (lane() == 0) s_prefix = e;
    }
    __syncthreads();
    const acc_t pre = P::C::op(s_prefix, wex);
    if (full) tile_store<P, true>(out, n, tile, ts, pre, exclusive != 0);
    else tile_store<P, false>(out, n, tile, ts, pre, exclusive != 0);
}

// S1 pass 1: tile totals
template <class P>
__global__ __launch_bounds__(kBlock) void scan_tile_totals(const typename P::in_t* in, int64_t n,
                                                           typename P::acc_t* sums) {
    using acc_t = typename P::acc_t;
    using C = typename P::C;
    constexpr int E = P::E, R = P::R;
    __shared__ acc_t lds[kWaves];
    const int64_t tile = blockIdx.x;
    const int w = threadIdx.x / kWave, l = lane();
    const int64_t wbase = tile * P::kTile + (int64_t)w * P::kWaveElems + (int64_t)l * E;
    const bool full = (tile + 1) * P::kTile <= n;
    acc_t a = C::id();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t idx = wbase + (int64_t)r * kWave * E;
        typename P::in_t raw[E];
        if (full || idx + E <= n) {
            load16(in + idx, raw);
#pragma unroll
            for (int e = 0; e < E; ++e) a = C::op(a, widen<acc_t>(raw[e]));
        } else {
            for (int e = 0; e < E; ++e)
                if (idx + e < n) a = C::op(a, widen<acc_t>(in[idx + e]));
        }
    }
    a = block_reduce<C>(a, lds);
    if (threadIdx.x == 0) sums[tile] = a;
}

// S1 pass 2: exclusive scan of the tile totals, in place, by one workgroup
template <class P>
__global__ __launch_bounds__(1024) void scan_tile_offsets(typename P::acc_t* sums,
                                                          int64_t ntiles) {
    using acc_t = typename P::acc_t;
    using C = typename P::C;
    constexpr int NW = 1024 / kWave;
    __shared__ acc_t lds[NW];
    const int w = threadIdx.x / kWave, l = lane();
    acc_t carry = C::id();
    for (int64_t base = 0; base < ntiles; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const acc_t v = i < ntiles ? sums[i] : C::id();
        const acc_t incl = wave_inclusive_scan<C>(v);
        if (l == kWave - 1) lds[w] = incl;
        __syncthreads();
        acc_t wex = C::id(), total = C::id();
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            if (k < w) wex = C::op(wex, lds[k]);
            total = C::op(total, lds[k]);
        }
        acc_t lex = __shfl_up(incl, 1);
        if (l == 0) lex = C::id();
        if (i < ntiles) sums[i] = C::op(carry, C::op(wex, lex));
        carry = C::op(carry, total);
        __syncthreads();
    }
}

// S1 pass 3: rescan every tile with its offset
template <class P>
__global__ __launch_bounds__(kBlock) void scan_tile_apply(const typename P::in_t* in,
                                                          typename P::out_t* out, int64_t n,
                                                          const typename P::acc_t* offs,
                                                          int exclusive) {
    using acc_t = typename P::acc_t;
    __shared__ acc_t s_wtot[kWaves];
    const int64_t tile = blockIdx.x;
    const bool full = (tile + 1) * P::kTile <= n;
    TileState<P> ts;
    acc_t wtot = full ? tile_load_scan<P, true>(in, n, tile, ts)
                      : tile_load_scan<P, false>(in, n, tile, ts);
    if (lane() == 0) s_wtot[threadIdx.x / kWave] = wtot;
    __syncthreads();
    acc_t wex, agg;
    combine_waves<P>(s_wtot, &wex, &agg);
    const acc_t pre = P::C::op(offs[tile], wex);
    if (full) tile_store<P, true>(out, n, tile, ts, pre, exclusive != 0);
    else tile_store<P, false>(out, n, tile, ts, pre, exclusive != 0);
}

// S0: one workgroup, tiles in order
template <class P>
__global__ __launch_bounds__(kBlock) void scan_single(const typename P::in_t* in,
                                                      typename P::out_t* out, int64_t n,
                                                      int64_t ntiles, int exclusive) {
    using acc_t = typename P::acc_t;
    __shared__ acc_t s_wtot[kWaves];
    acc_t carry = P::C::id();
    for (int64_t tile = 0; tile < ntiles; ++tile) {
        const bool full = (tile + 1) * P::kTile <= n;
        TileState<P> ts;
        acc_t wtot = full ? tile_load_scan<P, true>(in, n, tile, ts)
                          : tile_load_scan<P, false>(in, n, tile, ts);
        if (lane() == 0) s_wtot[threadIdx.x / kWave] = wtot;
        __syncthreads();
        acc_t wex, agg;
        combine_waves<P>(s_wtot, &wex, &agg);
        const acc_t pre = P::C::op(carry, wex);
        if (full) tile_store<P, true>(out, n, tile, ts, pre, exclusive != 0);
        else tile_store<P, false>(out, n, tile, ts, pre, exclusive != 0);
        carry = P::C::op(carry, agg);
        __syncthreads();
    }
}

// --------------------------------------------------------------- launchers
template <int DIN, int DOUT, int OP>
skel_status scan_typed(int v, int kind, const void* x, void* y, int64_t n, LaunchCtx& lc) {
    using P = SP<DIN, DOUT, OP>;
    using in_t = typename P::in_t;
    using out_t = typename P::out_t;
    using acc_t = typename P::acc_t;
    const in_t* in = static_cast<const in_t*>(x);
    out_t* out = static_cast<out_t*>(y);
    const int64_t ntiles = (n + P::kTile - 1) / P::kTile;
    const int excl = kind == SKEL_EXCLUSIVE ? 1 : 0;
    hipStream_t st = lc.stream;
    switch (v) {
    case S0_SINGLE_WG:
        scan_single<P><<<1, kBlock, 0, st>>>(in, out, n, ntiles, excl);
        return launch_check("scan_single");
    case S1_REDUCE_THEN_SCAN: {
        void* mem = nullptr;
        skel_status e = ws_scratch(lc, (size_t)ntiles * sizeof(acc_t), &mem);
        if (e != SKEL_OK) return e;
        acc_t* sums = static_cast<acc_t*>(mem);
        scan_tile_totals<P><<<(unsigned)ntiles, kBlock, 0, st>>>(in, n, sums);
        if ((e = launch_check("scan_tile_totals")) != SKEL_OK) return e;
        scan_tile_offsets<P><<<1, 1024, 0, st>>>(sums, ntiles);
        if ((e = launch_check("scan_tile_offsets")) != SKEL_OK) return e;
        scan_tile_apply<P><<<(unsigned)ntiles, kBlock, 0, st>>>(in, out, n, sums, excl);
        return launch_check("scan_tile_apply");
    }
    default: {  // S2_LOOKBACK
        void* status = nullptr;
        uint32_t epoch = 0;
        skel_status e = ws_status(lc, (size_t)ntiles * 16, &status, &epoch);
        if (e != SKEL_OK) return e;
        scan_lookback<P><<<(unsigned)ntiles, kBlock, 0, st>>>(
            in, out, n, ntiles, excl, static_cast<u64*>(status), lc.ws->sync, epoch);
        return launch_check("scan_lookback");
    }
    }
}

template <int DIN, int DOUT>
skel_status scan_op(int v, int kind, int op, const void* x, void* y, int64_t n,
                    LaunchCtx& lc) {
    switch (op) {
    case SKEL_SUM: return scan_typed<DIN, DOUT, SKEL_SUM>(v, kind, x, y, n, lc);
    case SKEL_MIN: return scan_typed<DIN, DOUT, SKEL_MIN>(v, kind, x, y, n, lc);
    default: return scan_typed<DIN, DOUT, SKEL_MAX>(v, kind, x, y, n, lc);
    }
}

}  // namespace

skel_status launch_scan(int v, int kind, int op, skel_dtype din, skel_dtype dout,
                        const void* x, void* y, int64_t n, LaunchCtx& lc) {
    if (din == SKEL_I32 && dout == SKEL_I32) return scan_op<SKEL_I32, SKEL_I32>(v, kind, op, x, y, n, lc);
    if (din == SKEL_I32) return scan_op<SKEL_I32, SKEL_I64>(v, kind, op, x, y, n, lc);
    if (din == SKEL_I64) return scan_op<SKEL_I64, SKEL_I64>(v, kind, op, x, y, n, lc);
    return scan_op<SKEL_F32, SKEL_F32>(v, kind, op, x, y, n, lc);
}

}  // namespace skel
