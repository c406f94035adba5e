// Scan skeleton kernels (Section III, scan): inclusive out[i] = x[0] op ...
// op x[i]; exclusive out[0] = identity, out[i] = x[0] op ... op x[i-1].  The
// reverse kinds combine from the end (out[i] = x[i] op ... op x[n-1], and its
// exclusive form); they are the adjoints of the forward sum scans and run in
// the single-pass variant, which visits tiles, rows, lanes and vector
// elements in descending order while keeping the ascending 16-byte layout.
//
// Tile layout (all variants): a workgroup of NW wavefronts (16, or 8 for 8-byte
// inputs) owns a tile of NW * 2048 elements; each wavefront owns a contiguous
// slice of 2048 and walks
// it in rows of 64 lanes x one 16-byte vector, so every load and store
// instruction of a wavefront covers one contiguous 1 KiB span (no LDS
// transposition).  Only the raw inputs stay in registers across the
// inter-tile wait: phase 1 needs just each lane's sum and one wavefront
// reduction to produce the tile total, and the row scans (a lane scans its
// own vector serially, the wavefront scans the 64 lane totals with lane
// shifts, rows are chained by a running carry) run after the tile's prefix is
// known.
//
// Variants:
//   S0  one workgroup walks all tiles in order carrying the prefix (small n)
//   S1  reduce-then-scan: tile totals, one workgroup scans the totals, then
//       every tile rescans with its offset (three launches, input read twice)
//   S2  single pass with decoupled look-back: each tile publishes its total
//       as soon as it has it, then wavefront 0 inspects the 64 preceding tile
//       descriptors at once and combines back to the nearest finished prefix;
//       on a retry only the descriptors that were not yet valid are re-read.
//       Tiles are numbered by an atomic counter in start order, so every tile
//       waited on is already resident: the wait always ends.
//   S4  S2 with tiles of two wavefronts (4096 elements for 4-byte inputs,
//       2048 for 8-byte): for arrays of a few million elements, whose 32768-
//       element tiles would leave most CUs idle (2^20 elements: 256 tiles
//       instead of 32)
//   S5  flat look-back over S4's tiles for arrays of at most 1024 of them:
//       tiles numbered by workgroup index, and each tile reads the totals of
//       all its predecessors in one round of parallel loads (no prefix chain,
//       no atomic counter)
//   S3  S2's tile step run by persistent workgroups (one per resident slot)
//       that loop over tile ids; a workgroup takes its next id once its
//       stores are issued, so no workgroup launch sits between one tile's
//       stores and the next tile's loads, and the counter's round trip
//       overlaps the stores' drain (2^27 i32 -> i64 exclusive: 310 us against
//       337 us for S2 on MI355X).
//
// Tile descriptors are self-validating tagged words (two per tile), written
// and read with single-copy-atomic device-scope accesses, so no fences and no
// clearing pass are needed; the host gives every call a fresh epoch.  The
// look-back wait is bounded: on expiry the kernel raises a flag that
// skel_sync reports, and finishes (with wrong values) instead of hanging.
#include <mutex>

#include "kcommon.hpp"
#include "dispatch.hpp"
#include "kepoch.hpp"
#include "launch.hpp"

#ifndef SKEL_SCAN_WAVES
#define SKEL_SCAN_WAVES 16
#endif


namespace skel {
namespace {

using namespace dev;

constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kFlatPerLane = 8;  // S5: descriptors each lane reads per round

template <int DIN, int DOUT, int OP, int WAVES = SKEL_SCAN_WAVES>
struct SP {
    using in_t = typename Stored<DIN>::type;
    using out_t = typename Stored<DOUT>::type;
    using acc_t = typename Acc<DIN, DOUT, OP>::type;
    using C = Comb<acc_t, OP>;
    static constexpr int E = 16 / sizeof(in_t);           // elements per lane per row
    static constexpr int R = sizeof(in_t) == 4 ? 8 : 16;  // rows per wavefront
    static constexpr int kWaveElems = kWave * E * R;      // 2048
    // wavefronts per workgroup: 16 for 4-byte inputs; 8 for 8-byte inputs,
    // whose raw rows need twice the registers
    static constexpr int NW = sizeof(in_t) == 4 ? WAVES : (WAVES > 1 ? WAVES / 2 : 1);
    static constexpr int kBlock = NW * kWave;
    static constexpr int64_t kTile = (int64_t)NW * kWaveElems;
};

template <class P>
using Raw = typename P::in_t[P::R][P::E];

template <class P>
__device__ __forceinline__ int64_t lane_base(int64_t tile) {
    return tile * P::kTile + (int64_t)(threadIdx.x / kWave) * P::kWaveElems +
           (int64_t)lane() * P::E;
}

// Load the lane's share of `tile` (rows of 16-byte vectors); NT marks the
// loads non-temporal (input read once: measured a few percent faster for the
// single-pass scan).
template <class P, bool FULL, bool NT = false>
__device__ __forceinline__ void tile_load(const typename P::in_t* in, int64_t n, int64_t tile,
                                          Raw<P>& raw) {
    const int64_t b = lane_base<P>(tile);
#pragma unroll
    for (int r = 0; r < P::R; ++r) {
        const int64_t idx = b + (int64_t)r * kWave * P::E;
        if (FULL || idx + P::E <= n) {
            if constexpr (NT) load16_nt(in + idx, raw[r]);
            else load16(in + idx, raw[r]);
        } else {
#pragma unroll
            for (int e = 0; e < P::E; ++e) raw[r][e] = idx + e < n ? in[idx + e] : 0;
        }
    }
}

// op over the lane's elements below n
template <class P, bool FULL>
__device__ __forceinline__ typename P::acc_t lane_total(int64_t n, int64_t tile,
                                                        const Raw<P>& raw) {
    using C = typename P::C;
    const int64_t b = lane_base<P>(tile);
    typename P::acc_t t = C::id();
#pragma unroll
    for (int r = 0; r < P::R; ++r)
#pragma unroll
        for (int e = 0; e < P::E; ++e)
            if (FULL || b + (int64_t)r * kWave * P::E + e < n)
                t = C::op(t, widen<typename P::acc_t>(raw[r][e]));
    return t;
}

// Compiler-only barrier on the raw inputs (emits no instruction): without it
// the compiler keeps the widened values of phase 1 alive across the tile wait
// to reuse them in the store phase, which doubles the live registers.
template <class P>
__device__ __forceinline__ void keep_raw_only(Raw<P>& raw) {
#pragma unroll
    for (int r = 0; r < P::R; ++r)
#pragma unroll
        for (int e = 0; e < P::E; ++e) asm volatile("" : "+v"(raw[r][e]));
}

// Scan the wavefront's slice given its exclusive prefix, and store it.  REV:
// the slice is combined from its last element down (the prefix then holds
// everything after the slice).
// Returns prefix op (the slice's elements below n).
template <class P, bool FULL, bool REV = false>
__device__ __forceinline__ typename P::acc_t tile_scan_store(typename P::out_t* out, int64_t n,
                                                             int64_t tile, const Raw<P>& raw,
                                                             typename P::acc_t prefix,
                                                             bool exclusive) {
    using acc_t = typename P::acc_t;
    using out_t = typename P::out_t;
    using C = typename P::C;
    constexpr int E = P::E;
    const int l = lane();
    const int64_t b = lane_base<P>(tile);
    acc_t running = prefix;
#pragma unroll
    for (int rr = 0; rr < P::R; ++rr) {
        const int r = REV ? P::R - 1 - rr : rr;
        const int64_t idx = b + (int64_t)r * kWave * E;
        acc_t loc[E];  // lane-local inclusive scan of the row vector (in scan order)
        acc_t t = C::id();
#pragma unroll
        for (int ee = 0; ee < E; ++ee) {
            const int e = REV ? E - 1 - ee : ee;
            const acc_t x = (FULL || idx + e < n) ? widen<acc_t>(raw[r][e]) : C::id();
            t = C::op(t, x);
            loc[e] = t;
        }
        const acc_t incl = REV ? wave_inclusive_suffix_scan<C>(t) : wave_inclusive_scan<C>(t);
        const acc_t tot = lane_value(incl, REV ? 0 : kWave - 1);
        const acc_t ex = REV ? wave_shift_down(incl, C::id()) : wave_shift_up(incl, C::id());
        const bool first = REV ? l == kWave - 1 : l == 0;
        const acc_t base = C::op(running, first ? C::id() : ex);
        out_t o[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int before = REV ? e + 1 : e - 1;  // previous element in scan order
            const bool none = REV ? e == E - 1 : e == 0;
            const acc_t v = exclusive ? (none ? base : C::op(base, loc[before]))
                                      : C::op(base, loc[e]);
            o[e] = (out_t)v;
        }
        if (FULL || idx + E <= n) {
            // plain stores: with a row's stores outstanding per lane they
            // stream faster than non-temporal ones (i32 -> i64 exclusive scan
            // of 2^27: 353 us against 417 us)
            store_vecs<out_t, E>(out + idx, o);
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (idx + e < n) out[idx + e] = o[e];
        }
        running = C::op(running, tot);
        // one row at a time: keeps the live registers to one row's temporaries
        // (interleaving rows would spill at 1024 lanes per workgroup)
        __builtin_amdgcn_sched_barrier(0);
    }
    return running;
}

// Wavefront totals -> LDS; returns (exclusive prefix of this wavefront within
// the tile, tile total) in every thread.  Contains one barrier.
template <class P, bool REV = false>
__device__ __forceinline__ void tile_totals(typename P::acc_t lane_t, typename P::acc_t* s_wtot,
                                            typename P::acc_t* wex, typename P::acc_t* agg) {
    using C = typename P::C;
    const int w = threadIdx.x / kWave;
    const typename P::acc_t wt = wave_reduce<C>(lane_t);
    if (lane() == 0) s_wtot[w] = wt;
    __syncthreads();
    *wex = C::id();
    *agg = C::id();
#pragma unroll
    for (int k = 0; k < P::NW; ++k) {
        const typename P::acc_t t = s_wtot[k];
        if (REV ? k > w : k < w) *wex = C::op(*wex, t);
        *agg = C::op(*agg, t);
    }
}

// --------------------------------------------------------- tile descriptors
// two self-validating words per tile (see tagged_put / tagged_get)
enum { ST_INVALID = 0, ST_AGG = 1, ST_PREFIX = 2 };

template <class A>
__device__ __forceinline__ void publish(u64* st, int64_t t, int state, A val, uint32_t epoch) {
    tagged_put(st + 2 * t, state, epoch, val);
}

// Run by one whole wavefront.  Publishes the tile total, finds the exclusive
// prefix of the tile from its predecessors' descriptors, publishes the
// inclusive prefix, and returns the exclusive prefix (in every lane).  Lane l
// inspects tile base - l; a descriptor once seen valid (AGG or PREFIX) is
// final for this call, so a retry re-reads only the lanes still invalid.
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
    int s = ST_INVALID;
    acc_t val = C::id();
    while (true) {
        if (s == ST_INVALID) {
            const int64_t j = base - l;
            s = j >= 0 ? tagged_get(status + 2 * j, epoch, val) : ST_PREFIX;
            if (j < 0) val = C::id();
        }
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
        s = ST_INVALID;
    }
    if (l == 0) publish(status, tile, ST_PREFIX, C::op(excl, agg), epoch);
    return excl;
}

// ------------------------------------------------------------------ kernels
// `seq` is the tile's position in scan order (descriptor index), `tile` the
// data tile it covers (they differ for the reverse kinds)
// s_next (persistent form only): thread 0 takes the workgroup's next tile id
// after issuing this tile's stores, so the counter's round trip overlaps their
// drain
template <class P, bool FULL, bool REV>
__device__ __forceinline__ void lookback_tile(const typename P::in_t* in,
                                              typename P::out_t* out, int64_t n, int64_t seq,
                                              int64_t tile, int exclusive, u64* status,
                                              u64* sync, uint32_t epoch,
                                              int64_t* s_next = nullptr) {
    using acc_t = typename P::acc_t;
    __shared__ acc_t s_wtot[P::NW];
    __shared__ acc_t s_prefix;
    Raw<P> raw;
    tile_load<P, FULL, true>(in, n, tile, raw);
    acc_t wex, agg;
    tile_totals<P, REV>(lane_total<P, FULL>(n, tile, raw), s_wtot, &wex, &agg);
    if (threadIdx.x < kWave) {
        const acc_t e = lookback<P>(status, seq, agg, epoch, sync + SYNC_ERROR);
        if (threadIdx.x == 0) s_prefix = e;
    }
    __syncthreads();
    keep_raw_only<P>(raw);
    tile_scan_store<P, FULL, REV>(out, n, tile, raw, P::C::op(s_prefix, wex), exclusive != 0);
    // the next id is taken only once this tile's stores are issued: an id held
    // longer delays the tiles after it, which wait on its descriptor (taking
    // it before the stores measured 3% slower, a whole tile ahead 34%)
    if (s_next != nullptr && threadIdx.x == 0)
        *s_next = (int64_t)atomicAdd(&sync[SYNC_TILE_COUNTER], 1ull);
}

template <class P, bool REV>
__global__ __launch_bounds__(P::kBlock) void scan_lookback(const typename P::in_t* in,
                                                        typename P::out_t* out, int64_t n,
                                                        int64_t ntiles, int exclusive,
                                                        u64* status, u64* sync) {
    __shared__ int64_t s_tile;
    __shared__ uint32_t s_epoch;
    if (threadIdx.x == 0) {
        s_epoch = epoch_of_call(sync);  // before taking a tile id (see below)
        const u64 t = atomicAdd(&sync[SYNC_TILE_COUNTER], 1ull);
        if (t == (u64)ntiles - 1)  // every other tile id has been taken
            __hip_atomic_store(&sync[SYNC_TILE_COUNTER], 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        s_tile = (int64_t)t;
    }
    __syncthreads();
    const int64_t seq = s_tile;
    const int64_t tile = REV ? ntiles - 1 - seq : seq;  // data tile in scan order
    const uint32_t epoch = s_epoch;
    if ((tile + 1) * P::kTile <= n)
        lookback_tile<P, true, REV>(in, out, n, seq, tile, exclusive, status, sync, epoch);
    else
        lookback_tile<P, false, REV>(in, out, n, seq, tile, exclusive, status, sync, epoch);
    // The workgroup that finishes last (every other one has passed its last
    // descriptor access) resets the counter and advances the epoch for the
    // next call.
    if (threadIdx.x == 0) {
        const u64 d = atomicAdd(&sync[SYNC_DONE], 1ull);
        if (d == (u64)ntiles - 1) {
            __hip_atomic_store(&sync[SYNC_DONE], 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            epoch_advance(sync);
        }
    }
}

// Persistent form: one workgroup per resident slot loops over tile ids taken
// from the counter (ids >= ntiles end the loop).  A tile waits only on tiles
// with smaller ids, all held by running workgroups that never wait on larger
// ids, so every wait ends.  Every workgroup takes exactly one id >= ntiles;
// the last one to leave has seen every tile finish and every id taken, so it
// resets the counters and advances the epoch.
template <class P, bool REV>
__global__ __launch_bounds__(P::kBlock) void scan_lookback_persist(
    const typename P::in_t* in, typename P::out_t* out, int64_t n, int64_t ntiles,
    int exclusive, u64* status, u64* sync) {
    __shared__ int64_t s_tile;
    __shared__ uint32_t s_epoch;
    if (threadIdx.x == 0) {
        s_epoch = epoch_of_call(sync);
        s_tile = (int64_t)atomicAdd(&sync[SYNC_TILE_COUNTER], 1ull);
    }
    __syncthreads();
    const uint32_t epoch = s_epoch;
    int64_t seq = s_tile;
    while (seq < ntiles) {
        const int64_t tile = REV ? ntiles - 1 - seq : seq;
        if ((tile + 1) * P::kTile <= n)
            lookback_tile<P, true, REV>(in, out, n, seq, tile, exclusive, status, sync, epoch,
                                        &s_tile);
        else
            lookback_tile<P, false, REV>(in, out, n, seq, tile, exclusive, status, sync, epoch,
                                         &s_tile);
        __syncthreads();
        seq = s_tile;
        __syncthreads();  // s_tile is rewritten during the next tile
    }
    if (threadIdx.x == 0) {
        const u64 d = atomicAdd(&sync[SYNC_DONE], 1ull);
        if (d == (u64)gridDim.x - 1) {
            __hip_atomic_store(&sync[SYNC_TILE_COUNTER], 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&sync[SYNC_DONE], 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            epoch_advance(sync);
        }
    }
}

// S5: flat look-back.  The tile is the workgroup index: workgroups start in
// index order, so every tile waited on has already started (and with at most
// kFlatMaxTiles small tiles all of them are resident at once).  Each tile
// publishes its total, then every lane of the workgroup reads its share of the
// totals of all preceding tiles -- one round of parallel loads, re-reading only
// those not yet valid -- and the workgroup combines them.  A tile so waits for
// one publish-to-read latency, not for a chain of prefixes, and takes no
// ticket from an atomic counter (device-scope atomics on one word serialise).
// The last tile in scan order advances the epoch once it has seen every other
// tile's total: by then every tile has read this call's epoch.
template <class P>
__device__ __forceinline__ typename P::acc_t flat_prefix(u64* status, int64_t seq,
                                                         uint32_t epoch, u64* err) {
    using acc_t = typename P::acc_t;
    using C = typename P::C;
    acc_t a = C::id();
    for (int64_t base = 0; base < seq; base += (int64_t)kFlatPerLane * P::kBlock) {
        acc_t v[kFlatPerLane];
        bool ready[kFlatPerLane];
#pragma unroll
        for (int k = 0; k < kFlatPerLane; ++k) {
            v[k] = C::id();
            ready[k] = base + k * P::kBlock + (int64_t)threadIdx.x >= seq;
        }
        uint32_t spins = 0;
        while (true) {
            bool all = true;
#pragma unroll
            for (int k = 0; k < kFlatPerLane; ++k) {
                if (ready[k]) continue;
                const int64_t j = base + k * P::kBlock + threadIdx.x;
                ready[k] = tagged_get(status + 2 * j, epoch, v[k]) != ST_INVALID;
                all = all && ready[k];
            }
            if (all) break;
            if (++spins > kSpinLimit) {  // bounded: flag it and finish
                atomicOr(err, 1ull);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int k = 0; k < kFlatPerLane; ++k) a = C::op(a, ready[k] ? v[k] : C::id());
    }
    return a;
}

template <class P, bool FULL, bool REV>
__device__ __forceinline__ void flat_tile(const typename P::in_t* in, typename P::out_t* out,
                                          int64_t n, int64_t seq, int64_t tile, int64_t ntiles,
                                          int exclusive, u64* status, u64* sync) {
    using acc_t = typename P::acc_t;
    using C = typename P::C;
    __shared__ acc_t s_wtot[P::NW];
    __shared__ acc_t s_red[P::NW];
    __shared__ acc_t s_prefix;
    __shared__ uint32_t s_epoch;
    uint32_t ep = 0;
    if (threadIdx.x == 0) ep = epoch_of_call(sync);  // in flight with the tile's loads
    Raw<P> raw;
    tile_load<P, FULL, true>(in, n, tile, raw);
    acc_t wex, agg;
    tile_totals<P, REV>(lane_total<P, FULL>(n, tile, raw), s_wtot, &wex, &agg);
    if (threadIdx.x == 0) {
        s_epoch = ep;
        if (seq + 1 < ntiles) publish(status, seq, ST_AGG, agg, ep);
    }
    __syncthreads();
    const acc_t part = flat_prefix<P>(status, seq, s_epoch, sync + SYNC_ERROR);
    const acc_t pre = block_reduce<C>(part, s_red);
    if (threadIdx.x == 0) {
        s_prefix = pre;
        if (seq == ntiles - 1) epoch_advance(sync);
    }
    __syncthreads();
    keep_raw_only<P>(raw);
    tile_scan_store<P, FULL, REV>(out, n, tile, raw, C::op(s_prefix, wex), exclusive != 0);
}

template <class P, bool REV>
__global__ __launch_bounds__(P::kBlock) void scan_flat(const typename P::in_t* in,
                                                       typename P::out_t* out, int64_t n,
                                                       int64_t ntiles, int exclusive,
                                                       u64* status, u64* sync) {
    const int64_t seq = blockIdx.x;
    const int64_t tile = REV ? ntiles - 1 - seq : seq;  // data tile in scan order
    if ((tile + 1) * P::kTile <= n)
        flat_tile<P, true, REV>(in, out, n, seq, tile, ntiles, exclusive, status, sync);
    else
        flat_tile<P, false, REV>(in, out, n, seq, tile, ntiles, exclusive, status, sync);
}

// S1 pass 1: tile totals
template <class P, bool FULL>
__device__ __forceinline__ typename P::acc_t tile_sum(const typename P::in_t* in, int64_t n,
                                                      int64_t tile) {
    Raw<P> raw;
    tile_load<P, FULL>(in, n, tile, raw);
    return lane_total<P, FULL>(n, tile, raw);
}

template <class P>
__global__ __launch_bounds__(P::kBlock) void scan_tile_totals(const typename P::in_t* in, int64_t n,
                                                           typename P::acc_t* sums) {
    __shared__ typename P::acc_t lds[P::NW];
    const int64_t tile = blockIdx.x;
    typename P::acc_t a = (tile + 1) * P::kTile <= n ? tile_sum<P, true>(in, n, tile)
                                                     : tile_sum<P, false>(in, n, tile);
    a = block_reduce<typename P::C>(a, lds);
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
        const acc_t lex = wave_shift_up(incl, C::id());
        if (i < ntiles) sums[i] = C::op(carry, C::op(wex, lex));
        carry = C::op(carry, total);
        __syncthreads();
    }
}

// S1 pass 3: rescan every tile with its offset
template <class P, bool FULL>
__device__ __forceinline__ void apply_tile(const typename P::in_t* in, typename P::out_t* out,
                                           int64_t n, int64_t tile, typename P::acc_t offset,
                                           int exclusive) {
    __shared__ typename P::acc_t s_wtot[P::NW];
    Raw<P> raw;
    tile_load<P, FULL>(in, n, tile, raw);
    typename P::acc_t wex, agg;
    tile_totals<P>(lane_total<P, FULL>(n, tile, raw), s_wtot, &wex, &agg);
    keep_raw_only<P>(raw);
    tile_scan_store<P, FULL>(out, n, tile, raw, P::C::op(offset, wex), exclusive != 0);
}

template <class P>
__global__ __launch_bounds__(P::kBlock) void scan_tile_apply(const typename P::in_t* in,
                                                          typename P::out_t* out, int64_t n,
                                                          const typename P::acc_t* offs,
                                                          int exclusive) {
    const int64_t tile = blockIdx.x;
    if ((tile + 1) * P::kTile <= n)
        apply_tile<P, true>(in, out, n, tile, offs[tile], exclusive);
    else
        apply_tile<P, false>(in, out, n, tile, offs[tile], exclusive);
}

// S0: one workgroup, tiles in order; the carry is held identically by every
// thread (it is combined from the same LDS totals)
template <class P, bool FULL>
__device__ __forceinline__ typename P::acc_t single_tile(const typename P::in_t* in,
                                                         typename P::out_t* out, int64_t n,
                                                         int64_t tile, typename P::acc_t carry,
                                                         int exclusive) {
    __shared__ typename P::acc_t s_wtot[P::NW];
    Raw<P> raw;
    tile_load<P, FULL>(in, n, tile, raw);
    typename P::acc_t wex, agg;
    tile_totals<P>(lane_total<P, FULL>(n, tile, raw), s_wtot, &wex, &agg);
    keep_raw_only<P>(raw);
    tile_scan_store<P, FULL>(out, n, tile, raw, P::C::op(carry, wex), exclusive != 0);
    __syncthreads();  // s_wtot is rewritten by the next tile
    return P::C::op(carry, agg);
}

template <class P>
__global__ __launch_bounds__(P::kBlock) void scan_single(const typename P::in_t* in,
                                                      typename P::out_t* out, int64_t n,
                                                      int64_t ntiles, int exclusive) {
    typename P::acc_t carry = P::C::id();
    for (int64_t tile = 0; tile < ntiles; ++tile) {
        if ((tile + 1) * P::kTile <= n) carry = single_tile<P, true>(in, out, n, tile, carry, exclusive);
        else carry = single_tile<P, false>(in, out, n, tile, carry, exclusive);
    }
}

// ----------------------------------------------------------- row-wise scans
// Every row of a rows x cols matrix scanned on its own (a batch of Scan
// instances of one length).  SR1: one wavefront per row, walking it in chunks
// of 2048 elements laid out like one wavefront's slice of a tile and carrying
// the running prefix from chunk to chunk (REV: from the row's end).  Rows
// whose starts are not 16-byte aligned take 64-element chunks of single-element
// accesses instead.
template <int DIN, int DOUT, int OP>
struct SPW : SP<DIN, DOUT, OP> {
    static constexpr int NW = 1;
    static constexpr int kBlock = kWave;
    static constexpr int64_t kTile = SP<DIN, DOUT, OP>::kWaveElems;
};

template <class P, bool REV>
__global__ __launch_bounds__(kWave) void scan_rows_vec(const typename P::in_t* in,
                                                       typename P::out_t* out, int64_t rows,
                                                       int64_t cols, int exclusive) {
    using acc_t = typename P::acc_t;
    const int64_t nch = (cols + P::kTile - 1) / P::kTile;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const typename P::in_t* src = in + row * cols;
        typename P::out_t* dst = out + row * cols;
        acc_t carry = P::C::id();
        for (int64_t q = 0; q < nch; ++q) {
            const int64_t ch = REV ? nch - 1 - q : q;
            Raw<P> raw;
            if ((ch + 1) * P::kTile <= cols) {
                tile_load<P, true, true>(src, cols, ch, raw);
                keep_raw_only<P>(raw);
                carry = tile_scan_store<P, true, REV>(dst, cols, ch, raw, carry, exclusive != 0);
            } else {
                tile_load<P, false, true>(src, cols, ch, raw);
                keep_raw_only<P>(raw);
                carry = tile_scan_store<P, false, REV>(dst, cols, ch, raw, carry, exclusive != 0);
            }
        }
    }
}

template <class P, bool REV>
__global__ __launch_bounds__(kWave) void scan_rows_scalar(const typename P::in_t* in,
                                                          typename P::out_t* out, int64_t rows,
                                                          int64_t cols, int exclusive) {
    using acc_t = typename P::acc_t;
    using C = typename P::C;
    const int l = lane();
    const int64_t nch = (cols + kWave - 1) / kWave;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const typename P::in_t* src = in + row * cols;
        typename P::out_t* dst = out + row * cols;
        acc_t carry = C::id();
        for (int64_t q = 0; q < nch; ++q) {
            const int64_t i = (REV ? nch - 1 - q : q) * kWave + l;
            const acc_t x = i < cols ? widen<acc_t>(src[i]) : C::id();
            const acc_t incl = REV ? wave_inclusive_suffix_scan<C>(x) : wave_inclusive_scan<C>(x);
            const acc_t nb = REV ? wave_shift_down(incl, C::id()) : wave_shift_up(incl, C::id());
            const bool first = REV ? l == kWave - 1 : l == 0;
            const acc_t v = C::op(carry, exclusive ? (first ? C::id() : nb) : incl);
            if (i < cols) dst[i] = (typename P::out_t)v;
            carry = C::op(carry, lane_value(incl, REV ? 0 : kWave - 1));
        }
    }
}

// --------------------------------------------------------------- launchers
// S1's three launches; `sums` holds one accumulator per tile (written by the
// first launch before the others read it, so it needs no clearing)
template <class P>
skel_status reduce_then_scan(const typename P::in_t* in, typename P::out_t* out, int64_t n,
                             int excl, typename P::acc_t* sums, hipStream_t st) {
    const int64_t ntiles = (n + P::kTile - 1) / P::kTile;
    skel_status e;
    scan_tile_totals<P><<<(unsigned)ntiles, P::kBlock, 0, st>>>(in, n, sums);
    if ((e = launch_check("scan_tile_totals")) != SKEL_OK) return e;
    scan_tile_offsets<P><<<1, 1024, 0, st>>>(sums, ntiles);
    if ((e = launch_check("scan_tile_offsets")) != SKEL_OK) return e;
    scan_tile_apply<P><<<(unsigned)ntiles, P::kBlock, 0, st>>>(in, out, n, sums, excl);
    return launch_check("scan_tile_apply");
}

template <int DIN, int DOUT, int OP>
skel_status scan_typed(int v, int kind, const void* x, void* y, int64_t n, LaunchCtx& lc) {
    using P = SP<DIN, DOUT, OP>;
    using in_t = typename P::in_t;
    using out_t = typename P::out_t;
    using acc_t = typename P::acc_t;
    const in_t* in = static_cast<const in_t*>(x);
    out_t* out = static_cast<out_t*>(y);
    const int64_t ntiles = (n + P::kTile - 1) / P::kTile;
    const bool rev = kind == SKEL_REVERSE_INCLUSIVE || kind == SKEL_REVERSE_EXCLUSIVE;
    const int excl = (kind == SKEL_EXCLUSIVE || kind == SKEL_REVERSE_EXCLUSIVE) ? 1 : 0;
    hipStream_t st = lc.stream;
    if (rev && v != S2_LOOKBACK && v != S3_PERSISTENT_LOOKBACK && v != S4_SMALL_TILE_LOOKBACK &&
        v != S5_FLAT_LOOKBACK)
        return fail(SKEL_E_UNSUPPORTED, "reverse scans run in the single-pass variants only");
    if (v == S5_FLAT_LOOKBACK) {
        using PS = SP<DIN, DOUT, OP, 2>;
        static_assert(PS::kTile == scan_flat_tile(DIN), "S5 tile size known to the plan");
        const int64_t nts = (n + PS::kTile - 1) / PS::kTile;
        if (nts > kFlatMaxTiles)
            return fail(SKEL_E_UNSUPPORTED, "S5 takes at most %lld elements of this type",
                        (long long)(kFlatMaxTiles * PS::kTile));
        void* status = nullptr;
        skel_status e = ws_status(lc, (size_t)nts * 16, &status);
        if (e != SKEL_OK) return e;
        if (rev)
            scan_flat<PS, true><<<(unsigned)nts, PS::kBlock, 0, st>>>(
                in, out, n, nts, excl, static_cast<u64*>(status), lc.ws->sync);
        else
            scan_flat<PS, false><<<(unsigned)nts, PS::kBlock, 0, st>>>(
                in, out, n, nts, excl, static_cast<u64*>(status), lc.ws->sync);
        return launch_check("scan_flat");
    }
    if (v == S4_SMALL_TILE_LOOKBACK) {
        using PS = SP<DIN, DOUT, OP, 2>;
        const int64_t nts = (n + PS::kTile - 1) / PS::kTile;
        void* status = nullptr;
        skel_status e = ws_status(lc, (size_t)nts * 16, &status);
        if (e != SKEL_OK) return e;
        if (rev)
            scan_lookback<PS, true><<<(unsigned)nts, PS::kBlock, 0, st>>>(
                in, out, n, nts, excl, static_cast<u64*>(status), lc.ws->sync);
        else
            scan_lookback<PS, false><<<(unsigned)nts, PS::kBlock, 0, st>>>(
                in, out, n, nts, excl, static_cast<u64*>(status), lc.ws->sync);
        return launch_check("scan_lookback_small");
    }
    switch (v) {
    case S0_SINGLE_WG:
        scan_single<P><<<1, P::kBlock, 0, st>>>(in, out, n, ntiles, excl);
        return launch_check("scan_single");
    case S1_REDUCE_THEN_SCAN: {
        void* mem = nullptr;
        skel_status e = ws_scratch(lc, (size_t)ntiles * sizeof(acc_t), &mem);
        if (e != SKEL_OK) return e;
        return reduce_then_scan<P>(in, out, n, excl, static_cast<acc_t*>(mem), st);
    }
    case S3_PERSISTENT_LOOKBACK: {
        void* status = nullptr;
        skel_status e = ws_status(lc, (size_t)ntiles * 16, &status);
        if (e != SKEL_OK) return e;
        auto kern = rev ? scan_lookback_persist<P, true> : scan_lookback_persist<P, false>;
        const int64_t slots = resident_slots(reinterpret_cast<const void*>(kern), P::kBlock, lc);
        if (slots < 1) return fail(SKEL_E_HIP, "scan_lookback_persist does not fit a CU");
        kern<<<(unsigned)std::min<int64_t>(ntiles, slots), P::kBlock, 0, st>>>(
            in, out, n, ntiles, excl, static_cast<u64*>(status), lc.ws->sync);
        return launch_check("scan_lookback_persist");
    }
    default: {  // S2_LOOKBACK
        void* status = nullptr;
        skel_status e = ws_status(lc, (size_t)ntiles * 16, &status);
        if (e != SKEL_OK) return e;
        if (rev)
            scan_lookback<P, true><<<(unsigned)ntiles, P::kBlock, 0, st>>>(
                in, out, n, ntiles, excl, static_cast<u64*>(status), lc.ws->sync);
        else
            scan_lookback<P, false><<<(unsigned)ntiles, P::kBlock, 0, st>>>(
                in, out, n, ntiles, excl, static_cast<u64*>(status), lc.ws->sync);
        return launch_check("scan_lookback");
    }
    }
}

template <int DIN, int DOUT, int OP>
skel_status scan_rows_typed(int kind, const void* x, void* y, int64_t rows, int64_t cols,
                            bool vec, LaunchCtx& lc) {
    using P = SPW<DIN, DOUT, OP>;
    const auto* in = static_cast<const typename P::in_t*>(x);
    auto* out = static_cast<typename P::out_t*>(y);
    const bool rev = kind == SKEL_REVERSE_INCLUSIVE || kind == SKEL_REVERSE_EXCLUSIVE;
    const int excl = (kind == SKEL_EXCLUSIVE || kind == SKEL_REVERSE_EXCLUSIVE) ? 1 : 0;
    const unsigned grid = (unsigned)std::min<int64_t>(rows, INT64_C(1) << 20);
    hipStream_t st = lc.stream;
    if (vec) {
        if (rev) scan_rows_vec<P, true><<<grid, kWave, 0, st>>>(in, out, rows, cols, excl);
        else scan_rows_vec<P, false><<<grid, kWave, 0, st>>>(in, out, rows, cols, excl);
        return launch_check("scan_rows_vec");
    }
    if (rev) scan_rows_scalar<P, true><<<grid, kWave, 0, st>>>(in, out, rows, cols, excl);
    else scan_rows_scalar<P, false><<<grid, kWave, 0, st>>>(in, out, rows, cols, excl);
    return launch_check("scan_rows_scalar");
}

template <int DIN, int DOUT>
skel_status scan_rows_op(int kind, int op, const void* x, void* y, int64_t rows, int64_t cols,
                         bool vec, LaunchCtx& lc) {
    switch (op) {
    case SKEL_SUM: return scan_rows_typed<DIN, DOUT, SKEL_SUM>(kind, x, y, rows, cols, vec, lc);
    case SKEL_MIN: return scan_rows_typed<DIN, DOUT, SKEL_MIN>(kind, x, y, rows, cols, vec, lc);
    default: return scan_rows_typed<DIN, DOUT, SKEL_MAX>(kind, x, y, rows, cols, vec, lc);
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

skel_status launch_scan_rows(int kind, int op, skel_dtype din, skel_dtype dout, const void* x,
                             void* y, int64_t rows, int64_t cols, bool vec, LaunchCtx& lc) {
    if (din == SKEL_I32 && dout == SKEL_I32)
        return scan_rows_op<SKEL_I32, SKEL_I32>(kind, op, x, y, rows, cols, vec, lc);
    if (din == SKEL_I32) return scan_rows_op<SKEL_I32, SKEL_I64>(kind, op, x, y, rows, cols, vec, lc);
    if (din == SKEL_I64) return scan_rows_op<SKEL_I64, SKEL_I64>(kind, op, x, y, rows, cols, vec, lc);
    return scan_rows_op<SKEL_F32, SKEL_F32>(kind, op, x, y, rows, cols, vec, lc);
}

skel_status launch_scan(int v, int kind, int op, skel_dtype din, skel_dtype dout,
                        const void* x, void* y, int64_t n, LaunchCtx& lc) {
    if (din == SKEL_I32 && dout == SKEL_I32) return scan_op<SKEL_I32, SKEL_I32>(v, kind, op, x, y, n, lc);
    if (din == SKEL_I32) return scan_op<SKEL_I32, SKEL_I64>(v, kind, op, x, y, n, lc);
    if (din == SKEL_I64) return scan_op<SKEL_I64, SKEL_I64>(v, kind, op, x, y, n, lc);
    return scan_op<SKEL_F32, SKEL_F32>(v, kind, op, x, y, n, lc);
}

}  // namespace skel

// ------------------------------------------------- allocation-free Scan ----
// skel_scan_noalloc runs S1 with its tile totals in a file-scope device array
// instead of the stream's workspace, so a call allocates nothing.  Every GPU
// the library runs on holds its own copy of the array (until the process
// ends); host code reaches it only through the address hipGetSymbolAddress
// returns with that device current, never through the array's name.
namespace skel {

constexpr int64_t kNoAllocTiles = 32768;  // tile totals the array holds (8 bytes each)
static __device__ __align__(256) unsigned long long scratch[kNoAllocTiles];  // 256 KiB

namespace {

constexpr int kNoAllocMaxDevices = 64;
void* g_scratch_addr[kNoAllocMaxDevices];  // per device ordinal
std::mutex g_scratch_mu;

skel_status scratch_address(int device, void** out) {
    if (device < 0 || device >= kNoAllocMaxDevices)
        return fail(SKEL_E_INVAL, "device %d beyond the %d the allocation-free scan tracks",
                    device, kNoAllocMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return fail(SKEL_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                        hipGetErrorString(e));
        }
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return SKEL_OK;
}

template <int DIN, int DOUT, int OP>
skel_status noalloc_typed(const void* x, void* y, int64_t n, int excl, void* sums,
                          hipStream_t st) {
    using P = SP<DIN, DOUT, OP>;
    static_assert(sizeof(typename P::acc_t) <= sizeof(scratch[0]), "one array word per tile");
    return reduce_then_scan<P>(static_cast<const typename P::in_t*>(x),
                               static_cast<typename P::out_t*>(y), n, excl,
                               static_cast<typename P::acc_t*>(sums), st);
}

template <int DIN, int DOUT>
skel_status noalloc_op(int op, const void* x, void* y, int64_t n, int excl, void* sums,
                       hipStream_t st) {
    switch (op) {
    case SKEL_SUM: return noalloc_typed<DIN, DOUT, SKEL_SUM>(x, y, n, excl, sums, st);
    case SKEL_MIN: return noalloc_typed<DIN, DOUT, SKEL_MIN>(x, y, n, excl, sums, st);
    default: return noalloc_typed<DIN, DOUT, SKEL_MAX>(x, y, n, excl, sums, st);
    }
}

// the scan tile of an input type: what bounds n for a given array size
int64_t noalloc_tile(skel_dtype din) {
    return din == SKEL_I64 ? SP<SKEL_I64, SKEL_I64, SKEL_SUM>::kTile
                           : SP<SKEL_I32, SKEL_I32, SKEL_SUM>::kTile;
}

}  // namespace

skel_status scan_noalloc_setup(int device) {
    void* p = nullptr;
    return scratch_address(device, &p);
}

}  // namespace skel

using namespace skel;

extern "C" skel_status skel_scan_noalloc(const void* in, skel_dtype din, void* out,
                                         skel_dtype dout, int64_t n, skel_scan_kind kind,
                                         skel_reduce_op op, void* stream) {
    if (!rt().initialized) return fail(SKEL_E_NOINIT, "skel_init has not been called");
    if (kind == SKEL_REVERSE_INCLUSIVE || kind == SKEL_REVERSE_EXCLUSIVE)
        return fail(SKEL_E_UNSUPPORTED, "the allocation-free scan runs the forward kinds only");
    if (kind != SKEL_INCLUSIVE && kind != SKEL_EXCLUSIVE)
        return fail(SKEL_E_INVAL, "unknown scan kind %d", (int)kind);
    if (op < SKEL_SUM || op > SKEL_MAX) return fail(SKEL_E_INVAL, "unknown scan op %d", (int)op);
    const bool types_ok = (din == SKEL_I32 && (dout == SKEL_I32 || dout == SKEL_I64)) ||
                          (din == SKEL_I64 && dout == SKEL_I64) ||
                          (din == SKEL_F32 && dout == SKEL_F32);
    if (!types_ok)
        return fail(SKEL_E_DTYPE, "Scan %s -> %s not supported",
                    dtype_valid(din) ? dtype_name(din) : "?",
                    dtype_valid(dout) ? dtype_name(dout) : "?");
    if (n < 0) return fail(SKEL_E_INVAL, "negative element count %lld", (long long)n);
    if (n == 0) return SKEL_OK;
    const int64_t tile = noalloc_tile(din);
    if ((n + tile - 1) / tile > kNoAllocTiles)
        return fail(SKEL_E_SHAPE,
                    "n = %lld exceeds the allocation-free maximum of %lld elements for %s "
                    "input (%lld tiles of %lld)", (long long)n,
                    (long long)(kNoAllocTiles * tile), dtype_name(din),
                    (long long)kNoAllocTiles, (long long)tile);
    if (!in || !out) return fail(SKEL_E_INVAL, "null data pointer");
    if (reinterpret_cast<uintptr_t>(in) % 16 != 0 || reinterpret_cast<uintptr_t>(out) % 16 != 0)
        return fail(SKEL_E_INVAL, "in and out must be 16-byte aligned");
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(in), b0 = reinterpret_cast<uintptr_t>(out);
    const uintptr_t a1 = a0 + (uintptr_t)n * dtype_size(din);
    const uintptr_t b1 = b0 + (uintptr_t)n * dtype_size(dout);
    if (a0 < b1 && b0 < a1 && !(a0 == b0 && din == dout))
        return fail(SKEL_E_INVAL, "out must equal in (same types) or not overlap it");
    int device = -1;
    skel_status st = hip_check(hipGetDevice(&device), "hipGetDevice");
    if (st != SKEL_OK) return st;
    void* sums = nullptr;
    st = scratch_address(device, &sums);
    if (st != SKEL_OK) return st;
    const int excl = kind == SKEL_EXCLUSIVE ? 1 : 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (din == SKEL_I32 && dout == SKEL_I32)
        return noalloc_op<SKEL_I32, SKEL_I32>(op, in, out, n, excl, sums, s);
    if (din == SKEL_I32) return noalloc_op<SKEL_I32, SKEL_I64>(op, in, out, n, excl, sums, s);
    if (din == SKEL_I64) return noalloc_op<SKEL_I64, SKEL_I64>(op, in, out, n, excl, sums, s);
    return noalloc_op<SKEL_F32, SKEL_F32>(op, in, out, n, excl, sums, s);
}
