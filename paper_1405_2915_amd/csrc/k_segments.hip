// Segmented Reduce: many vectors of uneven length, stored back to back in one
// container and delimited by an offsets container, reduced in one call:
//   out[s] = op over x[offsets[s]] .. x[offsets[s+1] - 1]
// This is the batched form of the Reduce skeleton (Section III): one skeleton
// instance applied to a set of operands of different sizes.
//
// Variants:
//   B0  per segment: one two-pass Reduce per segment (2 launches each); the
//       plain loop a caller would write
//   B1  persistent work queue: a one-workgroup kernel turns the offsets into
//       an item table (segment, chunk of kChunk elements; empty segments get
//       one empty item), then a grid of 4 workgroups per CU walks the items;
//       a workgroup finds an item's segment with a 64-ary search by one
//       wavefront.
//       Each item's partial goes to an epoch-tagged slot and the item draws
//       its segment's ticket; the workgroup holding a segment's last ticket
//       combines that segment's slots in item order (deterministic).
// Offsets are read with clamping to [0, n], so malformed offsets give
// unspecified sums but never an out-of-bounds access.
#include "kcommon.hpp"
#include "dispatch.hpp"
#include "kepoch.hpp"
#include "launch.hpp"

namespace skel {
namespace {

using namespace dev;

constexpr int kBlock = 256;
// 32768-element items and 4 workgroups per CU measured fastest on the batch
// of 4096 log-uniform vectors (B1: 290 us; 16384-element items 302 us,
// 65536 295 us; 2 workgroups per CU 339 us, 8 per CU 342 us)
#ifndef SKEL_SEG_CHUNK
#define SKEL_SEG_CHUNK 32768
#endif
#ifndef SKEL_SEG_GROUPS_PER_CU
#define SKEL_SEG_GROUPS_PER_CU 4
#endif
constexpr int64_t kChunk = SKEL_SEG_CHUNK;        // elements per work item
constexpr int kGroupsPerCU = SKEL_SEG_GROUPS_PER_CU;  // persistent workgroups per CU
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kSlotReady = 1;

template <int OP>
using CF = Comb<float, OP>;

__device__ __forceinline__ void seg_range(const int64_t* off, int64_t s, int64_t n,
                                          int64_t* a, int64_t* b) {
    int64_t lo = off[s], hi = off[s + 1];
    lo = lo < 0 ? 0 : (lo > n ? n : lo);
    hi = hi < lo ? lo : (hi > n ? n : hi);
    *a = lo;
    *b = hi;
}

// item prefix: cpre[s] = sum over t < s of max(1, ceil(len_t / kChunk)),
// cpre[nseg] = number of items.  One workgroup of 1024 lanes.  Offsets that
// decrease or leave [0, n] raise error flag 4 and yield no items, so the
// item count never exceeds the slot array sized for n / kChunk + nseg items.
__global__ __launch_bounds__(1024) void seg_item_prefix(const int64_t* off, int64_t nseg,
                                                        int64_t n, int64_t* cpre, u64* err) {
    using C = Comb<int64_t, SKEL_SUM>;
    constexpr int NW = 1024 / kWave;
    __shared__ int64_t lds[NW];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const int w = threadIdx.x / kWave, l = lane();
    int64_t carry = 0;
    for (int64_t base = 0; base < nseg; base += 1024) {
        const int64_t s = base + threadIdx.x;
        int64_t cnt = 0;
        if (s < nseg) {
            const int64_t lo = off[s], hi = off[s + 1];
            if (lo < 0 || hi < lo || hi > n) bad = 1;
            int64_t a, b;
            seg_range(off, s, n, &a, &b);
            const int64_t len = b - a;
            cnt = len == 0 ? 1 : (len + kChunk - 1) / kChunk;
        }
        const int64_t incl = wave_inclusive_scan<C>(cnt);
        if (l == kWave - 1) lds[w] = incl;
        __syncthreads();
        int64_t wex = 0, total = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            if (k < w) wex += lds[k];
            total += lds[k];
        }
        if (s < nseg) cpre[s] = carry + wex + incl - cnt;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cpre[nseg] = bad ? 0 : carry;
        if (bad) atomicOr(err, 4ull);
    }
}

// largest s in [0, nseg) with cpre[s] <= k, by one wavefront: every round
// probes 64 evenly spaced entries at once (a 64-ary search: 3 rounds of
// parallel loads for 4096 segments instead of 12 dependent ones).  cpre is
// nondecreasing with cpre[0] = 0, so the probes that pass form a prefix.
__device__ __forceinline__ int64_t find_segment(const int64_t* cpre, int64_t nseg, int64_t k) {
    const int l = lane();
    int64_t lo = 0, hi = nseg - 1;  // the answer lies in [lo, hi], cpre[lo] <= k
    while (hi > lo) {
        const int64_t step = (hi - lo + kWave) / kWave;
        const int64_t p = lo + (int64_t)l * step;
        const bool ok = p <= hi && cpre[p] <= k;
        const u64 m = __ballot(ok);
        const int last = 63 - __clzll((long long)m);
        lo += (int64_t)last * step;
        const int64_t nhi = lo + step - 1;
        hi = nhi < hi ? nhi : hi;
    }
    return lo;
}

// op over x[a, b) by one workgroup: scalar head up to 16-byte alignment,
// 16-byte vectors, scalar tail
template <int OP>
__device__ __forceinline__ float range_reduce(const float* x, int64_t a, int64_t b,
                                              float* lds) {
    using C = CF<OP>;
    float acc = C::id();
    int64_t va = (a + 3) & ~int64_t(3);
    if (va > b) va = b;
    const int64_t vb = va + ((b - va) & ~int64_t(3));
    if (a + threadIdx.x < va) acc = C::op(acc, x[a + threadIdx.x]);
    const f32x4* xv = reinterpret_cast<const f32x4*>(x + va);
    const int64_t nv = (vb - va) >> 2;
    float acc2[4] = {C::id(), C::id(), C::id(), C::id()};
    int64_t i = threadIdx.x;
    for (; i + 3 * kBlock < nv; i += 4 * kBlock) {
        f32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(&xv[i + u * kBlock]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc2[u] = C::op(acc2[u], v[u].x);
            acc2[u] = C::op(acc2[u], v[u].y);
            acc2[u] = C::op(acc2[u], v[u].z);
            acc2[u] = C::op(acc2[u], v[u].w);
        }
    }
    for (; i < nv; i += kBlock) {
        const f32x4 v = xv[i];
        acc2[0] = C::op(C::op(C::op(C::op(acc2[0], v.x), v.y), v.z), v.w);
    }
    if (vb + threadIdx.x < b) acc = C::op(acc, x[vb + threadIdx.x]);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = C::op(acc, acc2[u]);
    return block_reduce<C>(acc, lds);  // valid in wavefront 0
}

template <int OP>
__global__ __launch_bounds__(kBlock) void seg_reduce_persistent(
    const float* x, int64_t n, const int64_t* off, int64_t nseg, const int64_t* cpre,
    u64* slots, u64* tickets, u64* sync, float* out) {
    using C = CF<OP>;
    __shared__ float lds[kBlock / kWave];
    __shared__ uint32_t s_epoch;
    __shared__ int64_t s_seg;
    __shared__ int s_last;
    if (threadIdx.x == 0) s_epoch = epoch_of_call(sync);
    __syncthreads();
    const uint32_t epoch = s_epoch;
    const int64_t items = cpre[nseg];  // 0 if the offsets were rejected
    for (int64_t k = blockIdx.x; k < items; k += gridDim.x) {
        if (threadIdx.x < kWave) {
            const int64_t sk = find_segment(cpre, nseg, k);
            if (threadIdx.x == 0) s_seg = sk;
        }
        __syncthreads();
        const int64_t s = s_seg;
        int64_t a, b;
        seg_range(off, s, n, &a, &b);
        const int64_t j = k - cpre[s];
        const int64_t ca = a + j * kChunk;
        const int64_t cb = ca + kChunk < b ? ca + kChunk : b;
        const float part = range_reduce<OP>(x, ca < b ? ca : b, cb, lds);
        if (threadIdx.x == 0) {
            tagged_put(slots + 2 * k, kSlotReady, epoch, part);
            const int64_t nitems = cpre[s + 1] - cpre[s];
            const u64 t = atomicAdd(&tickets[s], 1ull);
            s_last = t == (u64)nitems - 1;
        }
        __syncthreads();
        if (s_last) {
            // this workgroup finished the segment's last item: combine its
            // slots in item order
            const int64_t k0 = cpre[s], k1 = cpre[s + 1];
            float acc = C::id();
            for (int64_t q = k0 + threadIdx.x; q < k1; q += kBlock) {
                float v = C::id();
                uint32_t spins = 0;
                while (tagged_get(slots + 2 * q, epoch, v) != kSlotReady) {
                    if (++spins > kSpinLimit) {
                        atomicOr(sync + SYNC_ERROR, 2ull);
                        v = C::id();
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                acc = C::op(acc, v);
            }
            acc = block_reduce<C>(acc, lds);
            if (threadIdx.x == 0) {
                out[s] = acc;
                __hip_atomic_store(&tickets[s], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();  // lds and s_seg are reused by the next item
    }
    // the workgroup that finishes last advances the epoch for the next call
    if (threadIdx.x == 0) {
        const u64 d = atomicAdd(sync + SYNC_DONE, 1ull);
        if (d == (u64)gridDim.x - 1) {
            __hip_atomic_store(sync + SYNC_DONE, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            epoch_advance(sync);
        }
    }
}

// B0: one segment per launch pair (partials, then finish)
template <int OP>
__global__ __launch_bounds__(kBlock) void seg_one_partials(const float* x, int64_t a, int64_t b,
                                                           float* part) {
    __shared__ float lds[kBlock / kWave];
    using C = CF<OP>;
    // grid-stride over this segment with the workgroup's range share
    const int64_t len = b - a;
    const int64_t per = (len + gridDim.x - 1) / gridDim.x;
    const int64_t ca = a + (int64_t)blockIdx.x * per;
    int64_t cb = ca + per;
    if (cb > b) cb = b;
    const float v = range_reduce<OP>(x, ca < b ? ca : b, cb, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
    (void)sizeof(C);
}

template <int OP>
__global__ __launch_bounds__(1024) void seg_one_finish(const float* part, int g, float* out) {
    __shared__ float lds[1024 / kWave];
    using C = CF<OP>;
    float a = C::id();
    for (int i = threadIdx.x; i < g; i += 1024) a = C::op(a, part[i]);
    a = block_reduce<C>(a, lds);
    if (threadIdx.x == 0) *out = a;
}

template <int OP>
skel_status run_segments(int v, const float* x, int64_t n, const int64_t* off_dev,
                         const int64_t* off_host, int64_t nseg, float* out, LaunchCtx& lc) {
    hipStream_t st = lc.stream;
    if (v == B0_PER_SEGMENT) {
        const int gmax = lc.dev->cus * 4;
        void* part = nullptr;
        skel_status e = ws_scratch(lc, (size_t)gmax * sizeof(float), &part);
        if (e != SKEL_OK) return e;
        for (int64_t s = 0; s < nseg; ++s) {
            int64_t a = off_host[s], b = off_host[s + 1];
            a = a < 0 ? 0 : (a > n ? n : a);
            b = b < a ? a : (b > n ? n : b);
            int64_t g = (b - a + 2047) / 2048;
            if (g < 1) g = 1;
            if (g > gmax) g = gmax;
            seg_one_partials<OP><<<(unsigned)g, kBlock, 0, st>>>(x, a, b,
                                                                 static_cast<float*>(part));
            seg_one_finish<OP><<<1, 1024, 0, st>>>(static_cast<float*>(part), (int)g, out + s);
        }
        return launch_check("reduce_segments_per_segment");
    }
    // B1: item table, then the persistent pass
    const int64_t max_items = n / kChunk + nseg + 1;
    void* cpre = nullptr;
    skel_status e = ws_scratch(lc, (size_t)(nseg + 1) * sizeof(int64_t), &cpre);
    if (e != SKEL_OK) return e;
    void* status = nullptr;
    e = ws_status(lc, (size_t)max_items * 16, &status);
    if (e != SKEL_OK) return e;
    void* counters = nullptr;
    e = ws_counters(lc, (size_t)nseg * 8, &counters);
    if (e != SKEL_OK) return e;
    u64* slots = static_cast<u64*>(status);
    u64* tickets = static_cast<u64*>(counters);
    seg_item_prefix<<<1, 1024, 0, st>>>(off_dev, nseg, n, static_cast<int64_t*>(cpre),
                                        lc.ws->sync + SYNC_ERROR);
    if ((e = launch_check("reduce_segments_items")) != SKEL_OK) return e;
    const int g = lc.dev->cus * kGroupsPerCU;
    seg_reduce_persistent<OP><<<g, kBlock, 0, st>>>(x, n, off_dev, nseg,
                                                    static_cast<const int64_t*>(cpre), slots,
                                                    tickets, lc.ws->sync, out);
    return launch_check("reduce_segments_persistent");
}

}  // namespace

skel_status launch_reduce_segments(int v, int op, const float* x, int64_t n,
                                   const int64_t* off_dev, const int64_t* off_host,
                                   int64_t nseg, float* out, LaunchCtx& lc) {
    switch (op) {
    case SKEL_SUM: return run_segments<SKEL_SUM>(v, x, n, off_dev, off_host, nseg, out, lc);
    case SKEL_MIN: return run_segments<SKEL_MIN>(v, x, n, off_dev, off_host, nseg, out, lc);
    default: return run_segments<SKEL_MAX>(v, x, n, off_dev, off_host, nseg, out, lc);
    }
}

}  // namespace skel
