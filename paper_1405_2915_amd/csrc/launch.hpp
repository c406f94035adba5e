// Host-side launch interface between the skeleton entry points and the HIP
// kernels.  Every launcher takes device pointers that the container protocol
// has made valid, plain sizes, and a LaunchCtx naming the stream, the device
// limits and the per-stream workspace.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace skel {

struct DevInfo {
    int cus = 256;            // compute units
    int lds_bytes = 65536;    // LDS per workgroup
    int wave = 64;            // wavefront width
    int max_threads = 1024;   // per workgroup
};

// Per-stream device scratch.  `sync` is a small persistent area that is zero
// when allocated and that kernels keep consistent between calls: each ticket
// or counter is reset by the workgroup that takes its last value, and the
// descriptor epoch is advanced on the device by the last workgroup of each
// call that uses `status` (so calls captured in a graph replay correctly).
// `status` holds self-validating descriptors tagged with that epoch, so it
// never needs clearing between calls.
struct Workspace {
    void* stream = nullptr;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    unsigned long long* sync = nullptr;
    void* status = nullptr;
    size_t status_bytes = 0;
    uint64_t epoch_calls = 0;  // calls that advanced the device epoch since its last reset
    void* counters = nullptr;  // zero when allocated; every user resets what it counts
    size_t counters_bytes = 0;
};

// slots of the sync area, as indices of 64-bit words; each slot has its own
// 128-byte cache line, because every workgroup of a call hits some of them
// atomically and sharing a line serialises those accesses
enum SyncSlot {
    SYNC_TICKET = 0,         // reduce / mapreduce "last workgroup" ticket
    SYNC_TILE_COUNTER = 16,  // scan dynamic tile id counter
    SYNC_ERROR = 32,         // nonzero: a kernel's bounded wait expired
    SYNC_EPOCH = 48,         // descriptor epoch - 1 (0 when allocated)
    SYNC_DONE = 64,          // finished-workgroup counter
    SYNC_SUB_TICKET = 128,   // kSubTickets first-level reduce tickets, 16 words apart
    SYNC_SLOTS = 128 + 16 * 16
};

// first-level tickets of the single-pass reduce: workgroup b draws from
// ticket b % kSubTickets, and the last drawer of each draws from the
// top-level ticket, so no counter takes more than g / kSubTickets atomics
constexpr int kSubTickets = 16;

// descriptor epochs run 1 .. kEpochMax (30 bits, never 0)
constexpr uint32_t kEpochMax = (1u << 30) - 1;

struct LaunchCtx {
    hipStream_t stream;
    const DevInfo* dev;
    Workspace* ws;
};

// runtime.cpp
const DevInfo& device_info();
skel_status workspace_for(void* stream, Workspace** out);
skel_status ws_scratch(LaunchCtx& lc, size_t bytes, void** p);
void retire(Workspace* w, void* p);  // free at skel_finalize, not before
// zero-initialised counter array of at least `bytes` (kernels leave it zero)
skel_status ws_counters(LaunchCtx& lc, size_t bytes, void** p);
// descriptor array of at least `bytes` for one call that advances the device
// epoch; fails with SKEL_E_STATE if the array would have to grow (or be
// cleared) while the stream is being captured into a graph
skel_status ws_status(LaunchCtx& lc, size_t bytes, void** p);
// SKEL_E_STATE, before anything is enqueued, if `calls` calls that each take a
// descriptor array (of `bytes`; 0: the size is checked by the first call
// itself) would have to enlarge or reset it while the stream is captured
// (outside a capture they may: nothing to check)
skel_status ws_status_ready(LaunchCtx& lc, size_t bytes, int64_t calls);
skel_status hip_check(hipError_t e, const char* what);
skel_status launch_check(const char* kernel);
// workgroups of `block` threads of `kernel` that the device holds at once
// (0 if the kernel does not fit); queried once per kernel
int64_t resident_slots(const void* kernel, int block, LaunchCtx& lc);

// kernels (k_*.hip); all return SKEL_OK or SKEL_E_HIP
skel_status launch_map(int variant, int op, float p0, float p1, const float* x,
                       const float* y, float* out, int64_t n, LaunchCtx& lc);
skel_status launch_reduce(int variant, int op, skel_dtype din, skel_dtype dout,
                          const void* x, int64_t n, void* out, LaunchCtx& lc);
skel_status launch_mapreduce(int variant, int map_op, float p0, float p1,
                             skel_dtype din, const void* x, const void* y,
                             int64_t n, int op, float* out, LaunchCtx& lc);
skel_status launch_overlap1d(int variant, const float* x, float* out, int64_t n,
                             const float* w, int r, int edge, float pad,
                             LaunchCtx& lc);
// `fields` images of rows x cols stored back to back, each mapped on its own
// (its own borders); one launch covers up to kMaxFieldsPerLaunch of them
constexpr int64_t kMaxFieldsPerLaunch = 65535;
skel_status launch_overlap2d(int variant, const float* x, float* out,
                             int64_t rows, int64_t cols, int64_t fields, const float* w2d,
                             const float* wy, const float* wx, int ry, int rx,
                             int edge, float pad, LaunchCtx& lc);
skel_status launch_reduce_segments(int variant, int op, const float* x, int64_t n,
                                   const int64_t* off_dev, const int64_t* off_host,
                                   int64_t nseg, float* out, LaunchCtx& lc);
skel_status launch_scan(int variant, int kind, int op, skel_dtype din,
                        skel_dtype dout, const void* x, void* out, int64_t n,
                        LaunchCtx& lc);
// every row of a rows x cols matrix scanned on its own, one wavefront per row;
// vec: row starts are 16-byte aligned for both types (16-byte accesses)
skel_status launch_scan_rows(int kind, int op, skel_dtype din, skel_dtype dout, const void* x,
                             void* y, int64_t rows, int64_t cols, bool vec, LaunchCtx& lc);
// the call chain Map -> MapOverlap 2D -> Reduce SUM over `fields` images of
// rows x cols (k_chain.hip): out[0] = the sum; the backward pass writes
// dx = d(sum)/dx * g1[0] and, if dparams is not NULL, the parameter gradients
skel_status launch_chain(int variant, int map_op, float p0, float p1, const float* x,
                         int64_t rows, int64_t cols, int64_t fields, const float* w2d,
                         const float* wy, const float* wx, int ry, int rx, int edge, float pad,
                         float* out, LaunchCtx& lc);
skel_status launch_chain_backward(int variant, int map_op, float p0, float p1, const float* x,
                                  int64_t rows, int64_t cols, int64_t fields, const float* w2d,
                                  const float* wy, const float* wx, int ry, int rx, int edge,
                                  const float* g1, float* dx, float* dparams, LaunchCtx& lc);
// device address of the allocation-free scan's array on `device` (k_scan.hip),
// looked up once per device with that device current (skel_init)
skel_status scan_noalloc_setup(int device);
// adjoints (k_grad.hip); g_broadcast: g holds one value for every element
skel_status launch_map_backward(int op, float p0, float p1, const float* x, const float* y,
                                const float* g, bool g_broadcast, float* dx, float* dy,
                                int64_t n, float* dparams, LaunchCtx& lc);
skel_status launch_overlap1d_adjoint(int variant, const float* g, float* dx, int64_t n,
                                     const float* w, int r, int edge, LaunchCtx& lc);
skel_status launch_overlap2d_adjoint(int variant, const float* g, float* dx, int64_t rows,
                                     int64_t cols, int64_t fields, const float* w2d,
                                     const float* wy, const float* wx, int ry, int rx,
                                     int edge, LaunchCtx& lc);

}  // namespace skel
