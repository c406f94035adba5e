// Device runtime of libskel: initialisation, the HIP implementation of the
// container backend, per-stream workspaces and error reporting.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "dispatch.hpp"
#include "launch.hpp"

namespace skel {

skel_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return SKEL_OK;
    return fail(SKEL_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

skel_status launch_check(const char* kernel) {
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return SKEL_OK;
    return fail(SKEL_E_HIP, "launch of %s: %s", kernel, hipGetErrorString(e));
}

int64_t resident_slots(const void* kernel, int block, LaunchCtx& lc) {
    // per kernel and block size, on the single device the library drives
    static std::mutex mu;
    static std::unordered_map<const void*, int> per_cu;
    std::lock_guard<std::mutex> g(mu);
    auto it = per_cu.find(kernel);
    if (it == per_cu.end()) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, 0) != hipSuccess) {
            (void)hipGetLastError();
            nb = 0;
        }
        it = per_cu.emplace(kernel, nb).first;
    }
    return (int64_t)it->second * lc.dev->cus;
}

namespace {

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

void* dev_malloc(const skel_allocator& a, size_t bytes, void* stream) {
    if (a.alloc) return a.alloc(bytes, stream, a.ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void dev_mfree(const skel_allocator& a, void* p, void* stream) {
    if (!p) return;
    if (a.free) a.free(p, stream, a.ctx);
    else (void)hipFree(p);
}

class HipBackend final : public Backend {
  public:
    skel_status host_alloc(void** p, size_t bytes) override {
        hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(SKEL_E_NOMEM, "hipHostMalloc(%zu): %s", bytes,
                        hipGetErrorString(e));
        }
        return SKEL_OK;
    }
    void host_free(void* p) override { (void)hipHostFree(p); }
    skel_status dev_alloc(const skel_allocator& a, void** p, size_t bytes,
                          void* stream) override {
        void* q = dev_malloc(a, bytes, stream);
        if (!q) return fail(SKEL_E_NOMEM, "device allocation of %zu bytes failed", bytes);
        if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {
            dev_mfree(a, q, stream);
            return fail(SKEL_E_NOMEM, "allocator returned memory not 256-byte aligned");
        }
        *p = q;
        return SKEL_OK;
    }
    void dev_free(const skel_allocator& a, void* p, void* stream) override {
        dev_mfree(a, p, stream);
    }
    skel_status copy_h2d(void* dst, const void* src, size_t bytes, void* s) override {
        return hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, S(s)),
                         "hipMemcpyAsync H2D");
    }
    skel_status copy_d2h(void* dst, const void* src, size_t bytes, void* s) override {
        return hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, S(s)),
                         "hipMemcpyAsync D2H");
    }
    skel_status event_create(void** ev) override {
        hipEvent_t e;
        skel_status st = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming),
                                   "hipEventCreate");
        if (st == SKEL_OK) *ev = e;
        return st;
    }
    void event_destroy(void* ev) override { (void)hipEventDestroy((hipEvent_t)ev); }
    skel_status event_record(void* ev, void* s) override {
        return hip_check(hipEventRecord((hipEvent_t)ev, S(s)), "hipEventRecord");
    }
    skel_status stream_wait_event(void* s, void* ev) override {
        return hip_check(hipStreamWaitEvent(S(s), (hipEvent_t)ev, 0), "hipStreamWaitEvent");
    }
    skel_status event_sync(void* ev) override {
        return hip_check(hipEventSynchronize((hipEvent_t)ev), "hipEventSynchronize");
    }
    skel_status stream_sync(void* s) override {
        return hip_check(hipStreamSynchronize(S(s)), "hipStreamSynchronize");
    }
};

HipBackend g_hip_backend;
DevInfo g_dev;
std::mutex g_ws_mu;
std::unordered_map<void*, Workspace*> g_ws;

// Superseded workspace buffers, kept until skel_finalize because a graph
// captured before they were replaced may still reference them.
std::unordered_map<Workspace*, std::vector<void*>> g_retired;

void free_workspace(Workspace* w) {
    const skel_allocator& a = rt().allocator;
    dev_mfree(a, w->scratch, w->stream);
    dev_mfree(a, w->sync, w->stream);
    dev_mfree(a, w->status, w->stream);
    dev_mfree(a, w->counters, w->stream);
    for (void* p : g_retired[w]) dev_mfree(a, p, w->stream);
    g_retired.erase(w);
    delete w;
}

}  // namespace

void retire(Workspace* w, void* p) {
    if (p) g_retired[w].push_back(p);
}

const DevInfo& device_info() { return g_dev; }

// The workspace of `stream`, created with a zeroed sync area on first use.
skel_status workspace_for(void* stream, Workspace** out) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find(stream);
    if (it != g_ws.end()) {
        *out = it->second;
        return SKEL_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(S(stream), &cs) != hipSuccess) {
        (void)hipGetLastError();
        cs = hipStreamCaptureStatusNone;
    }
    if (cs != hipStreamCaptureStatusNone)
        return fail(SKEL_E_STATE,
                    "first use of this stream is inside a graph capture; run a call on the "
                    "stream once before capturing (its workspace is cleared by a fill)");
    auto* w = new Workspace();
    w->stream = stream;
    size_t sb = SYNC_SLOTS * sizeof(unsigned long long);
    w->sync = static_cast<unsigned long long*>(dev_malloc(rt().allocator, sb, stream));
    if (!w->sync) {
        delete w;
        return fail(SKEL_E_NOMEM, "workspace allocation failed");
    }
    skel_status st = hip_check(hipMemsetAsync(w->sync, 0, sb, S(stream)), "hipMemsetAsync");
    if (st != SKEL_OK) {
        free_workspace(w);
        return st;
    }
    g_ws[stream] = w;
    *out = w;
    return SKEL_OK;
}

skel_status ws_scratch(LaunchCtx& lc, size_t bytes, void** p) {
    Workspace* w = lc.ws;
    if (w->scratch_bytes < bytes) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(lc.stream, &cs) != hipSuccess) {
            (void)hipGetLastError();
            cs = hipStreamCaptureStatusNone;
        }
        if (cs != hipStreamCaptureStatusNone)
            return fail(SKEL_E_STATE,
                        "the scratch workspace must grow to %zu bytes while the stream is "
                        "captured; run the same call once before capture", bytes);
        size_t want = bytes < (size_t(1) << 20) ? (size_t(1) << 20) : bytes;
        want = (want + 4095) & ~size_t(4095);
        retire(w, w->scratch);  // a graph captured earlier may still use it
        w->scratch = nullptr;
        w->scratch_bytes = 0;
        void* q = dev_malloc(rt().allocator, want, w->stream);
        if (!q) return fail(SKEL_E_NOMEM, "scratch allocation of %zu bytes failed", want);
        w->scratch = q;
        w->scratch_bytes = want;
    }
    *p = w->scratch;
    return SKEL_OK;
}

skel_status ws_counters(LaunchCtx& lc, size_t bytes, void** p) {
    Workspace* w = lc.ws;
    if (w->counters_bytes < bytes) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(lc.stream, &cs) != hipSuccess) {
            (void)hipGetLastError();
            cs = hipStreamCaptureStatusNone;
        }
        if (cs != hipStreamCaptureStatusNone)
            return fail(SKEL_E_STATE,
                        "the counter workspace must grow while the stream is captured; run "
                        "the same call once before capture");
        size_t want = bytes < 4096 ? 4096 : ((bytes + 4095) & ~size_t(4095));
        void* q = dev_malloc(rt().allocator, want, w->stream);
        if (!q) return fail(SKEL_E_NOMEM, "counter allocation of %zu bytes failed", want);
        skel_status st = hip_check(hipMemsetAsync(q, 0, want, lc.stream), "hipMemsetAsync");
        if (st != SKEL_OK) {
            dev_mfree(rt().allocator, q, w->stream);
            return st;
        }
        retire(w, w->counters);
        w->counters = q;
        w->counters_bytes = want;
    }
    *p = w->counters;
    return SKEL_OK;
}

skel_status ws_status(LaunchCtx& lc, size_t bytes, void** p) {
    Workspace* w = lc.ws;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(lc.stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        cs = hipStreamCaptureStatusNone;
    }
    const bool capturing = cs != hipStreamCaptureStatusNone;
    // Growing the array, or clearing it before the device epoch can wrap onto
    // words of an earlier cycle, resets the epoch; both enqueue fills, which
    // must not happen inside a captured graph.
    const bool grow = w->status_bytes < bytes;
    const bool wrap = w->epoch_calls >= (uint64_t)kEpochMax - 1;
    if ((grow || wrap) && capturing)
        return fail(SKEL_E_STATE,
                    "the descriptor workspace must be %s while the stream is captured; "
                    "run the same call once before capture",
                    grow ? "enlarged" : "reset");
    if (grow) {
        size_t want = bytes < (size_t(1) << 16) ? (size_t(1) << 16) : bytes;
        want = (want + 4095) & ~size_t(4095);
        retire(w, w->status);  // a graph captured earlier may still use it
        w->status = nullptr;
        w->status_bytes = 0;
        void* q = dev_malloc(rt().allocator, want, w->stream);
        if (!q) return fail(SKEL_E_NOMEM, "status allocation of %zu bytes failed", want);
        w->status = q;
        w->status_bytes = want;
    }
    if (grow || wrap) {
        skel_status st = hip_check(hipMemsetAsync(w->status, 0, w->status_bytes, lc.stream),
                                   "hipMemsetAsync");
        if (st == SKEL_OK)
            st = hip_check(hipMemsetAsync(w->sync + SYNC_EPOCH, 0, 8, lc.stream),
                           "hipMemsetAsync");
        if (st != SKEL_OK) return st;
        w->epoch_calls = 0;
    }
    w->epoch_calls += 1;
    *p = w->status;
    return SKEL_OK;
}

skel_status ws_status_ready(LaunchCtx& lc, size_t bytes, int64_t calls) {
    if (calls <= 0) return SKEL_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(lc.stream, &cs) != hipSuccess) {
        (void)hipGetLastError();
        cs = hipStreamCaptureStatusNone;
    }
    if (cs == hipStreamCaptureStatusNone) return SKEL_OK;
    const Workspace* w = lc.ws;
    if (w->status_bytes < bytes || w->epoch_calls + (uint64_t)calls >= (uint64_t)kEpochMax - 1)
        return fail(SKEL_E_STATE,
                    "the descriptor workspace would have to be enlarged or reset while the "
                    "stream is captured; run the same call once before capture");
    return SKEL_OK;
}

}  // namespace skel

using namespace skel;

extern "C" {

skel_status skel_init(int device, const skel_allocator* alloc) {
    clear_error();
    int count = 0;
    skel_status st = hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
    if (st != SKEL_OK) return st;
    if (device < 0 || device >= count)
        return fail(SKEL_E_INVAL, "device %d out of range (%d devices)", device, count);
    if (rt().initialized && rt().device != device)
        return fail(SKEL_E_INVAL, "already initialised on device %d", rt().device);
    st = hip_check(hipSetDevice(device), "hipSetDevice");
    if (st != SKEL_OK) return st;
    hipDeviceProp_t prop;
    st = hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (st != SKEL_OK) return st;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SKEL_E_UNSUPPORTED, "device %d is %s; this library is built for gfx950",
                    device, prop.gcnArchName);
    if (prop.warpSize != 64)
        return fail(SKEL_E_UNSUPPORTED, "wavefront size %d, expected 64", prop.warpSize);
    g_dev.cus = prop.multiProcessorCount;
    g_dev.lds_bytes = (int)prop.sharedMemPerBlock;
    g_dev.wave = prop.warpSize;
    g_dev.max_threads = prop.maxThreadsPerBlock;
    st = scan_noalloc_setup(device);
    if (st != SKEL_OK) return st;
    rt().backend = &g_hip_backend;
    rt().device = device;
    rt().allocator = alloc ? *alloc : skel_allocator{nullptr, nullptr, nullptr};
    rt().initialized = true;
    const char* table = std::getenv("SKEL_PLAN_FILE");
    if (table && *table) {
        st = load_plan_table(table);
        if (st != SKEL_OK) return st;
    }
    return SKEL_OK;
}

skel_status skel_finalize(void) {
    if (!rt().initialized) return SKEL_OK;
    skel_status st = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    for (auto& kv : g_ws) free_workspace(kv.second);
    g_ws.clear();
    return st;
}

skel_status skel_sync(void* stream) {
    if (!rt().initialized) return fail(SKEL_E_NOINIT, "skel_init has not been called");
    skel_status st = hip_check(hipStreamSynchronize((hipStream_t)stream),
                               "hipStreamSynchronize");
    if (st != SKEL_OK) return st;
    Workspace* w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        auto it = g_ws.find(stream);
        if (it != g_ws.end()) w = it->second;
    }
    if (!w) return SKEL_OK;
    unsigned long long flag = 0;
    st = hip_check(hipMemcpy(&flag, w->sync + SYNC_ERROR, sizeof flag,
                             hipMemcpyDeviceToHost),
                   "hipMemcpy");
    if (st != SKEL_OK) return st;
    if (flag) {
        (void)hipMemset(w->sync + SYNC_ERROR, 0, sizeof flag);
        return fail(SKEL_E_TIMEOUT,
                    "a bounded inter-workgroup wait expired (flag 0x%llx: 1 = scan "
                    "look-back, 2 = reduce partials); results of the "
                    "calls since the last skel_sync on this stream are invalid",
                    flag);
    }
    return SKEL_OK;
}

}  // extern "C"
