// Host-memory stand-in for the device runtime, linked with the library's
// container protocol and execution plan into libskel_hosttest.so (g++ only, no
// HIP).  "Device" memory is malloc'd, copies are memcpy, streams are opaque
// tokens, and every operation is counted so tests can check exactly which
// transfers and synchronisations the protocol issued.  Failures of device
// allocation and of copies can be injected.
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "chain_table.hpp"
#include "common.hpp"

namespace {

struct Counts {
    unsigned long long host_allocs, host_frees, dev_allocs, dev_frees, h2d, d2h,
        event_creates, event_records, stream_waits, event_syncs, stream_syncs;
};
Counts g_counts;
int g_fail_dev_alloc = 0;
int g_fail_copy = 0;
// (stream, event) of every stream_wait_event, for ordering checks
std::vector<std::pair<void*, void*>> g_waits;

// Ordering model: every operation enqueued on a stream (copies, and the test's
// stand-ins for kernels) gets the stream's next position; a vector clock per
// stream holds, for every other stream, the last position known to complete
// before the stream's next operation.  An event record snapshots the
// recording stream's clock and position, a stream wait merges a snapshot into
// the waiting stream's clock, and an event (or stream) sync merges it into the
// host's.
using Clock = std::map<void*, long>;
struct Op {
    void* stream;
    long pos;
    Clock clock;  // the stream's clock when the operation was enqueued
};
std::map<void*, long> g_pos;
std::map<void*, Clock> g_clock;
std::map<void*, Clock> g_snap;  // event -> snapshot of its last record
Clock g_host;
std::vector<Op> g_ops;

void merge(Clock& into, const Clock& from) {
    for (const auto& kv : from)
        if (into[kv.first] < kv.second) into[kv.first] = kv.second;
}

// the host issues an operation after everything it has seen complete
int enqueue(void* s) {
    merge(g_clock[s], g_host);
    const long p = ++g_pos[s];
    g_ops.push_back({s, p, g_clock[s]});
    return (int)g_ops.size() - 1;
}

class FakeBackend final : public skel::Backend {
  public:
    skel_status host_alloc(void** p, size_t bytes) override {
        *p = std::malloc(bytes);
        if (!*p) return skel::fail(SKEL_E_NOMEM, "fake host alloc failed");
        g_counts.host_allocs++;
        return SKEL_OK;
    }
    void host_free(void* p) override {
        g_counts.host_frees++;
        std::free(p);
    }
    skel_status dev_alloc(const skel_allocator&, void** p, size_t bytes, void*) override {
        if (g_fail_dev_alloc > 0) {
            g_fail_dev_alloc--;
            return skel::fail(SKEL_E_NOMEM, "injected device allocation failure");
        }
        *p = std::aligned_alloc(256, (bytes + 255) & ~size_t(255));
        g_counts.dev_allocs++;
        return SKEL_OK;
    }
    void dev_free(const skel_allocator&, void* p, void*) override {
        g_counts.dev_frees++;
        std::free(p);
    }
    skel_status copy_h2d(void* dst, const void* src, size_t bytes, void* s) override {
        if (g_fail_copy > 0) {
            g_fail_copy--;
            return skel::fail(SKEL_E_HIP, "injected copy failure");
        }
        std::memcpy(dst, src, bytes);
        g_counts.h2d++;
        enqueue(s);
        return SKEL_OK;
    }
    skel_status copy_d2h(void* dst, const void* src, size_t bytes, void* s) override {
        if (g_fail_copy > 0) {
            g_fail_copy--;
            return skel::fail(SKEL_E_HIP, "injected copy failure");
        }
        std::memcpy(dst, src, bytes);
        g_counts.d2h++;
        enqueue(s);
        return SKEL_OK;
    }
    skel_status event_create(void** ev) override {
        *ev = new int(0);
        g_counts.event_creates++;
        return SKEL_OK;
    }
    void event_destroy(void* ev) override { delete static_cast<int*>(ev); }
    skel_status event_record(void* ev, void* s) override {
        ++*static_cast<int*>(ev);
        g_counts.event_records++;
        Clock snap = g_clock[s];
        snap[s] = g_pos[s];
        g_snap[ev] = snap;
        return SKEL_OK;
    }
    skel_status stream_wait_event(void* s, void* ev) override {
        g_counts.stream_waits++;
        g_waits.emplace_back(s, ev);
        merge(g_clock[s], g_snap[ev]);
        return SKEL_OK;
    }
    skel_status event_sync(void* ev) override {
        g_counts.event_syncs++;
        merge(g_host, g_snap[ev]);
        return SKEL_OK;
    }
    skel_status stream_sync(void* s) override {
        g_counts.stream_syncs++;
        merge(g_host, g_clock[s]);
        if (g_host[s] < g_pos[s]) g_host[s] = g_pos[s];
        return SKEL_OK;
    }
};

FakeBackend g_fake;

}  // namespace

extern "C" {

skel_status skel_hosttest_init(void) {
    skel::rt().backend = &g_fake;
    skel::rt().device = 0;
    skel::rt().initialized = true;
    std::memset(&g_counts, 0, sizeof g_counts);
    g_fail_dev_alloc = g_fail_copy = 0;
    g_waits.clear();
    g_pos.clear();
    g_clock.clear();
    g_snap.clear();
    g_host.clear();
    g_ops.clear();
    return SKEL_OK;
}

void skel_hosttest_fail_dev_alloc(int k) { g_fail_dev_alloc = k; }
void skel_hosttest_fail_copy(int k) { g_fail_copy = k; }

// host_allocs, host_frees, dev_allocs, dev_frees, h2d, d2h, event_creates,
// event_records, stream_waits, event_syncs, stream_syncs
void skel_hosttest_counts(unsigned long long* out11) {
    std::memcpy(out11, &g_counts, sizeof g_counts);
}

// The fused chain's weight of every element of one rows x cols field, as the
// kernels look it up (row class x column class of the host table), into
// out[rows * cols]; *pad_total receives the table's constant pad term.
void skel_hosttest_chain_weights(int64_t rows, int64_t cols, int64_t fields, const float* w2d,
                                 const float* wy, const float* wx, int ry, int rx, int edge,
                                 float pad, float* out, double* pad_total) {
    skel::ChainTable t;
    skel::chain_table(rows, cols, fields, w2d, wy, wx, ry, rx, edge, pad, &t);
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c)
            out[r * cols + c] =
                t.tab[skel::chain_row_class(t, r) * t.ncc + skel::chain_col_class(t, c)];
    *pad_total = t.pad_total;
}

int skel_hosttest_wait_count_on(void* stream) {
    int k = 0;
    for (auto& w : g_waits)
        if (w.first == stream) ++k;
    return k;
}

// Stand-in for a kernel enqueued on `stream`: returns its operation index.
int skel_hosttest_enqueue(void* stream) { return enqueue(stream); }

// Operations enqueued so far (copies included).
int skel_hosttest_op_count(void) { return (int)g_ops.size(); }

// 1 if operation i completes before operation j starts (same stream: stream
// order; otherwise j's stream had waited on an event recorded after i).
int skel_hosttest_op_before(int i, int j) {
    const Op& a = g_ops.at((size_t)i);
    const Op& b = g_ops.at((size_t)j);
    if (a.stream == b.stream) return a.pos < b.pos ? 1 : 0;
    const auto it = b.clock.find(a.stream);
    return it != b.clock.end() && it->second >= a.pos ? 1 : 0;
}

// 1 if operation i is known complete on the host (an event or stream sync).
int skel_hosttest_op_before_host(int i) {
    const Op& a = g_ops.at((size_t)i);
    const auto it = g_host.find(a.stream);
    return it != g_host.end() && it->second >= a.pos ? 1 : 0;
}

}  // extern "C"
