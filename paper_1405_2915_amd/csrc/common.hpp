// Shared host-side definitions of libskel: status/error reporting, element
// sizes, the copy/allocation backend interface and the global runtime state.
// No HIP headers here: the container protocol and the execution plan compile
// with any C++17 compiler, which is how they are tested without a GPU.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "skel.h"

namespace skel {

// Record `st` with a printf-style message as the calling thread's last error
// and return `st` (so call sites can `return fail(...)`).
skel_status fail(skel_status st, const char* fmt, ...)
    __attribute__((format(printf, 2, 3)));
void clear_error();

inline size_t dtype_size(skel_dtype t) {
    switch (t) {
    case SKEL_F32: return 4;
    case SKEL_BF16: return 2;
    case SKEL_I32: return 4;
    case SKEL_I64: return 8;
    }
    return 0;
}
inline bool dtype_valid(int t) { return t >= SKEL_F32 && t <= SKEL_I64; }

// every row of a matrix with `cols` columns starts 16-byte aligned in both an
// input of type a and an output of type b (the matrices themselves are)
inline bool rows_aligned(skel_dtype a, skel_dtype b, int64_t cols) {
    return (cols * (int64_t)dtype_size(a)) % 16 == 0 && (cols * (int64_t)dtype_size(b)) % 16 == 0;
}
const char* dtype_name(skel_dtype t);

// Everything the container protocol needs from the device runtime.  The HIP
// implementation lives in runtime.cpp; tests substitute a host-memory fake.
struct Backend {
    virtual ~Backend() = default;
    virtual skel_status host_alloc(void** p, size_t bytes) = 0;  // pinned
    virtual void host_free(void* p) = 0;
    virtual skel_status dev_alloc(const skel_allocator& a, void** p,
                                  size_t bytes, void* stream) = 0;
    virtual void dev_free(const skel_allocator& a, void* p, void* stream) = 0;
    // asynchronous copies on `stream`
    virtual skel_status copy_h2d(void* dst, const void* src, size_t bytes,
                                 void* stream) = 0;
    virtual skel_status copy_d2h(void* dst, const void* src, size_t bytes,
                                 void* stream) = 0;
    virtual skel_status event_create(void** ev) = 0;
    virtual void event_destroy(void* ev) = 0;
    virtual skel_status event_record(void* ev, void* stream) = 0;
    virtual skel_status stream_wait_event(void* stream, void* ev) = 0;
    virtual skel_status event_sync(void* ev) = 0;
    virtual skel_status stream_sync(void* stream) = 0;
};

struct Runtime {
    bool initialized = false;
    int device = -1;
    Backend* backend = nullptr;
    skel_allocator allocator{nullptr, nullptr, nullptr};
};

Runtime& rt();

}  // namespace skel
