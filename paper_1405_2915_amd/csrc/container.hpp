// Smart containers (Section IV of the paper): a host copy and a device copy
// of one operand, each with a validity bit, plus the bookkeeping that lets a
// skeleton call find a valid copy close to the device, copy lazily, and never
// read a stale one.  Dependences between asynchronous calls (Section V) are
// carried by a per-container event recorded after the last device access.
#pragma once

#include <vector>

#include "common.hpp"

// Sorted, disjoint element ranges [first, last) of one copy that hold current
// data (range-granular coherence: Section IV's partial copies).
struct skel_ranges {
    std::vector<std::pair<int64_t, int64_t>> r;
};

struct skel_container {
    skel_dtype dtype;
    int64_t rows, cols, n;
    size_t bytes;
    skel_allocator allocator;  // device-memory provider captured at creation

    void* host = nullptr;  // pinned host copy, allocated on first need
    void* dev = nullptr;   // device copy, allocated on first device acquire
    bool dev_external = false;  // dev is caller-owned (wrapped): never freed here
    // element ranges of each copy that are current; every acquire updates
    // them for the range it names (a whole-container acquire names [0, n))
    skel_ranges valid_host, valid_dev;

    // One event per stream that has accessed the device copy.  A device release
    // only marks the stream `pending`; the event is recorded when someone must
    // order after that work -- a device access on another stream, a host
    // access, or destroy.  Recording later on the same stream is conservative
    // (it also covers later work on that stream) and keeps event markers off
    // the single-stream fast path.
    struct StreamEvent {
        void* stream;
        void* event;
        bool recorded;  // the event holds a record
        bool pending;   // work enqueued on the stream since the last record
        uint64_t gen;   // number of records so far
        bool pending_write;  // that work writes the device copy
        uint64_t wgen;       // first record that follows the stream's last write (0: none)
        // (other stream, generation of its event this stream already waited on)
        std::vector<std::pair<void*, uint64_t>> seen;
    };
    std::vector<StreamEvent> events;
    void* last_stream = nullptr;  // stream of the most recent device access

    int host_readers = 0, dev_readers = 0;
    int writer = -1;  // place holding an outstanding WRITE/RW acquire, or -1

    skel_xfer_stats stats{};
};

namespace skel {

// interval-set operations on skel_ranges
void ranges_add(skel_ranges& s, int64_t lo, int64_t hi);
void ranges_sub(skel_ranges& s, int64_t lo, int64_t hi);
// the parts of [lo, hi) that `s` does not cover, in order
std::vector<std::pair<int64_t, int64_t>> ranges_missing(const skel_ranges& s, int64_t lo,
                                                        int64_t hi);

// Check, without side effects, that `access` to elements [lo, hi) at `place`
// would succeed (whole container: lo = 0, hi = n).
skel_status check_acquire(const skel_container* c, skel_place place, skel_access access,
                          int64_t lo, int64_t hi);
inline skel_status check_acquire(const skel_container* c, skel_place place,
                                 skel_access access) {
    return check_acquire(c, place, access, 0, c ? c->n : 0);
}

// The coherence protocol proper (see skel_container_acquire in skel.h); *ptr
// receives the address of element lo of the copy.
skel_status acquire(skel_container* c, skel_place place, skel_access access, int64_t lo,
                    int64_t hi, void* stream, void** ptr);
inline skel_status acquire(skel_container* c, skel_place place, skel_access access,
                           void* stream, void** ptr) {
    return acquire(c, place, access, 0, c ? c->n : 0, stream, ptr);
}
skel_status release(skel_container* c, skel_place place, void* stream);

}  // namespace skel
