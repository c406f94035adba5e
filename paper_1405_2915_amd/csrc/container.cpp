// Smart-container coherence protocol (Section IV) and its C ABI.
//
// Each container has a host copy and a device copy with one validity bit
// each.  Reading a copy that is stale triggers exactly one transfer from the
// other (the only other holder on a one-GPU system); writing a copy makes the
// other stale.  Nothing is ever copied eagerly: results stay on the device
// until the host asks for them, which is what removes the redundant transfers
// of call sequences (lazy memory copying).
#include "container.hpp"

#include <cstring>
#include <new>

namespace skel {

namespace {

bool has_read(skel_access a) { return (a & SKEL_READ) != 0; }
bool has_write(skel_access a) { return (a & SKEL_WRITE) != 0; }

skel_container::StreamEvent* event_for(skel_container* c, void* stream,
                                       skel_status* st) {
    for (auto& e : c->events)
        if (e.stream == stream) return &e;
    void* ev = nullptr;
    *st = rt().backend->event_create(&ev);
    if (*st != SKEL_OK) return nullptr;
    c->events.push_back({stream, ev, false, false, 0, false, 0, {}});
    return &c->events.back();
}

// Record the stream's event now if work was enqueued since its last record.
skel_status flush_pending(skel_container::StreamEvent& e) {
    if (!e.pending) return SKEL_OK;
    skel_status st = rt().backend->event_record(e.event, e.stream);
    if (st != SKEL_OK) return st;
    e.recorded = true;
    e.pending = false;
    e.gen += 1;
    if (e.pending_write) {
        e.wgen = e.gen;
        e.pending_write = false;
    }
    return SKEL_OK;
}

// Make `stream` wait for the device accesses of other streams that conflict
// with an access of kind `writing` (Section V: the dependences of a call are
// found from its operands).  A writer waits for every other stream's last
// access (reads and writes); a reader only for other streams' writes, which
// include the copies of stale ranges that a reader's acquire enqueued: reads
// on different streams run concurrently.  Events whose generation this stream
// already waited on are skipped.
skel_status order_after_other_streams(skel_container* c, void* stream, bool writing) {
    skel_status st = SKEL_OK;
    if (!event_for(c, stream, &st)) return st;  // entry for `stream` exists now
    size_t me = 0;
    while (c->events[me].stream != stream) ++me;
    for (size_t k = 0; k < c->events.size(); ++k) {
        if (k == me) continue;
        auto& seen = c->events[me].seen;
        auto it = seen.begin();
        while (it != seen.end() && it->first != c->events[k].stream) ++it;
        const uint64_t waited = it != seen.end() ? it->second : 0;
        if (!writing && !c->events[k].pending_write &&
            (c->events[k].wgen == 0 || waited >= c->events[k].wgen))
            continue;  // no write of stream k this one is not yet ordered after
        st = flush_pending(c->events[k]);
        if (st != SKEL_OK) return st;
        const auto& e = c->events[k];
        if (!e.recorded) continue;
        if (waited == e.gen) continue;
        st = rt().backend->stream_wait_event(stream, e.event);
        if (st != SKEL_OK) return st;
        if (it != seen.end()) it->second = e.gen;
        else seen.emplace_back(e.stream, e.gen);
    }
    return SKEL_OK;
}

// Block until every device access of the container has finished.
skel_status wait_device_idle(skel_container* c) {
    for (auto& e : c->events) {
        skel_status st = flush_pending(e);
        if (st != SKEL_OK) return st;
        if (!e.recorded) continue;
        st = rt().backend->event_sync(e.event);
        if (st != SKEL_OK) return st;
    }
    return SKEL_OK;
}

skel_status ensure_host(skel_container* c) {
    if (c->host || c->bytes == 0) return SKEL_OK;
    return rt().backend->host_alloc(&c->host, c->bytes);
}

}  // namespace

void ranges_add(skel_ranges& s, int64_t lo, int64_t hi) {
    if (lo >= hi) return;
    std::vector<std::pair<int64_t, int64_t>> out;
    out.reserve(s.r.size() + 1);
    bool placed = false;
    for (const auto& q : s.r) {
        if (q.second < lo) {
            out.push_back(q);  // entirely before (not touching)
        } else if (q.first > hi) {
            if (!placed) out.emplace_back(lo, hi), placed = true;
            out.push_back(q);  // entirely after
        } else {  // overlaps or touches: merge into [lo, hi)
            lo = q.first < lo ? q.first : lo;
            hi = q.second > hi ? q.second : hi;
        }
    }
    if (!placed) out.emplace_back(lo, hi);
    s.r.swap(out);
}

void ranges_sub(skel_ranges& s, int64_t lo, int64_t hi) {
    if (lo >= hi) return;
    std::vector<std::pair<int64_t, int64_t>> out;
    out.reserve(s.r.size() + 1);
    for (const auto& q : s.r) {
        if (q.second <= lo || q.first >= hi) {
            out.push_back(q);
            continue;
        }
        if (q.first < lo) out.emplace_back(q.first, lo);
        if (q.second > hi) out.emplace_back(hi, q.second);
    }
    s.r.swap(out);
}

std::vector<std::pair<int64_t, int64_t>> ranges_missing(const skel_ranges& s, int64_t lo,
                                                        int64_t hi) {
    std::vector<std::pair<int64_t, int64_t>> gaps;
    int64_t at = lo;
    for (const auto& q : s.r) {
        if (q.second <= at) continue;
        if (q.first >= hi) break;
        if (q.first > at) gaps.emplace_back(at, q.first);
        at = q.second;
        if (at >= hi) break;
    }
    if (at < hi) gaps.emplace_back(at, hi);
    return gaps;
}

skel_status check_acquire(const skel_container* c, skel_place place, skel_access access,
                          int64_t lo, int64_t hi) {
    if (!c) return fail(SKEL_E_INVAL, "null container");
    if (place != SKEL_HOST && place != SKEL_DEVICE)
        return fail(SKEL_E_INVAL, "bad place %d", (int)place);
    if (access != SKEL_READ && access != SKEL_WRITE && access != SKEL_RW)
        return fail(SKEL_E_INVAL, "bad access mode %d", (int)access);
    if (lo < 0 || hi < lo || hi > c->n)
        return fail(SKEL_E_INVAL, "element range [%lld, %lld) outside [0, %lld)", (long long)lo,
                    (long long)hi, (long long)c->n);
    if (c->writer != -1)
        return fail(SKEL_E_STATE, "container has an outstanding %s write access",
                    c->writer == SKEL_HOST ? "host" : "device");
    if (has_write(access) && (c->host_readers + c->dev_readers) > 0)
        return fail(SKEL_E_STATE,
                    "write access requested while %d read access(es) are outstanding",
                    c->host_readers + c->dev_readers);
    if (has_read(access)) {
        // every element read must be current in one of the copies
        for (const auto& m : ranges_missing(c->valid_host, lo, hi))
            if (!ranges_missing(c->valid_dev, m.first, m.second).empty())
                return fail(SKEL_E_STATE, "read of an uninitialised container (elements "
                            "[%lld, %lld) were never written)", (long long)m.first,
                            (long long)m.second);
    }
    return SKEL_OK;
}

skel_status acquire(skel_container* c, skel_place place, skel_access access, int64_t lo,
                    int64_t hi, void* stream, void** ptr) {
    skel_status st = check_acquire(c, place, access, lo, hi);
    if (st != SKEL_OK) return st;
    Backend* be = rt().backend;
    const size_t es = dtype_size(c->dtype);

    if (place == SKEL_DEVICE) {
        if (c->bytes > 0) {
            if (!c->dev) {
                st = be->dev_alloc(c->allocator, &c->dev, c->bytes, stream);
                if (st != SKEL_OK) return st;
            }
            // order after device work on other streams (Section V dependences)
            const auto missing = has_read(access) ? ranges_missing(c->valid_dev, lo, hi)
                                                  : std::vector<std::pair<int64_t, int64_t>>{};
            st = order_after_other_streams(c, stream, has_write(access) || !missing.empty());
            if (st != SKEL_OK) return st;
            if (!missing.empty()) {
                // this stream now writes the device copy: later readers on
                // other streams order after it
                skel_container::StreamEvent* me = event_for(c, stream, &st);
                if (!me) return st;
                me->pending = true;
                me->pending_write = true;
            }
            if (has_read(access)) {
                // copy only the stale parts of the range (partial copies)
                for (const auto& m : missing) {
                    const size_t off = (size_t)m.first * es, len = (size_t)(m.second - m.first) * es;
                    st = be->copy_h2d(static_cast<char*>(c->dev) + off,
                                      static_cast<const char*>(c->host) + off, len, stream);
                    if (st != SKEL_OK) return st;
                    c->stats.h2d += 1;
                    c->stats.h2d_bytes += len;
                    ranges_add(c->valid_dev, m.first, m.second);
                }
            }
        }
        ranges_add(c->valid_dev, lo, hi);
        if (has_write(access)) ranges_sub(c->valid_host, lo, hi);
        c->last_stream = stream;
        if (has_write(access)) c->writer = SKEL_DEVICE;
        else c->dev_readers += 1;
        *ptr = c->dev ? static_cast<char*>(c->dev) + (size_t)lo * es : nullptr;
    } else {
        st = wait_device_idle(c);
        if (st != SKEL_OK) return st;
        if (c->bytes > 0) {
            st = ensure_host(c);
            if (st != SKEL_OK) return st;
            if (has_read(access)) {
                const auto gaps = ranges_missing(c->valid_host, lo, hi);
                for (const auto& m : gaps) {
                    const size_t off = (size_t)m.first * es, len = (size_t)(m.second - m.first) * es;
                    st = be->copy_d2h(static_cast<char*>(c->host) + off,
                                      static_cast<const char*>(c->dev) + off, len,
                                      c->last_stream);
                    if (st != SKEL_OK) return st;
                    c->stats.d2h += 1;
                    c->stats.d2h_bytes += len;
                }
                if (!gaps.empty()) {
                    skel_container::StreamEvent* e = event_for(c, c->last_stream, &st);
                    if (!e) return st;
                    st = be->event_record(e->event, c->last_stream);
                    if (st == SKEL_OK) st = be->event_sync(e->event);
                    if (st != SKEL_OK) return st;
                    e->recorded = true;
                    e->pending = false;
                    e->gen += 1;
                    for (const auto& m : gaps) ranges_add(c->valid_host, m.first, m.second);
                }
            }
        }
        ranges_add(c->valid_host, lo, hi);
        if (has_write(access)) ranges_sub(c->valid_dev, lo, hi);
        if (has_write(access)) c->writer = SKEL_HOST;
        else c->host_readers += 1;
        *ptr = c->host ? static_cast<char*>(c->host) + (size_t)lo * es : nullptr;
    }
    c->stats.acquires += 1;
    return SKEL_OK;
}

skel_status release(skel_container* c, skel_place place, void* stream) {
    if (!c) return fail(SKEL_E_INVAL, "null container");
    if (place != SKEL_HOST && place != SKEL_DEVICE)
        return fail(SKEL_E_INVAL, "bad place %d", (int)place);
    if (place == SKEL_DEVICE) {
        if (c->writer != SKEL_DEVICE && c->dev_readers == 0)
            return fail(SKEL_E_STATE, "device release without a device acquire");
        if (c->bytes > 0) {
            skel_status st;
            skel_container::StreamEvent* e = event_for(c, stream, &st);
            if (!e) return st;
            e->pending = true;  // recorded lazily, when someone must order after it
            if (c->writer == SKEL_DEVICE) e->pending_write = true;
            c->last_stream = stream;
        }
        if (c->writer == SKEL_DEVICE) c->writer = -1;
        else c->dev_readers -= 1;
    } else {
        if (c->writer != SKEL_HOST && c->host_readers == 0)
            return fail(SKEL_E_STATE, "host release without a host acquire");
        if (c->writer == SKEL_HOST) c->writer = -1;
        else c->host_readers -= 1;
    }
    return SKEL_OK;
}

}  // namespace skel

using namespace skel;

extern "C" {

skel_status skel_container_create(skel_dtype dtype, int64_t rows, int64_t cols,
                                  const void* host_src, skel_container** out) {
    if (!rt().initialized) return fail(SKEL_E_NOINIT, "skel_init has not been called");
    if (!out) return fail(SKEL_E_INVAL, "null output pointer");
    if (!dtype_valid(dtype)) return fail(SKEL_E_DTYPE, "unknown dtype %d", (int)dtype);
    if (rows < 1 || cols < 0)
        return fail(SKEL_E_SHAPE, "bad shape %lld x %lld", (long long)rows,
                    (long long)cols);
    const int64_t lim = INT64_C(1) << 31;
    if (rows > lim || cols > lim || (cols > 0 && rows > (INT64_C(1) << 40) / cols))
        return fail(SKEL_E_SHAPE, "shape %lld x %lld too large", (long long)rows,
                    (long long)cols);
    auto* c = new (std::nothrow) skel_container();
    if (!c) return fail(SKEL_E_NOMEM, "out of host memory");
    c->dtype = dtype;
    c->rows = rows;
    c->cols = cols;
    c->n = rows * cols;
    c->bytes = (size_t)c->n * dtype_size(dtype);
    c->allocator = rt().allocator;
    if (c->bytes == 0) {
        // nothing to hold: every (empty) range is current
    } else if (host_src) {
        skel_status st = rt().backend->host_alloc(&c->host, c->bytes);
        if (st != SKEL_OK) {
            delete c;
            return st;
        }
        std::memcpy(c->host, host_src, c->bytes);
        ranges_add(c->valid_host, 0, c->n);
    }
    *out = c;
    return SKEL_OK;
}

skel_status skel_container_wrap_device(skel_dtype dtype, int64_t rows, int64_t cols,
                                       void* dev_ptr, void* stream, skel_container** out) {
    if (!rt().initialized) return fail(SKEL_E_NOINIT, "skel_init has not been called");
    if (!out) return fail(SKEL_E_INVAL, "null output pointer");
    if (!dtype_valid(dtype)) return fail(SKEL_E_DTYPE, "unknown dtype %d", (int)dtype);
    if (rows < 1 || cols < 0)
        return fail(SKEL_E_SHAPE, "bad shape %lld x %lld", (long long)rows, (long long)cols);
    const int64_t lim = INT64_C(1) << 31;
    if (rows > lim || cols > lim || (cols > 0 && rows > (INT64_C(1) << 40) / cols))
        return fail(SKEL_E_SHAPE, "shape %lld x %lld too large", (long long)rows,
                    (long long)cols);
    const size_t bytes = (size_t)(rows * cols) * dtype_size(dtype);
    if (bytes > 0 && !dev_ptr) return fail(SKEL_E_INVAL, "null device pointer");
    if ((reinterpret_cast<uintptr_t>(dev_ptr) & 15) != 0)
        return fail(SKEL_E_INVAL, "wrapped device memory must be 16-byte aligned");
    auto* c = new (std::nothrow) skel_container();
    if (!c) return fail(SKEL_E_NOMEM, "out of host memory");
    c->dtype = dtype;
    c->rows = rows;
    c->cols = cols;
    c->n = rows * cols;
    c->bytes = bytes;
    c->allocator = rt().allocator;
    if (bytes > 0) {
        c->dev = dev_ptr;
        c->dev_external = true;
        ranges_add(c->valid_dev, 0, c->n);
        // the contents were produced in `stream` order: treat that as the
        // container's last device access (its event is recorded when another
        // stream or the host first needs it)
        skel_status st = SKEL_OK;
        auto* e = event_for(c, stream, &st);
        if (!e) {
            delete c;
            return st;
        }
        e->pending = true;
        e->pending_write = true;
        c->last_stream = stream;
    }
    *out = c;
    return SKEL_OK;
}

skel_status skel_container_destroy(skel_container* c) {
    if (!c) return fail(SKEL_E_INVAL, "null container");
    if (c->writer != -1 || c->host_readers || c->dev_readers)
        return fail(SKEL_E_STATE, "destroy with an outstanding acquire");
    Backend* be = rt().backend;
    // a wrapped container without a host copy frees nothing that its device
    // work still uses, so destroying it does not wait
    if (!(c->dev_external && !c->host)) {
        skel_status st = wait_device_idle(c);
        if (st != SKEL_OK) return st;
    }
    if (c->dev && !c->dev_external) be->dev_free(c->allocator, c->dev, c->last_stream);
    if (c->host) be->host_free(c->host);
    for (auto& e : c->events) be->event_destroy(e.event);
    delete c;
    return SKEL_OK;
}

skel_status skel_container_acquire(skel_container* c, skel_place place,
                                   skel_access access, void* stream,
                                   void** ptr_out) {
    if (!rt().initialized) return fail(SKEL_E_NOINIT, "skel_init has not been called");
    if (!ptr_out) return fail(SKEL_E_INVAL, "null ptr_out");
    return acquire(c, place, access, stream, ptr_out);
}

skel_status skel_container_acquire_range(skel_container* c, skel_place place,
                                         skel_access access, int64_t first, int64_t count,
                                         void* stream, void** ptr_out) {
    if (!rt().initialized) return fail(SKEL_E_NOINIT, "skel_init has not been called");
    if (!ptr_out) return fail(SKEL_E_INVAL, "null ptr_out");
    if (count < 0 || first < 0) return fail(SKEL_E_INVAL, "negative range");
    return acquire(c, place, access, first, first + count, stream, ptr_out);
}

skel_status skel_container_valid_ranges(const skel_container* c, skel_place place,
                                        int64_t* pairs, int64_t max_pairs, int64_t* count) {
    if (!c || !count) return fail(SKEL_E_INVAL, "null argument");
    if (place != SKEL_HOST && place != SKEL_DEVICE)
        return fail(SKEL_E_INVAL, "bad place %d", (int)place);
    const auto& s = place == SKEL_HOST ? c->valid_host : c->valid_dev;
    *count = (int64_t)s.r.size();
    if (pairs)
        for (int64_t k = 0; k < *count && k < max_pairs; ++k) {
            pairs[2 * k] = s.r[k].first;
            pairs[2 * k + 1] = s.r[k].second;
        }
    return SKEL_OK;
}

skel_status skel_container_release(skel_container* c, skel_place place,
                                   void* stream) {
    if (!rt().initialized) return fail(SKEL_E_NOINIT, "skel_init has not been called");
    return release(c, place, stream);
}

skel_status skel_container_stats(const skel_container* c, skel_xfer_stats* out) {
    if (!c || !out) return fail(SKEL_E_INVAL, "null argument");
    *out = c->stats;
    return SKEL_OK;
}

skel_status skel_container_info(const skel_container* c, skel_dtype* dtype,
                                int64_t* rows, int64_t* cols) {
    if (!c) return fail(SKEL_E_INVAL, "null container");
    if (dtype) *dtype = c->dtype;
    if (rows) *rows = c->rows;
    if (cols) *cols = c->cols;
    return SKEL_OK;
}

}  // extern "C"
