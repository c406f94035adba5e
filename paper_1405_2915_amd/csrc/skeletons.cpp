// Skeleton entry points of the C ABI.  Each call: validate the arguments and
// the operands' container states (no side effect on failure), let the
// execution plan pick a variant (Section III), acquire every operand on the
// device through the coherence protocol (Section IV: this is where lazy
// copies happen), enqueue the kernels on the caller's stream, and release the
// operands, which records their dependence events (Section V).  Nothing
// waits: results stay on the device until a host acquire.
#include <cmath>
#include <cstring>
#include <vector>

#include "container.hpp"
#include "dispatch.hpp"
#include "launch.hpp"

namespace skel {

namespace {

// The operands of one call.  A container named twice is acquired once with
// the union of the access modes (e.g. in-place Map: READ + WRITE = RW).
class Operands {
  public:
    skel_status add(skel_container* c, skel_access a) {
        if (!c) return fail(SKEL_E_INVAL, "null container operand");
        for (int i = 0; i < n_; ++i)
            if (ops_[i].c == c) {
                ops_[i].access = (skel_access)(ops_[i].access | a);
                count_eager(c, a);
                return SKEL_OK;
            }
        ops_[n_] = Op();
        ops_[n_].c = c;
        ops_[n_].access = a;
        ops_[n_].ptr = nullptr;
        ops_[n_].held = false;
        ++n_;
        count_eager(c, a);
        return SKEL_OK;
    }
    skel_status check() const {
        for (int i = 0; i < n_; ++i) {
            skel_status st = check_acquire(ops_[i].c, SKEL_DEVICE, ops_[i].access);
            if (st != SKEL_OK) return st;
        }
        return SKEL_OK;
    }
    // Acquire every operand on the device.  The validity of each written
    // operand is remembered first, so that a call failing before its kernels
    // are enqueued (an acquire, or a workspace that cannot grow) can put it
    // back: a failed call has no side effect on the coherence state.
    skel_status acquire_all(void* stream) {
        for (int i = 0; i < n_; ++i)
            if (ops_[i].access & SKEL_WRITE) {
                ops_[i].saved_host = ops_[i].c->valid_host;
                ops_[i].saved_dev = ops_[i].c->valid_dev;
            }
        for (int i = 0; i < n_; ++i) {
            skel_status st = acquire(ops_[i].c, SKEL_DEVICE, ops_[i].access, stream,
                                     &ops_[i].ptr);
            if (st != SKEL_OK) {
                release_all(stream);
                restore_written();
                return st;
            }
            ops_[i].held = true;
            ops_[i].acquired = true;
        }
        return SKEL_OK;
    }
    // Undo the validity changes of the written operands (the call enqueued
    // nothing that writes them).
    void restore_written() {
        for (int i = 0; i < n_; ++i)
            if (ops_[i].acquired && (ops_[i].access & SKEL_WRITE)) {
                ops_[i].c->valid_host = ops_[i].saved_host;
                ops_[i].c->valid_dev = ops_[i].saved_dev;
                ops_[i].acquired = false;
            }
    }
    void release_all(void* stream) {
        for (int i = 0; i < n_; ++i)
            if (ops_[i].held) {
                release(ops_[i].c, SKEL_DEVICE, stream);
                ops_[i].held = false;
            }
    }
    // Eager-equivalent accounting (Section IV comparison point): an eager
    // scheme copies every input in and every output out at every call.
    void commit_eager() {
        for (int i = 0; i < pending_n_; ++i) pending_[i].c->stats.eager_equiv += pending_[i].k;
    }
    void* ptr(const skel_container* c) const {
        for (int i = 0; i < n_; ++i)
            if (ops_[i].c == c) return ops_[i].ptr;
        return nullptr;
    }

  private:
    struct Op {
        skel_container* c;
        skel_access access;
        void* ptr;
        bool held;
        bool acquired = false;
        skel_ranges saved_host, saved_dev;  // validity before the call (written operands)
    };
    struct Pending {
        skel_container* c;
        uint64_t k;
    };
    void count_eager(skel_container* c, skel_access a) {
        uint64_t k = ((a & SKEL_READ) ? 1 : 0) + ((a & SKEL_WRITE) ? 1 : 0);
        pending_[pending_n_++] = {c, k};
    }
    Op ops_[8];
    int n_ = 0;
    Pending pending_[16];
    int pending_n_ = 0;
};

skel_status begin(void* stream, LaunchCtx* lc) {
    if (!rt().initialized) return fail(SKEL_E_NOINIT, "skel_init has not been called");
    lc->stream = reinterpret_cast<hipStream_t>(stream);
    lc->dev = &device_info();
    return SKEL_OK;
}

// Run `launch` between acquire and release of the operands.
template <class F>
skel_status run(Operands& ops, void* stream, LaunchCtx& lc, F&& launch) {
    skel_status st = ops.check();
    if (st != SKEL_OK) return st;
    st = workspace_for(stream, &lc.ws);
    if (st != SKEL_OK) return st;
    st = ops.acquire_all(stream);
    if (st != SKEL_OK) return st;
    st = launch();
    ops.release_all(stream);
    if (st == SKEL_OK) {
        ops.commit_eager();
    } else if (st == SKEL_E_STATE || st == SKEL_E_NOMEM) {
        // the launchers take their workspace before enqueuing any kernel, so
        // these failures leave the operands' data as it was
        ops.restore_written();
    }
    return st;
}

bool map_op_valid(int op) { return op >= SKEL_MAP_IDENTITY && op <= SKEL_MAP_SQUARE; }
int map_inputs(int op) { return (op == SKEL_MAP_AXPY || op == SKEL_MAP_MUL) ? 2 : 1; }
int map_params(int op) {
    switch (op) {
    case SKEL_MAP_AXPY: return 1;
    case SKEL_MAP_AFFINE:
    case SKEL_MAP_AFFINE_TANH: return 2;
    default: return 0;
    }
}
bool reduce_op_valid(int op) { return op >= SKEL_SUM && op <= SKEL_MAX; }

skel_status check_map_args(int op, const double* params, int nparams,
                           skel_container* const* in, int nin, float* p0, float* p1) {
    if (!map_op_valid(op)) return fail(SKEL_E_INVAL, "unknown map op %d", op);
    if (nin != map_inputs(op))
        return fail(SKEL_E_INVAL, "map op %d takes %d input(s), got %d", op,
                    map_inputs(op), nin);
    if (!in) return fail(SKEL_E_INVAL, "null input array");
    if (nparams < map_params(op) || (nparams > 0 && !params))
        return fail(SKEL_E_INVAL, "map op %d needs %d parameter(s)", op, map_params(op));
    *p0 = nparams > 0 ? (float)params[0] : 0.0f;
    *p1 = nparams > 1 ? (float)params[1] : 0.0f;
    for (int i = 0; i < nin; ++i)
        if (!in[i]) return fail(SKEL_E_INVAL, "null input container %d", i);
    return SKEL_OK;
}

}  // namespace
}  // namespace skel

using namespace skel;

extern "C" {

skel_status skel_map(skel_map_op op, const double* params, int nparams,
                     skel_container* const* in, int nin, skel_container* out,
                     int variant, void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    float p0, p1;
    st = check_map_args(op, params, nparams, in, nin, &p0, &p1);
    if (st != SKEL_OK) return st;
    if (!out) return fail(SKEL_E_INVAL, "null output container");
    for (int i = 0; i < nin; ++i) {
        if (in[i]->dtype != SKEL_F32) return fail(SKEL_E_DTYPE, "Map inputs must be f32");
        if (in[i]->n != out->n) return fail(SKEL_E_SHAPE, "Map operand sizes differ");
    }
    if (out->dtype != SKEL_F32) return fail(SKEL_E_DTYPE, "Map output must be f32");
    CallContext cc;
    cc.skeleton = SKEL_SK_MAP;
    cc.n = out->n;
    cc.op = op;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    for (int i = 0; i < nin; ++i) ops.add(in[i], SKEL_READ);
    ops.add(out, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        if (out->n == 0) return SKEL_OK;
        const float* x = (const float*)ops.ptr(in[0]);
        const float* y = nin > 1 ? (const float*)ops.ptr(in[1]) : nullptr;
        return launch_map(v, op, p0, p1, x, y, (float*)ops.ptr(out), out->n, lc);
    });
}

skel_status skel_reduce(skel_reduce_op op, skel_container* in, skel_container* out1,
                        int variant, void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!reduce_op_valid(op)) return fail(SKEL_E_INVAL, "unknown reduce op %d", (int)op);
    if (!in || !out1) return fail(SKEL_E_INVAL, "null container");
    if (in == out1) return fail(SKEL_E_INVAL, "Reduce output must differ from its input");
    if (out1->n != 1) return fail(SKEL_E_SHAPE, "Reduce output must hold one element");
    const skel_dtype a = in->dtype, b = out1->dtype;
    bool ok = (a == SKEL_F32 && b == SKEL_F32) || (a == SKEL_BF16 && b == SKEL_F32) ||
              (a == SKEL_I32 && (b == SKEL_I32 || b == SKEL_I64)) ||
              (a == SKEL_I64 && b == SKEL_I64);
    if (!ok)
        return fail(SKEL_E_DTYPE, "Reduce %s -> %s not supported", dtype_name(a),
                    dtype_name(b));
    CallContext cc;
    cc.skeleton = SKEL_SK_REDUCE;
    cc.din = a;
    cc.dout = b;
    cc.n = in->n;
    cc.op = op;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    ops.add(in, SKEL_READ);
    ops.add(out1, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        return launch_reduce(v, op, a, b, ops.ptr(in), in->n, ops.ptr(out1), lc);
    });
}

skel_status skel_mapreduce(skel_map_op map_op, const double* params, int nparams,
                           skel_container* const* in, int nin, skel_reduce_op op,
                           skel_container* out1, int variant, void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    float p0, p1;
    st = check_map_args(map_op, params, nparams, in, nin, &p0, &p1);
    if (st != SKEL_OK) return st;
    if (!reduce_op_valid(op)) return fail(SKEL_E_INVAL, "unknown reduce op %d", (int)op);
    if (!out1) return fail(SKEL_E_INVAL, "null output container");
    if (out1->n != 1 || out1->dtype != SKEL_F32)
        return fail(SKEL_E_SHAPE, "MapReduce output must be one f32 element");
    const skel_dtype a = in[0]->dtype;
    for (int i = 0; i < nin; ++i) {
        if (in[i] == out1) return fail(SKEL_E_INVAL, "MapReduce output aliases an input");
        if (in[i]->dtype != a) return fail(SKEL_E_DTYPE, "MapReduce inputs differ in dtype");
        if (in[i]->n != in[0]->n) return fail(SKEL_E_SHAPE, "MapReduce input sizes differ");
    }
    bool bf16_ok = map_op == SKEL_MAP_IDENTITY || map_op == SKEL_MAP_MUL ||
                   map_op == SKEL_MAP_SQUARE;
    if (!(a == SKEL_F32 || (a == SKEL_BF16 && bf16_ok)))
        return fail(SKEL_E_DTYPE, "MapReduce over %s with map op %d not supported",
                    dtype_name(a), (int)map_op);
    CallContext cc;
    cc.skeleton = SKEL_SK_MAPREDUCE;
    cc.din = a;
    cc.n = in[0]->n;
    cc.op = op;
    cc.map_op = map_op;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    for (int i = 0; i < nin; ++i) ops.add(in[i], SKEL_READ);
    ops.add(out1, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        const void* x = ops.ptr(in[0]);
        const void* y = nin > 1 ? ops.ptr(in[1]) : nullptr;
        return launch_mapreduce(v, map_op, p0, p1, a, x, y, in[0]->n, op,
                                (float*)ops.ptr(out1), lc);
    });
}

skel_status skel_mapoverlap1d(skel_container* in, skel_container* out, const float* w,
                              int radius, skel_edge edge, float pad, int variant,
                              void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!in || !out || !w) return fail(SKEL_E_INVAL, "null argument");
    if (in == out) return fail(SKEL_E_INVAL, "MapOverlap cannot run in place");
    if (radius < 0 || radius > SKEL_MAX_RADIUS_1D)
        return fail(SKEL_E_INVAL, "radius %d outside 0..%d", radius, SKEL_MAX_RADIUS_1D);
    if (edge < SKEL_EDGE_CLAMP || edge > SKEL_EDGE_CYCLIC)
        return fail(SKEL_E_INVAL, "unknown edge rule %d", (int)edge);
    if (in->dtype != SKEL_F32 || out->dtype != SKEL_F32)
        return fail(SKEL_E_DTYPE, "MapOverlap operands must be f32");
    if (in->n != out->n) return fail(SKEL_E_SHAPE, "MapOverlap operand sizes differ");
    CallContext cc;
    cc.skeleton = SKEL_SK_MAPOVERLAP1D;
    cc.n = in->n;
    cc.radius = radius;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    ops.add(in, SKEL_READ);
    ops.add(out, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        if (in->n == 0) return SKEL_OK;
        return launch_overlap1d(v, (const float*)ops.ptr(in), (float*)ops.ptr(out), in->n,
                                w, radius, edge, pad, lc);
    });
}

skel_status skel_mapoverlap2d_fields(skel_container* in, skel_container* out, int64_t fields,
                                     const float* w2d, const float* wy, const float* wx, int ry,
                                     int rx, skel_edge edge, float pad, int variant,
                                     void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!in || !out) return fail(SKEL_E_INVAL, "null container");
    if (in == out) return fail(SKEL_E_INVAL, "MapOverlap cannot run in place");
    if (!w2d && (!wy || !wx))
        return fail(SKEL_E_INVAL, "need w2d or both separable factors wy, wx");
    if (ry < 0 || rx < 0 || ry > SKEL_MAX_RADIUS_2D || rx > SKEL_MAX_RADIUS_2D)
        return fail(SKEL_E_INVAL, "radii (%d, %d) outside 0..%d", ry, rx,
                    SKEL_MAX_RADIUS_2D);
    if (edge < SKEL_EDGE_CLAMP || edge > SKEL_EDGE_CYCLIC)
        return fail(SKEL_E_INVAL, "unknown edge rule %d", (int)edge);
    if (in->dtype != SKEL_F32 || out->dtype != SKEL_F32)
        return fail(SKEL_E_DTYPE, "MapOverlap operands must be f32");
    if (in->rows != out->rows || in->cols != out->cols)
        return fail(SKEL_E_SHAPE, "MapOverlap operand shapes differ");
    if (fields < 1 || in->rows % fields != 0)
        return fail(SKEL_E_SHAPE, "%lld rows do not split into %lld fields",
                    (long long)in->rows, (long long)fields);
    const int64_t frows = in->rows / fields;
    CallContext cc;
    cc.skeleton = SKEL_SK_MAPOVERLAP2D;
    cc.n = in->n;
    cc.rows = frows;
    cc.cols = in->cols;
    cc.separable = w2d ? 0 : 1;
    cc.radius = ry > rx ? ry : rx;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    ops.add(in, SKEL_READ);
    ops.add(out, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        if (in->n == 0) return SKEL_OK;
        return launch_overlap2d(v, (const float*)ops.ptr(in), (float*)ops.ptr(out), frows,
                                in->cols, fields, w2d, w2d ? nullptr : wy, w2d ? nullptr : wx,
                                ry, rx, edge, pad, lc);
    });
}

skel_status skel_mapoverlap2d(skel_container* in, skel_container* out, const float* w2d,
                              const float* wy, const float* wx, int ry, int rx,
                              skel_edge edge, float pad, int variant, void* stream) {
    return skel_mapoverlap2d_fields(in, out, 1, w2d, wy, wx, ry, rx, edge, pad, variant, stream);
}

skel_status skel_reduce_segments(skel_reduce_op op, skel_container* in,
                                 skel_container* offsets, skel_container* out, int variant,
                                 void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!reduce_op_valid(op)) return fail(SKEL_E_INVAL, "unknown reduce op %d", (int)op);
    if (!in || !offsets || !out) return fail(SKEL_E_INVAL, "null container");
    if (in == out || in == offsets || offsets == out)
        return fail(SKEL_E_INVAL, "segmented Reduce operands must be distinct containers");
    if (in->dtype != SKEL_F32 || out->dtype != SKEL_F32 || offsets->dtype != SKEL_I64)
        return fail(SKEL_E_DTYPE, "segmented Reduce takes f32 values, i64 offsets, f32 out");
    if (offsets->n != out->n + 1)
        return fail(SKEL_E_SHAPE, "offsets must hold one more element than out");
    CallContext cc;
    cc.skeleton = SKEL_SK_REDUCE_SEGMENTS;
    cc.n = in->n;
    cc.op = op;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    const int64_t nseg = out->n;
    std::vector<int64_t> off_host;
    if (v == B0_PER_SEGMENT && nseg > 0) {
        // the per-segment loop reads the offsets on the host (lazily copied)
        void* hp = nullptr;
        st = acquire(offsets, SKEL_HOST, SKEL_READ, stream, &hp);
        if (st != SKEL_OK) return st;
        const int64_t* o = static_cast<const int64_t*>(hp);
        off_host.assign(o, o + nseg + 1);
        release(offsets, SKEL_HOST, stream);
        for (int64_t s = 0; s < nseg; ++s)
            if (off_host[s] < 0 || off_host[s + 1] < off_host[s] || off_host[s + 1] > in->n)
                return fail(SKEL_E_INVAL, "offsets[%lld..%lld] = %lld, %lld not within [0, %lld]"
                            " and nondecreasing", (long long)s, (long long)s + 1,
                            (long long)off_host[s], (long long)off_host[s + 1], (long long)in->n);
    }
    Operands ops;
    ops.add(in, SKEL_READ);
    ops.add(offsets, SKEL_READ);
    ops.add(out, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        if (nseg == 0) return SKEL_OK;
        return launch_reduce_segments(v, op, (const float*)ops.ptr(in), in->n,
                                      (const int64_t*)ops.ptr(offsets),
                                      off_host.empty() ? nullptr : off_host.data(), nseg,
                                      (float*)ops.ptr(out), lc);
    });
}

skel_status skel_scan(skel_container* in, skel_container* out, skel_scan_kind kind,
                      skel_reduce_op op, int variant, void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!in || !out) return fail(SKEL_E_INVAL, "null container");
    if (kind < SKEL_INCLUSIVE || kind > SKEL_REVERSE_EXCLUSIVE)
        return fail(SKEL_E_INVAL, "unknown scan kind %d", (int)kind);
    if (!reduce_op_valid(op)) return fail(SKEL_E_INVAL, "unknown scan op %d", (int)op);
    const skel_dtype a = in->dtype, b = out->dtype;
    bool ok = (a == SKEL_I32 && (b == SKEL_I32 || b == SKEL_I64)) ||
              (a == SKEL_I64 && b == SKEL_I64) || (a == SKEL_F32 && b == SKEL_F32);
    if (!ok)
        return fail(SKEL_E_DTYPE, "Scan %s -> %s not supported", dtype_name(a),
                    dtype_name(b));
    if (in->n != out->n) return fail(SKEL_E_SHAPE, "Scan operand sizes differ");
    CallContext cc;
    cc.skeleton = SKEL_SK_SCAN;
    cc.din = a;
    cc.dout = b;
    cc.n = in->n;
    cc.op = op;
    cc.reverse = kind == SKEL_REVERSE_INCLUSIVE || kind == SKEL_REVERSE_EXCLUSIVE;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    ops.add(in, SKEL_READ);
    ops.add(out, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        if (in->n == 0) return SKEL_OK;
        return launch_scan(v, kind, op, a, b, ops.ptr(in), ops.ptr(out), in->n, lc);
    });
}

skel_status skel_scan_rows(skel_container* in, skel_container* out, skel_scan_kind kind,
                           skel_reduce_op op, int variant, void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!in || !out) return fail(SKEL_E_INVAL, "null container");
    if (kind < SKEL_INCLUSIVE || kind > SKEL_REVERSE_EXCLUSIVE)
        return fail(SKEL_E_INVAL, "unknown scan kind %d", (int)kind);
    if (!reduce_op_valid(op)) return fail(SKEL_E_INVAL, "unknown scan op %d", (int)op);
    const skel_dtype a = in->dtype, b = out->dtype;
    bool ok = (a == SKEL_I32 && (b == SKEL_I32 || b == SKEL_I64)) ||
              (a == SKEL_I64 && b == SKEL_I64) || (a == SKEL_F32 && b == SKEL_F32);
    if (!ok)
        return fail(SKEL_E_DTYPE, "Scan %s -> %s not supported", dtype_name(a),
                    dtype_name(b));
    if (in->rows != out->rows || in->cols != out->cols)
        return fail(SKEL_E_SHAPE, "row-wise Scan operand shapes differ");
    CallContext cc;
    cc.skeleton = SKEL_SK_SCAN_ROWS;
    cc.din = a;
    cc.dout = b;
    cc.n = in->n;
    cc.rows = in->rows;
    cc.cols = in->cols;
    cc.op = op;
    cc.reverse = kind == SKEL_REVERSE_INCLUSIVE || kind == SKEL_REVERSE_EXCLUSIVE;
    cc.rows_aligned = rows_aligned(a, b, in->cols);
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    int flat = -1;
    if (v == SR0_PER_ROW && in->n > 0) {
        // each row runs the flat Scan variant the plan picks for its length
        CallContext fc = cc;
        fc.skeleton = SKEL_SK_SCAN;
        fc.n = in->cols;
        fc.rows = fc.cols = 0;
        flat = choose_variant(SKEL_VARIANT_AUTO, fc, &st);
        if (flat < 0) return st;
    }
    Operands ops;
    ops.add(in, SKEL_READ);
    ops.add(out, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        if (in->n == 0) return SKEL_OK;
        if (v == SR1_WAVE_PER_ROW)
            return launch_scan_rows(kind, op, a, b, ops.ptr(in), ops.ptr(out), in->rows,
                                    in->cols, cc.rows_aligned != 0, lc);
        // every row's single-pass scan takes the same descriptor array and
        // advances the epoch once: the first row's call sizes the array
        // before it enqueues anything; that no later row has to reset it
        // inside a capture is checked here, before the first row
        if (flat == S2_LOOKBACK || flat == S3_PERSISTENT_LOOKBACK ||
            flat == S4_SMALL_TILE_LOOKBACK || flat == S5_FLAT_LOOKBACK) {
            const skel_status ready = ws_status_ready(lc, 0, in->rows);
            if (ready != SKEL_OK) return ready;
        }
        const size_t sa = dtype_size(a), sb = dtype_size(b);
        const char* x = static_cast<const char*>(ops.ptr(in));
        char* y = static_cast<char*>(ops.ptr(out));
        for (int64_t r = 0; r < in->rows; ++r) {
            const skel_status e = launch_scan(flat, kind, op, a, b, x + r * in->cols * sa,
                                              y + r * in->cols * sb, in->cols, lc);
            if (e != SKEL_OK) return e;
        }
        return SKEL_OK;
    });
}

skel_status skel_map_backward(skel_map_op op, const double* params, int nparams,
                              skel_container* const* in, int nin, skel_container* g,
                              skel_container* const* grad_in, skel_container* grad_params,
                              void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    float p0, p1;
    st = check_map_args(op, params, nparams, in, nin, &p0, &p1);
    if (st != SKEL_OK) return st;
    if (!g || !grad_in) return fail(SKEL_E_INVAL, "null gradient argument");
    const int64_t n = in[0]->n;
    for (int i = 0; i < nin; ++i) {
        if (!grad_in[i]) return fail(SKEL_E_INVAL, "null gradient container %d", i);
        if (in[i]->dtype != SKEL_F32 || grad_in[i]->dtype != SKEL_F32)
            return fail(SKEL_E_DTYPE, "Map backward operands must be f32");
        if (in[i]->n != n || grad_in[i]->n != n)
            return fail(SKEL_E_SHAPE, "Map backward operand sizes differ");
        if (grad_in[i] == g) return fail(SKEL_E_INVAL, "gradient output aliases g");
        for (int k = 0; k < nin; ++k)
            if (grad_in[i] == in[k]) return fail(SKEL_E_INVAL, "gradient output aliases an input");
        if (i == 1 && grad_in[1] == grad_in[0])
            return fail(SKEL_E_INVAL, "the two gradient outputs alias");
    }
    if (g->dtype != SKEL_F32) return fail(SKEL_E_DTYPE, "g must be f32");
    const bool bcast = g->n == 1 && n != 1;
    if (!bcast && g->n != n) return fail(SKEL_E_SHAPE, "g has %lld elements, expected %lld or 1",
                                         (long long)g->n, (long long)n);
    const int np = op == SKEL_MAP_AXPY ? 1 : (op == SKEL_MAP_AFFINE || op == SKEL_MAP_AFFINE_TANH) ? 2 : 0;
    if (grad_params) {
        if (grad_params->dtype != SKEL_F32) return fail(SKEL_E_DTYPE, "grad_params must be f32");
        if (grad_params->n != np)
            return fail(SKEL_E_SHAPE, "grad_params has %lld elements, the op has %d parameter(s)",
                        (long long)grad_params->n, np);
        for (int k = 0; k < nin; ++k)
            if (grad_params == in[k] || grad_params == grad_in[k] || grad_params == g)
                return fail(SKEL_E_INVAL, "grad_params aliases another operand");
    }
    Operands ops;
    for (int i = 0; i < nin; ++i) ops.add(in[i], SKEL_READ);
    ops.add(g, SKEL_READ);
    for (int i = 0; i < nin; ++i) ops.add(grad_in[i], SKEL_WRITE);
    if (grad_params && np > 0) ops.add(grad_params, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        float* dp = grad_params && np > 0 ? (float*)ops.ptr(grad_params) : nullptr;
        if (n == 0 && !dp) return SKEL_OK;  // (n = 0 with parameters: empty sums, zeros)
        const float* x = (const float*)ops.ptr(in[0]);
        const float* y = nin > 1 ? (const float*)ops.ptr(in[1]) : nullptr;
        float* dy = nin > 1 ? (float*)ops.ptr(grad_in[1]) : nullptr;
        return launch_map_backward(op, p0, p1, x, y, (const float*)ops.ptr(g), bcast,
                                   (float*)ops.ptr(grad_in[0]), dy, n, dp, lc);
    });
}

skel_status skel_mapoverlap1d_backward(skel_container* g, skel_container* grad_in,
                                       const float* w, int radius, skel_edge edge,
                                       int variant, void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!g || !grad_in || !w) return fail(SKEL_E_INVAL, "null argument");
    if (g == grad_in) return fail(SKEL_E_INVAL, "MapOverlap backward cannot run in place");
    if (radius < 0 || radius > SKEL_MAX_RADIUS_1D)
        return fail(SKEL_E_INVAL, "radius %d outside 0..%d", radius, SKEL_MAX_RADIUS_1D);
    if (edge < SKEL_EDGE_CLAMP || edge > SKEL_EDGE_CYCLIC)
        return fail(SKEL_E_INVAL, "unknown edge rule %d", (int)edge);
    if (g->dtype != SKEL_F32 || grad_in->dtype != SKEL_F32)
        return fail(SKEL_E_DTYPE, "MapOverlap backward operands must be f32");
    if (g->n != grad_in->n) return fail(SKEL_E_SHAPE, "MapOverlap backward sizes differ");
    CallContext cc;
    cc.skeleton = SKEL_SK_MAPOVERLAP1D_BACKWARD;
    cc.n = g->n;
    cc.radius = radius;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    ops.add(g, SKEL_READ);
    ops.add(grad_in, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        if (g->n == 0) return SKEL_OK;
        return launch_overlap1d_adjoint(v, (const float*)ops.ptr(g), (float*)ops.ptr(grad_in),
                                        g->n, w, radius, edge, lc);
    });
}

skel_status skel_mapoverlap2d_fields_backward(skel_container* g, skel_container* grad_in,
                                              int64_t fields, const float* w2d, const float* wy,
                                              const float* wx, int ry, int rx, skel_edge edge,
                                              int variant, void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!g || !grad_in) return fail(SKEL_E_INVAL, "null container");
    if (g == grad_in) return fail(SKEL_E_INVAL, "MapOverlap backward cannot run in place");
    if (!w2d && (!wy || !wx))
        return fail(SKEL_E_INVAL, "need w2d or both separable factors wy, wx");
    if (ry < 0 || rx < 0 || ry > SKEL_MAX_RADIUS_2D || rx > SKEL_MAX_RADIUS_2D)
        return fail(SKEL_E_INVAL, "radii (%d, %d) outside 0..%d", ry, rx, SKEL_MAX_RADIUS_2D);
    if (edge < SKEL_EDGE_CLAMP || edge > SKEL_EDGE_CYCLIC)
        return fail(SKEL_E_INVAL, "unknown edge rule %d", (int)edge);
    if (g->dtype != SKEL_F32 || grad_in->dtype != SKEL_F32)
        return fail(SKEL_E_DTYPE, "MapOverlap backward operands must be f32");
    if (g->rows != grad_in->rows || g->cols != grad_in->cols)
        return fail(SKEL_E_SHAPE, "MapOverlap backward shapes differ");
    if (fields < 1 || g->rows % fields != 0)
        return fail(SKEL_E_SHAPE, "%lld rows do not split into %lld fields",
                    (long long)g->rows, (long long)fields);
    const int64_t frows = g->rows / fields;
    CallContext cc;
    cc.skeleton = SKEL_SK_MAPOVERLAP2D_BACKWARD;
    cc.n = g->n;
    cc.rows = frows;
    cc.cols = g->cols;
    cc.separable = w2d ? 0 : 1;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    ops.add(g, SKEL_READ);
    ops.add(grad_in, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        if (g->n == 0) return SKEL_OK;
        return launch_overlap2d_adjoint(v, (const float*)ops.ptr(g), (float*)ops.ptr(grad_in),
                                        frows, g->cols, fields, w2d, wy, wx, ry, rx, edge, lc);
    });
}

skel_status skel_mapoverlap2d_backward(skel_container* g, skel_container* grad_in,
                                       const float* w2d, const float* wy, const float* wx,
                                       int ry, int rx, skel_edge edge, int variant,
                                       void* stream) {
    return skel_mapoverlap2d_fields_backward(g, grad_in, 1, w2d, wy, wx, ry, rx, edge, variant,
                                             stream);
}

// the chain's Map step: a one-input element function
static bool chain_map_op_valid(int op) {
    return op == SKEL_MAP_IDENTITY || op == SKEL_MAP_AFFINE || op == SKEL_MAP_TANH ||
           op == SKEL_MAP_AFFINE_TANH || op == SKEL_MAP_SQUARE;
}

// arguments common to the chain's forward and backward calls
static skel_status check_chain_args(skel_map_op map_op, const double* params, int nparams,
                                    skel_container* in, int64_t fields, const float* w2d,
                                    const float* wy, const float* wx, int ry, int rx,
                                    skel_edge edge, float* p0, float* p1, int64_t* frows) {
    if (!chain_map_op_valid(map_op))
        return fail(SKEL_E_INVAL, "the chain's Map takes a one-input element function, not %d",
                    (int)map_op);
    skel_status st = check_map_args(map_op, params, nparams, &in, 1, p0, p1);
    if (st != SKEL_OK) return st;
    if (!w2d && (!wy || !wx))
        return fail(SKEL_E_INVAL, "need w2d or both separable factors wy, wx");
    if (ry < 0 || rx < 0 || ry > SKEL_MAX_RADIUS_2D || rx > SKEL_MAX_RADIUS_2D)
        return fail(SKEL_E_INVAL, "radii (%d, %d) outside 0..%d", ry, rx, SKEL_MAX_RADIUS_2D);
    if (edge < SKEL_EDGE_CLAMP || edge > SKEL_EDGE_CYCLIC)
        return fail(SKEL_E_INVAL, "unknown edge rule %d", (int)edge);
    if (in->dtype != SKEL_F32) return fail(SKEL_E_DTYPE, "the chain's input must be f32");
    if (fields < 1 || in->rows % fields != 0)
        return fail(SKEL_E_SHAPE, "%lld rows do not split into %lld fields",
                    (long long)in->rows, (long long)fields);
    *frows = in->rows / fields;
    return SKEL_OK;
}

skel_status skel_map_overlap2d_reduce(skel_map_op map_op, const double* params, int nparams,
                                      skel_container* in, int64_t fields, const float* w2d,
                                      const float* wy, const float* wx, int ry, int rx,
                                      skel_edge edge, float pad, skel_container* out1,
                                      int variant, void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!in || !out1) return fail(SKEL_E_INVAL, "null container");
    float p0, p1;
    int64_t frows = 0;
    st = check_chain_args(map_op, params, nparams, in, fields, w2d, wy, wx, ry, rx, edge, &p0,
                          &p1, &frows);
    if (st != SKEL_OK) return st;
    if (out1 == in) return fail(SKEL_E_INVAL, "the chain's output aliases its input");
    if (out1->n != 1 || out1->dtype != SKEL_F32)
        return fail(SKEL_E_SHAPE, "the chain's output must be one f32 element");
    CallContext cc;
    cc.skeleton = SKEL_SK_MAP_OVERLAP2D_REDUCE;
    cc.n = in->n;
    cc.rows = frows;
    cc.cols = in->cols;
    cc.op = map_op;
    cc.separable = w2d ? 0 : 1;
    cc.radius = ry > rx ? ry : rx;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    ops.add(in, SKEL_READ);
    ops.add(out1, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        if (in->n == 0)  // no pixels, no terms: the empty sum
            return launch_reduce(R0_SINGLE_WG, SKEL_SUM, SKEL_F32, SKEL_F32, nullptr, 0,
                                 ops.ptr(out1), lc);
        return launch_chain(v, map_op, p0, p1, (const float*)ops.ptr(in), frows, in->cols, fields,
                            w2d, w2d ? nullptr : wy, w2d ? nullptr : wx, ry, rx, edge, pad,
                            (float*)ops.ptr(out1), lc);
    });
}

skel_status skel_map_overlap2d_reduce_backward(skel_map_op map_op, const double* params,
                                               int nparams, skel_container* in, int64_t fields,
                                               const float* w2d, const float* wy,
                                               const float* wx, int ry, int rx, skel_edge edge,
                                               skel_container* g1, skel_container* grad_in,
                                               skel_container* grad_params, int variant,
                                               void* stream) {
    LaunchCtx lc;
    skel_status st = begin(stream, &lc);
    if (st != SKEL_OK) return st;
    if (!in || !g1 || !grad_in) return fail(SKEL_E_INVAL, "null container");
    float p0, p1;
    int64_t frows = 0;
    st = check_chain_args(map_op, params, nparams, in, fields, w2d, wy, wx, ry, rx, edge, &p0,
                          &p1, &frows);
    if (st != SKEL_OK) return st;
    if (g1->n != 1 || g1->dtype != SKEL_F32)
        return fail(SKEL_E_SHAPE, "g1 must be one f32 element");
    if (grad_in->dtype != SKEL_F32 || grad_in->rows != in->rows || grad_in->cols != in->cols)
        return fail(SKEL_E_SHAPE, "grad_in must be an f32 container shaped like in");
    if (grad_in == in || grad_in == g1 || g1 == in)
        return fail(SKEL_E_INVAL, "the chain's backward operands must be distinct containers");
    const int np = map_op == SKEL_MAP_AFFINE || map_op == SKEL_MAP_AFFINE_TANH ? 2 : 0;
    if (grad_params) {
        if (grad_params->dtype != SKEL_F32) return fail(SKEL_E_DTYPE, "grad_params must be f32");
        if (grad_params->n != np)
            return fail(SKEL_E_SHAPE, "grad_params has %lld elements, the op has %d parameter(s)",
                        (long long)grad_params->n, np);
        if (grad_params == in || grad_params == g1 || grad_params == grad_in)
            return fail(SKEL_E_INVAL, "grad_params aliases another operand");
    }
    CallContext cc;
    cc.skeleton = SKEL_SK_MAP_OVERLAP2D_REDUCE;
    cc.n = in->n;
    cc.rows = frows;
    cc.cols = in->cols;
    cc.op = map_op;
    cc.separable = w2d ? 0 : 1;
    cc.radius = ry > rx ? ry : rx;
    int v = choose_variant(variant, cc, &st);
    if (v < 0) return st;
    Operands ops;
    ops.add(in, SKEL_READ);
    ops.add(g1, SKEL_READ);
    ops.add(grad_in, SKEL_WRITE);
    if (grad_params && np > 0) ops.add(grad_params, SKEL_WRITE);
    return run(ops, stream, lc, [&]() -> skel_status {
        float* dp = grad_params && np > 0 ? (float*)ops.ptr(grad_params) : nullptr;
        if (in->n == 0) {
            // an empty chain: the sum is 0 whatever the parameters
            return dp ? launch_map_backward(SKEL_MAP_AFFINE, 0.0f, 0.0f, nullptr, nullptr,
                                            (const float*)ops.ptr(g1), true, nullptr, nullptr, 0,
                                            dp, lc)
                      : SKEL_OK;
        }
        return launch_chain_backward(v, map_op, p0, p1, (const float*)ops.ptr(in), frows,
                                     in->cols, fields, w2d, w2d ? nullptr : wy,
                                     w2d ? nullptr : wx, ry, rx, edge, (const float*)ops.ptr(g1),
                                     (float*)ops.ptr(grad_in), dp, lc);
    });
}

}  // extern "C"
