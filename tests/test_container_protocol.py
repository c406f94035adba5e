"""Smart-container coherence protocol (Section IV of arXiv:1405.2915) and the
execution plan (Sections II-III), tested on the CPU.

libskel_hosttest.so links the library's own container, plan and error code
(compiled by g++) with a host-memory fake of the device runtime, so every
transfer the protocol issues is counted exactly.  A small Python model of the
validity state machine replays the same acquire/release traces and predicts
status codes and transfer counts.
"""
import ctypes as C
import os
import random

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# SKEL_HOSTTEST_LIB selects another build (the sanitizer build, for one)
LIB = os.environ.get("SKEL_HOSTTEST_LIB") or os.path.join(ROOT, "paper_1405_2915_amd",
                                                          "libskel_hosttest.so")

OK, E_INVAL, E_DTYPE, E_SHAPE, E_NOMEM, E_STATE, E_UNSUP, E_HIP = range(8)
F32, BF16, I32, I64 = range(4)
HOST, DEVICE = 0, 1
READ, WRITE, RW = 1, 2, 3


class Stats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in
                ("h2d", "d2h", "h2d_bytes", "d2h_bytes", "eager_equiv", "acquires")]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libskel_hosttest.so not built (paper_1405_2915_amd/build_lib.py)")
    L = C.CDLL(LIB)
    vp = C.c_void_p
    L.skel_container_create.argtypes = [C.c_int, C.c_int64, C.c_int64, vp, C.POINTER(vp)]
    L.skel_container_destroy.argtypes = [vp]
    L.skel_container_acquire.argtypes = [vp, C.c_int, C.c_int, vp, C.POINTER(vp)]
    L.skel_container_release.argtypes = [vp, C.c_int, vp]
    L.skel_container_stats.argtypes = [vp, C.POINTER(Stats)]
    L.skel_last_error.restype = C.c_char_p
    L.skel_hosttest_counts.argtypes = [C.POINTER(C.c_ulonglong)]
    L.skel_hosttest_wait_count_on.argtypes = [vp]
    L.skel_select_variant.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64, C.c_int64,
                                      C.c_int]
    L.skel_variant_name.restype = C.c_char_p
    L.skel_load_plan.argtypes = [C.c_char_p]
    return L


@pytest.fixture()
def rt(lib):
    lib.skel_hosttest_init()
    lib.skel_clear_plan()
    return lib


def counts(lib):
    a = (C.c_ulonglong * 11)()
    lib.skel_hosttest_counts(a)
    keys = ("host_allocs", "host_frees", "dev_allocs", "dev_frees", "h2d", "d2h",
            "event_creates", "event_records", "stream_waits", "event_syncs", "stream_syncs")
    return dict(zip(keys, a))


def create(lib, n, data=None, dtype=F32):
    h = C.c_void_p()
    src = None if data is None else C.c_void_p(data.ctypes.data)
    assert lib.skel_container_create(dtype, 1, n, src, C.byref(h)) == OK
    return h


def acquire(lib, h, place, access, stream=1):
    p = C.c_void_p()
    st = lib.skel_container_acquire(h, place, access, C.c_void_p(stream), C.byref(p))
    return st, p.value


def stats(lib, h):
    s = Stats()
    assert lib.skel_container_stats(h, C.byref(s)) == OK
    return {k: getattr(s, k) for k, _ in Stats._fields_}


class Model:
    """Validity bits and outstanding accesses of one container."""

    def __init__(self, initialised):
        self.valid = {HOST: initialised, DEVICE: False}
        self.readers = {HOST: 0, DEVICE: 0}
        self.writer = None
        self.h2d = self.d2h = 0

    def acquire(self, place, access):
        if self.writer is not None:
            return E_STATE
        if access & WRITE and (self.readers[HOST] + self.readers[DEVICE]):
            return E_STATE
        if access & READ and not (self.valid[HOST] or self.valid[DEVICE]):
            return E_STATE
        other = HOST if place == DEVICE else DEVICE
        if access & READ and not self.valid[place]:
            if place == DEVICE:
                self.h2d += 1
            else:
                self.d2h += 1
        self.valid[place] = True
        if access & WRITE:
            self.valid[other] = False
            self.writer = place
        else:
            self.readers[place] += 1
        return OK

    def release(self, place):
        if self.writer == place:
            self.writer = None
            return OK
        if self.readers[place] == 0:
            return E_STATE
        self.readers[place] -= 1
        return OK


def test_lazy_copies_and_data_flow(rt):
    x = np.arange(16, dtype=np.float32)
    h = create(rt, 16, x)
    # device read: one H2D
    st, dp = acquire(rt, h, DEVICE, READ)
    assert st == OK and dp
    got = np.frombuffer((C.c_float * 16).from_address(dp), dtype=np.float32)
    assert np.array_equal(got, x)
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    # second device read: copy still valid, no transfer
    st, _ = acquire(rt, h, DEVICE, READ)
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    assert stats(rt, h)["h2d"] == 1
    # a "kernel" writes the device copy in place
    st, dp = acquire(rt, h, DEVICE, RW)
    assert st == OK
    src = np.full(16, 7.0, np.float32)  # held while its address is in use
    C.memmove(dp, src.ctypes.data, 64)
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    # host read sees the device write: exactly one D2H, and it waited first
    before = counts(rt)["event_syncs"]
    st, hp = acquire(rt, h, HOST, READ)
    assert st == OK
    host = np.frombuffer((C.c_float * 16).from_address(hp), dtype=np.float32)
    assert np.all(host == 7.0)
    assert counts(rt)["event_syncs"] > before
    assert rt.skel_container_release(h, HOST, None) == OK
    s = stats(rt, h)
    assert (s["h2d"], s["d2h"], s["h2d_bytes"], s["d2h_bytes"]) == (1, 1, 64, 64)
    # host read again: no transfer
    st, _ = acquire(rt, h, HOST, READ)
    assert st == OK and rt.skel_container_release(h, HOST, None) == OK
    assert stats(rt, h)["d2h"] == 1
    assert rt.skel_container_destroy(h) == OK


def test_chain_of_twenty_device_calls(rt):
    # Section IV: lazy copying removes the redundant transfers of a call loop.
    # 20 dependent device calls over one in/out container move data twice.
    x = np.ones(1024, np.float32)
    h = create(rt, 1024, x)
    for _ in range(20):
        st, _ = acquire(rt, h, DEVICE, RW)
        assert st == OK
        assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    # one stream: stream order is enough, no event marker was enqueued
    assert counts(rt)["event_records"] == 0
    st, _ = acquire(rt, h, HOST, READ)
    assert st == OK and rt.skel_container_release(h, HOST, None) == OK
    s = stats(rt, h)
    assert (s["h2d"], s["d2h"]) == (1, 1)
    c = counts(rt)
    assert (c["h2d"], c["d2h"], c["dev_allocs"]) == (1, 1, 1)
    assert rt.skel_container_destroy(h) == OK


def test_write_only_acquire_copies_nothing(rt):
    h = create(rt, 64)  # uninitialised
    st, _ = acquire(rt, h, DEVICE, READ)
    assert st == E_STATE and b"uninitialised" in rt.skel_last_error()
    st, _ = acquire(rt, h, DEVICE, WRITE)
    assert st == OK
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    assert counts(rt)["h2d"] == 0 and counts(rt)["host_allocs"] == 0
    st, _ = acquire(rt, h, HOST, READ)
    assert st == OK and rt.skel_container_release(h, HOST, None) == OK
    assert counts(rt)["d2h"] == 1
    # host WRITE invalidates the device copy; next device read copies again
    st, _ = acquire(rt, h, HOST, WRITE)
    assert st == OK and rt.skel_container_release(h, HOST, None) == OK
    st, _ = acquire(rt, h, DEVICE, READ)
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    assert stats(rt, h)["h2d"] == 1
    assert rt.skel_container_destroy(h) == OK


def test_conflicts_and_release_errors(rt):
    h = create(rt, 8, np.zeros(8, np.float32))
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == E_STATE
    st, _ = acquire(rt, h, DEVICE, READ)
    assert st == OK
    st, _ = acquire(rt, h, HOST, READ)  # two readers are fine
    assert st == OK
    st, _ = acquire(rt, h, HOST, WRITE)  # writer while readers are out
    assert st == E_STATE
    assert rt.skel_container_destroy(h) == E_STATE
    assert rt.skel_container_release(h, HOST, None) == OK
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    st, _ = acquire(rt, h, DEVICE, WRITE)
    assert st == OK
    st, _ = acquire(rt, h, DEVICE, READ)  # anything while a writer is out
    assert st == E_STATE
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    assert rt.skel_container_acquire(h, 7, READ, None, C.byref(C.c_void_p())) == E_INVAL
    assert rt.skel_container_acquire(h, HOST, 0, None, C.byref(C.c_void_p())) == E_INVAL
    assert rt.skel_container_destroy(h) == OK


def test_cross_stream_dependence(rt):
    # Section V: containers carry dependences between asynchronous calls; an
    # access on another stream must wait for the last access's event
    h = create(rt, 32, np.zeros(32, np.float32))
    st, _ = acquire(rt, h, DEVICE, RW, stream=11)
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(11)) == OK
    assert rt.skel_hosttest_wait_count_on(C.c_void_p(22)) == 0
    st, _ = acquire(rt, h, DEVICE, READ, stream=22)
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(22)) == OK
    assert rt.skel_hosttest_wait_count_on(C.c_void_p(22)) == 1
    # same stream: stream order suffices, no wait
    st, _ = acquire(rt, h, DEVICE, READ, stream=22)
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(22)) == OK
    assert rt.skel_hosttest_wait_count_on(C.c_void_p(22)) == 1
    # a writer on a third stream waits for both earlier streams
    st, _ = acquire(rt, h, DEVICE, WRITE, stream=33)
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(33)) == OK
    assert rt.skel_hosttest_wait_count_on(C.c_void_p(33)) == 2
    assert rt.skel_container_destroy(h) == OK


def test_reads_on_other_streams_are_not_ordered(rt):
    # only conflicting accesses are ordered: reads of one operand on different
    # streams run concurrently, writes (a reader's copy of stale data included)
    # are ordered against everything
    h = create(rt, 32, np.zeros(32, np.float32))
    waits = lambda s: rt.skel_hosttest_wait_count_on(C.c_void_p(s))
    for s in (11, 22, 11, 33):  # 11 copies the host data: a write
        st, _ = acquire(rt, h, DEVICE, READ, stream=s)
        assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(s)) == OK
    assert (waits(11), waits(22), waits(33)) == (0, 1, 1)  # 22 and 33 after 11's copy only
    st, _ = acquire(rt, h, DEVICE, WRITE, stream=44)  # a writer waits for every reader
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(44)) == OK
    assert waits(44) == 3
    st, _ = acquire(rt, h, DEVICE, READ, stream=22)  # and a reader for the writer
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(22)) == OK
    assert waits(22) == 2
    assert rt.skel_container_destroy(h) == OK


def _device_access(rt, h, stream, access):
    """acquire on the device, one stand-in kernel, release; returns the
    (operation, writes) pairs of the access: its copies, then the kernel"""
    first = rt.skel_hosttest_op_count()
    st, _ = acquire(rt, h, DEVICE, access, stream=stream)
    if st != OK:
        return st, []
    copies = [(i, True) for i in range(first, rt.skel_hosttest_op_count())]
    k = rt.skel_hosttest_enqueue(C.c_void_p(stream))
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(stream)) == OK
    return st, copies + [(k, access != READ)]


@pytest.mark.parametrize("seed", range(16))
def test_random_stream_traces_order_every_conflict(rt, seed):
    """Random device and host accesses on four streams, checked against a
    vector-clock model of the fake runtime: every pair of operations that
    touch the device copy from different streams, one of them a write, is
    ordered (the earlier completes before the later starts); every host access
    comes after all earlier device operations."""
    rt.skel_hosttest_enqueue.argtypes = [C.c_void_p]
    rnd = random.Random(seed)
    h = create(rt, 16, np.zeros(16, np.float32))
    ops = []  # (operation, writes) of every device access so far
    unordered_reads = 0
    for _ in range(200):
        if rnd.random() < 0.15:
            access = rnd.choice((READ, WRITE, RW))
            first = rt.skel_hosttest_op_count()
            st, _ = acquire(rt, h, HOST, access)
            assert st == OK
            for i, _w in ops:
                assert rt.skel_hosttest_op_before_host(i), (seed, i)
            ops += [(i, False) for i in range(first, rt.skel_hosttest_op_count())]  # D2H
            assert rt.skel_container_release(h, HOST, None) == OK
            continue
        stream = rnd.choice((11, 22, 33, 44))
        st, mine = _device_access(rt, h, stream, rnd.choice((READ, READ, WRITE, RW)))
        assert st == OK
        for j, wj in mine:
            for i, wi in ops:
                if wi or wj:
                    assert rt.skel_hosttest_op_before(i, j), (seed, i, j)
                elif not rt.skel_hosttest_op_before(i, j):
                    unordered_reads += 1
        ops += mine
    assert rt.skel_container_destroy(h) == OK
    assert unordered_reads > 0  # reads on different streams did overlap


def test_injected_failures_leave_state_unchanged(rt):
    x = np.arange(8, dtype=np.float32)
    h = create(rt, 8, x)
    rt.skel_hosttest_fail_dev_alloc(1)
    st, _ = acquire(rt, h, DEVICE, READ)
    assert st == E_NOMEM
    rt.skel_hosttest_fail_copy(1)
    st, _ = acquire(rt, h, DEVICE, READ)
    assert st == E_HIP
    s = stats(rt, h)
    assert (s["h2d"], s["acquires"]) == (0, 0)
    st, _ = acquire(rt, h, DEVICE, READ)  # recovers
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    assert stats(rt, h)["h2d"] == 1
    assert rt.skel_container_destroy(h) == OK
    c = counts(rt)
    assert c["dev_allocs"] == c["dev_frees"] == 1
    assert c["host_allocs"] == c["host_frees"] == 1


@pytest.mark.parametrize("seed", range(12))
def test_random_traces_match_model(rt, seed):
    rnd = random.Random(seed)
    init = rnd.random() < 0.7
    h = create(rt, 4, np.zeros(4, np.int32) if init else None, dtype=I32)
    m = Model(init)
    held = []
    for _ in range(300):
        if held and rnd.random() < 0.45:
            place = held.pop(rnd.randrange(len(held)))
            assert rt.skel_container_release(h, place, C.c_void_p(1)) == m.release(place)
            continue
        place = rnd.choice((HOST, DEVICE))
        access = rnd.choice((READ, WRITE, RW))
        expect = m.acquire(place, access)
        st, _ = acquire(rt, h, place, access)
        assert st == expect, (place, access, rt.skel_last_error())
        if st == OK:
            held.append(place)
        s = stats(rt, h)
        assert (s["h2d"], s["d2h"]) == (m.h2d, m.d2h)
    for place in held:
        assert rt.skel_container_release(h, place, C.c_void_p(1)) == OK
    assert rt.skel_container_destroy(h) == OK


def test_create_validation(rt):
    h = C.c_void_p()
    assert rt.skel_container_create(9, 1, 4, None, C.byref(h)) == E_DTYPE
    assert rt.skel_container_create(F32, 0, 4, None, C.byref(h)) == E_SHAPE
    assert rt.skel_container_create(F32, 1, -1, None, C.byref(h)) == E_SHAPE
    assert rt.skel_container_create(F32, 1 << 33, 4, None, C.byref(h)) == E_SHAPE
    # empty containers are valid everywhere and never allocate
    assert rt.skel_container_create(F32, 1, 0, None, C.byref(h)) == OK
    st, p = acquire(rt, h, DEVICE, READ)
    assert st == OK and not p
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    assert rt.skel_container_destroy(h) == OK
    assert counts(rt)["dev_allocs"] == 0


# ------------------------------------------------------------ execution plan

SK_MAP, SK_REDUCE, SK_MAPREDUCE, SK_OV1, SK_OV2, SK_SCAN, SK_SEG, SK_OV1B, SK_OV2B, \
    SK_SCANROWS, SK_CHAIN = range(11)


def name_of(lib, sk, v):
    n = lib.skel_variant_name(sk, v)
    return n.decode() if n else None


def test_variant_registry(rt):
    want = {SK_MAP: 3, SK_REDUCE: 7, SK_MAPREDUCE: 7, SK_OV1: 3, SK_OV2: 5, SK_SCAN: 6,
            SK_SEG: 2, SK_OV1B: 2, SK_OV2B: 2, SK_SCANROWS: 2, SK_CHAIN: 2}
    for sk, k in want.items():
        assert rt.skel_variant_count(sk) == k
        names = [name_of(rt, sk, v) for v in range(k)]
        assert len(set(names)) == k and all(names)
        assert rt.skel_variant_name(sk, k) is None
    assert rt.skel_variant_count(99) == 0


def test_static_plan(rt):
    sel = lambda sk, n, dt=F32, sep=0: name_of(
        rt, sk, rt.skel_select_variant(sk, dt, n, 1, n, sep))
    assert sel(SK_REDUCE, 1000) == "R0_single_wg"
    assert sel(SK_REDUCE, 1 << 26) == "R6_gather"
    assert sel(SK_REDUCE, 1 << 20, I64) == "R6_gather"
    assert sel(SK_MAPREDUCE, 1 << 26) == "MR6_fused_gather"
    assert sel(SK_MAPREDUCE, 1000) == "MR3_fused_single_wg"
    # the flat look-back up to its 1024 tiles (4096 elements each, 2048 for
    # 64-bit inputs), then the persistent look-back
    assert sel(SK_SCAN, 100, I32) == "S5_flat_lookback"
    assert sel(SK_SCAN, 1 << 22, F32) == "S5_flat_lookback"
    assert sel(SK_SCAN, (1 << 22) + 1, F32) == "S3_persistent_lookback"
    assert sel(SK_SCAN, 1 << 21, I64) == "S5_flat_lookback"
    assert sel(SK_SCAN, (1 << 21) + 1, I64) == "S3_persistent_lookback"
    assert sel(SK_SCAN, 1 << 27, I32) == "S3_persistent_lookback"
    # aux = separable + 2 * radius: the marching window up to radius 2 on large
    # images (either weight form), else the separable L1 variant or, for dense
    # weights, the LDS tile (separable variants not selectable)
    assert sel(SK_OV2, 1 << 24, F32, 1) == "O2e_march"
    assert sel(SK_OV2, 1 << 24, F32, 1 + 2 * 5) == "O2d_separable_l1"
    assert sel(SK_OV2, 1 << 18, F32, 1 + 2 * 4) == "O2d_separable_l1"
    assert sel(SK_OV2, 1 << 24, F32, 2 * 1) == "O2e_march"
    assert sel(SK_OV2, 1 << 28, F32, 2 * 2) == "O2e_march"
    assert sel(SK_OV2, 1 << 24, F32, 2 * 4) == "O2b_lds_tile"
    assert sel(SK_OV2, 1 << 22, F32, 2 * 3) == "O2b_lds_tile"
    assert sel(SK_OV2, 1 << 20, F32, 2 * 2) == "O2e_march"
    assert sel(SK_OV2, 1 << 24, F32, 2 * 5) == "O2b_lds_tile"
    assert sel(SK_OV2, 1 << 18, F32, 2 * 1) == "O2b_lds_tile"
    assert sel(SK_OV2, 1 << 24, F32, 1 + 2 * 4) == "O2d_separable_l1"
    assert sel(SK_OV2, 1 << 24, F32, 1 + 2 * 2) == "O2e_march"
    assert sel(SK_OV1, 1 << 21, F32, 2) == "O1c_shuffle"   # aux = radius
    assert sel(SK_OV1, 1 << 20, F32, 3) == "O1a_direct"    # small arrays: direct
    assert sel(SK_OV1, 1 << 20, F32, 7) == "O1b_lds_tile"  # beyond 4 neighbours
    assert sel(SK_MAP, 1 << 20) == "M2_vec4x4_nt"
    assert sel(SK_OV1B, 1 << 20, F32, 2) == "A1_flipped_forward"
    assert sel(SK_OV2B, 1 << 20, F32, 1) == "A1_flipped_forward"
    assert rt.skel_select_variant(17, F32, 10, 1, 10, 0) == -1


def test_plan_table(rt, tmp_path):
    p = tmp_path / "plan.txt"
    p.write_text("# tuned\nREDUCE f32 10 R1_two_pass\nREDUCE f32 20 R3_atomic\n"
                 "SCAN i32 12 S1_reduce_then_scan\nMAPOVERLAP2D f32 10 O2c_lds_separable 0\n")
    assert rt.skel_load_plan(str(p).encode()) == OK
    sel = lambda sk, n, dt=F32, sep=0: name_of(
        rt, sk, rt.skel_select_variant(sk, dt, n, 1, n, sep))
    assert sel(SK_REDUCE, 1 << 15) == "R1_two_pass"
    assert sel(SK_REDUCE, (1 << 20) - 5) == "R3_atomic"   # ceil(log2) = 20
    assert sel(SK_REDUCE, 1 << 28) == "R3_atomic"          # extrapolate beyond
    assert sel(SK_REDUCE, 16) == "R1_two_pass"             # below the table
    assert sel(SK_SCAN, 1 << 20, I32) == "S1_reduce_then_scan"
    assert sel(SK_SCAN, 1 << 22, I64) == "S3_persistent_lookback"  # no entry: static
    # table entry not selectable for this call: static rule instead
    assert sel(SK_OV2, 1 << 20, F32, 0) == "O2e_march"
    # a bad file is rejected whole and the old table stays
    bad = tmp_path / "bad.txt"
    bad.write_text("REDUCE f32 10 R1_two_pass\nREDUCE f99 4 nope\n")
    assert rt.skel_load_plan(str(bad).encode()) == E_INVAL
    assert sel(SK_REDUCE, 1 << 15) == "R1_two_pass"
    assert rt.skel_clear_plan() == OK
    assert sel(SK_REDUCE, 1 << 15) == "R0_single_wg"
    # MapOverlap entries must name their stencil class; other entries must not
    for text in ("MAPOVERLAP2D f32 10 O2c_lds_separable\n", "MAPOVERLAP1D f32 10 O1a_direct\n",
                 "REDUCE f32 10 R1_two_pass 3\n", "MAPOVERLAP2D f32 10 O2a_direct -1\n"):
        bad.write_text(text)
        assert rt.skel_load_plan(str(bad).encode()) == E_INVAL, text


PLAN = os.path.join(ROOT, "paper_1405_2915_amd", "plans", "gfx950.plan")


def test_default_plan_applies_to_its_stencil_class_only(rt):
    """The shipped plan's MapOverlap entries were tuned on the 9 x 9 separable
    Gaussian and the 5-point 1D binomial; calls of any other class take the
    static rules (e.g. a separable 3 x 3 on 2^24 pixels: the marching
    window)."""
    assert rt.skel_load_plan(PLAN.encode()) == OK
    sel = lambda sk, n, aux, rows=4096: name_of(
        rt, sk, rt.skel_select_variant(sk, F32, n, rows, n // rows, aux))
    assert sel(SK_OV2, 1 << 26, 1 + 2 * 1, 8192) == "O2e_march"     # separable 3 x 3
    assert sel(SK_OV2, 1 << 26, 1 + 2 * 4, 8192) == "O2d_separable_l1"  # the tuned 9 x 9
    assert sel(SK_OV2, 1 << 22, 1 + 2 * 4, 2048) == "O2c_lds_separable"
    assert sel(SK_OV2, 1 << 24, 2 * 1) == "O2e_march"               # dense 5-point
    assert sel(SK_OV2, 1 << 24, 2 * 4) == "O2b_lds_tile"            # dense 9 x 9
    assert sel(SK_OV1, 1 << 24, 2) == "O1c_shuffle"                 # the tuned radius
    assert sel(SK_OV1, 1 << 24, 7) == "O1b_lds_tile"                # static: radius > 4
    # the forward and the flipped transpose of a separable 3 x 3 agree
    assert sel(SK_OV2B, 1 << 24, 1 + 2 * 1) == "A1_flipped_forward"


def test_environment_override(rt, monkeypatch):
    monkeypatch.setenv("SKEL_VARIANT_REDUCE", "R1_two_pass")
    assert name_of(rt, SK_REDUCE, rt.skel_select_variant(SK_REDUCE, F32, 100, 1, 100, 0)) \
        == "R1_two_pass"
    monkeypatch.setenv("SKEL_VARIANT_REDUCE", "3")
    assert rt.skel_select_variant(SK_REDUCE, F32, 100, 1, 100, 0) == 3
    # the compensated variant is floating-point SUM only: an integer call
    # falls through to the static rule
    monkeypatch.setenv("SKEL_VARIANT_REDUCE", "R4_compensated")
    assert rt.skel_select_variant(SK_REDUCE, F32, 100, 1, 100, 0) == 4
    assert rt.skel_select_variant(SK_REDUCE, BF16, 100, 1, 100, 0) == 4
    assert name_of(rt, SK_REDUCE, rt.skel_select_variant(SK_REDUCE, I32, 100, 1, 100, 0)) \
        == "R0_single_wg"
    monkeypatch.setenv("SKEL_VARIANT_MAPOVERLAP2D", "O2c_lds_separable")
    # override not selectable (weights not separable): falls through
    assert name_of(rt, SK_OV2, rt.skel_select_variant(SK_OV2, F32, 100, 10, 10, 0)) \
        == "O2b_lds_tile"


# ---------------------------------------------------- wrapped device memory

def test_wrap_device_memory(rt):
    """A container over caller-owned device memory: the device copy is valid
    from the start, device reads copy nothing, a host read copies once, and
    destroy never frees the caller's memory."""
    rt.skel_container_wrap_device.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_void_p,
                                              C.c_void_p, C.POINTER(C.c_void_p)]
    buf = np.arange(64, dtype=np.float32)  # stands in for device memory (fake backend)
    h = C.c_void_p()
    assert rt.skel_container_wrap_device(F32, 1, 64, C.c_void_p(buf.ctypes.data),
                                         C.c_void_p(1), C.byref(h)) == OK
    before = counts(rt)
    st, p = acquire(rt, h, DEVICE, READ, stream=1)
    assert st == OK and p == buf.ctypes.data
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    assert counts(rt)["h2d"] == before["h2d"] and counts(rt)["dev_allocs"] == 0
    # another stream orders after the wrap's stream: one event, one wait
    st, _ = acquire(rt, h, DEVICE, READ, stream=2)
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(2)) == OK
    assert counts(rt)["stream_waits"] == before["stream_waits"] + 1
    st, hp = acquire(rt, h, HOST, READ)
    assert st == OK
    got = np.ctypeslib.as_array(C.cast(hp, C.POINTER(C.c_float)), shape=(64,)).copy()
    assert rt.skel_container_release(h, HOST, None) == OK
    assert np.array_equal(got, buf) and counts(rt)["d2h"] == before["d2h"] + 1
    assert rt.skel_container_destroy(h) == OK
    c = counts(rt)
    assert c["dev_frees"] == 0 and c["host_frees"] == c["host_allocs"]


def test_wrap_device_rejects_bad_arguments(rt):
    rt.skel_container_wrap_device.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_void_p,
                                              C.c_void_p, C.POINTER(C.c_void_p)]
    h = C.c_void_p()
    buf = np.zeros(32, np.float32)
    assert rt.skel_container_wrap_device(F32, 1, 8, None, None, C.byref(h)) == E_INVAL
    assert rt.skel_container_wrap_device(F32, 1, 8, C.c_void_p(buf.ctypes.data + 4), None,
                                         C.byref(h)) == E_INVAL  # not 16-byte aligned
    assert rt.skel_container_wrap_device(F32, 0, 8, C.c_void_p(buf.ctypes.data), None,
                                         C.byref(h)) == E_SHAPE
    assert rt.skel_container_wrap_device(9, 1, 8, C.c_void_p(buf.ctypes.data), None,
                                         C.byref(h)) == E_DTYPE
    # an empty wrapped container needs no memory
    assert rt.skel_container_wrap_device(F32, 1, 0, None, None, C.byref(h)) == OK
    assert rt.skel_container_destroy(h) == OK


def test_scan_rows_plan(rt):
    sel = lambda rows, cols, dt=I32, rev=0: name_of(
        rt, SK_SCANROWS, rt.skel_select_variant(SK_SCANROWS, dt, rows * cols, rows, cols, rev))
    assert sel(64 * 2048, 2048) == "SR1_wave_per_row"       # many rows: one launch
    assert sel(4, 1 << 24) == "SR0_per_row"                 # few long rows
    assert sel(4, (1 << 24) + 2) == "SR1_wave_per_row"      # rows not 16-byte aligned
    assert sel(4, (1 << 24) + 2, I64) == "SR0_per_row"      # 8-byte elements: aligned
    assert sel(4, 1 << 24, I32, 1) == "SR0_per_row"         # reverse kinds too
    assert rt.skel_variant_name(SK_SCANROWS, 2) is None


def test_flat_scan_size_limit(rt, tmp_path):
    """S5 (flat look-back) takes at most 1024 tiles: 2^22 elements of 4 bytes,
    2^21 of 8; beyond that a table entry naming it falls back to the static
    rule, and a forced S5 is refused."""
    p = tmp_path / "plan.txt"
    p.write_text("SCAN i32 20 S5_flat_lookback\nSCAN i64 20 S5_flat_lookback\n")
    assert rt.skel_load_plan(str(p).encode()) == OK
    sel = lambda n, dt: name_of(rt, SK_SCAN, rt.skel_select_variant(SK_SCAN, dt, n, 1, n, 0))
    assert sel(1 << 22, I32) == "S5_flat_lookback"
    assert sel((1 << 22) + 1, I32) == "S3_persistent_lookback"
    assert sel(1 << 21, I64) == "S5_flat_lookback"
    assert sel((1 << 21) + 1, I64) == "S3_persistent_lookback"
    assert rt.skel_clear_plan() == OK


def test_reverse_scan_plan(rt):
    sel = lambda n, aux: name_of(rt, SK_SCAN, rt.skel_select_variant(SK_SCAN, I32, n, 1, n,
                                                                     aux))
    assert sel(100, 0) == "S5_flat_lookback"
    assert sel(100, 1) == "S5_flat_lookback"  # the flat look-back runs the reverse kinds too
    assert sel(1 << 27, 1) == "S3_persistent_lookback"


# ------------------------------------------------- range-granular coherence

def _runs(mask):
    """[(first, last), ...] runs of True in a boolean array."""
    out, i, n = [], 0, len(mask)
    while i < n:
        if mask[i]:
            j = i
            while j < n and mask[j]:
                j += 1
            out.append((i, j))
            i = j
        else:
            i += 1
    return out


def _ranges(rt, h, place):
    cnt = C.c_int64()
    assert rt.skel_container_valid_ranges(h, place, None, 0, C.byref(cnt)) == OK
    buf = (C.c_int64 * (2 * max(cnt.value, 1)))()
    assert rt.skel_container_valid_ranges(h, place, buf, cnt.value, C.byref(cnt)) == OK
    return [(buf[2 * k], buf[2 * k + 1]) for k in range(cnt.value)]


def _setup_range_api(rt):
    rt.skel_container_acquire_range.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int64,
                                                C.c_int64, C.c_void_p, C.POINTER(C.c_void_p)]
    rt.skel_container_valid_ranges.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int64),
                                               C.c_int64, C.POINTER(C.c_int64)]


def _acq_range(rt, h, place, access, first, count, stream=1):
    p = C.c_void_p()
    st = rt.skel_container_acquire_range(h, place, access, first, count, C.c_void_p(stream),
                                         C.byref(p))
    return st, p.value


def test_partial_host_write_sends_only_that_range(rt):
    _setup_range_api(rt)
    n = 1000
    data = np.arange(n, dtype=np.float32)
    h = create(rt, n, data)
    st, _ = acquire(rt, h, DEVICE, READ)          # first device read: whole copy
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    s0 = stats(rt, h)
    assert s0["h2d"] == 1 and s0["h2d_bytes"] == 4 * n
    st, p = _acq_range(rt, h, HOST, WRITE, 100, 50)
    assert st == OK
    src = np.full(50, -1.0, np.float32)  # held while its address is in use
    C.memmove(p, src.ctypes.data, 200)
    assert rt.skel_container_release(h, HOST, None) == OK
    assert _ranges(rt, h, DEVICE) == [(0, 100), (150, n)]
    assert _ranges(rt, h, HOST) == [(0, n)]
    st, dp = acquire(rt, h, DEVICE, READ)          # whole read: copies the 50 only
    assert st == OK and rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    s1 = stats(rt, h)
    assert s1["h2d"] == 2 and s1["h2d_bytes"] == 4 * n + 200
    dev = np.ctypeslib.as_array(C.cast(dp, C.POINTER(C.c_float)), shape=(n,))
    want = data.copy()
    want[100:150] = -1.0
    assert np.array_equal(dev, want)


def test_partial_host_read_copies_only_the_range(rt):
    _setup_range_api(rt)
    n = 512
    h = create(rt, n, np.zeros(n, np.float32))
    st, dp = acquire(rt, h, DEVICE, WRITE)        # a kernel rewrites everything
    src = np.arange(n, dtype=np.float32)  # held while its address is in use
    C.memmove(dp, src.ctypes.data, 4 * n)
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    assert _ranges(rt, h, HOST) == []
    st, p = _acq_range(rt, h, HOST, READ, 10, 20)
    got = np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_float)), shape=(20,)).copy()
    assert rt.skel_container_release(h, HOST, None) == OK
    assert np.array_equal(got, np.arange(10, 30, dtype=np.float32))
    s = stats(rt, h)
    assert s["d2h"] == 1 and s["d2h_bytes"] == 80
    assert _ranges(rt, h, HOST) == [(10, 30)]
    # a range that is already current copies nothing
    st, _ = _acq_range(rt, h, HOST, READ, 12, 5)
    assert st == OK and rt.skel_container_release(h, HOST, None) == OK
    assert stats(rt, h)["d2h"] == 1


def test_range_errors(rt):
    _setup_range_api(rt)
    h = create(rt, 16)                             # uninitialised
    st, _ = _acq_range(rt, h, HOST, WRITE, 0, 8)
    assert st == OK and rt.skel_container_release(h, HOST, None) == OK
    assert _acq_range(rt, h, DEVICE, READ, 0, 8)[0] == OK
    assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
    assert _acq_range(rt, h, DEVICE, READ, 4, 8)[0] == E_STATE   # [8, 12) never written
    assert _acq_range(rt, h, HOST, READ, 10, 10)[0] == E_INVAL   # past the end
    assert _acq_range(rt, h, HOST, READ, -1, 2)[0] == E_INVAL
    assert _acq_range(rt, h, HOST, READ, 3, 0)[0] == OK          # empty range
    assert rt.skel_container_release(h, HOST, None) == OK


def test_range_protocol_random_traces(rt):
    """Random range reads and writes at both places against a model of the
    per-element validity and of the data; every transfer is counted."""
    _setup_range_api(rt)
    rng = np.random.default_rng(1405)
    for trial in range(30):
        n = int(rng.integers(1, 300))
        truth = rng.standard_normal(n).astype(np.float32)
        h = create(rt, n, truth)
        hv, dv = np.ones(n, bool), np.zeros(n, bool)
        h2d = d2h = h2d_b = d2h_b = 0
        for step in range(60):
            a = int(rng.integers(0, n + 1))
            b = int(rng.integers(a, n + 1))
            if rng.random() < 0.2:
                a, b = 0, n
            kind = int(rng.integers(0, 4))
            if kind == 0:    # host write
                vals = rng.standard_normal(b - a).astype(np.float32)
                st, p = _acq_range(rt, h, HOST, WRITE, a, b - a)
                assert st == OK
                if b > a:
                    C.memmove(p, vals.ctypes.data, 4 * (b - a))
                assert rt.skel_container_release(h, HOST, None) == OK
                truth[a:b] = vals
                hv[a:b], dv[a:b] = True, False
            elif kind == 1:  # device write (stands in for a kernel)
                vals = rng.standard_normal(b - a).astype(np.float32)
                st, p = _acq_range(rt, h, DEVICE, WRITE, a, b - a)
                assert st == OK
                if b > a:
                    C.memmove(p, vals.ctypes.data, 4 * (b - a))
                assert rt.skel_container_release(h, DEVICE, C.c_void_p(1)) == OK
                truth[a:b] = vals
                dv[a:b], hv[a:b] = True, False
            else:            # read at one place
                place = HOST if kind == 2 else DEVICE
                valid = hv if place == HOST else dv
                gaps = _runs(~valid[a:b])
                st, p = _acq_range(rt, h, place, READ, a, b - a)
                assert st == OK, (trial, step)
                got = (np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_float)), shape=(b - a,))
                       .copy() if b > a else np.zeros(0, np.float32))
                assert rt.skel_container_release(h, place, None if place == HOST
                                                 else C.c_void_p(1)) == OK
                assert np.array_equal(got, truth[a:b]), (trial, step)
                moved = sum(e - s for s, e in gaps)
                if place == HOST:
                    d2h += len(gaps)
                    d2h_b += 4 * moved
                else:
                    h2d += len(gaps)
                    h2d_b += 4 * moved
                valid[a:b] = True
            s = stats(rt, h)
            assert (s["h2d"], s["h2d_bytes"], s["d2h"], s["d2h_bytes"]) == (h2d, h2d_b, d2h, d2h_b), \
                (trial, step)
            assert _ranges(rt, h, HOST) == _runs(hv)
            assert _ranges(rt, h, DEVICE) == _runs(dv)
        assert rt.skel_container_destroy(h) == OK
