"""Parity at the full workload sizes, with the variants the execution plan
selects (the launch configuration the benchmark times):

  * plain skeletons on 2^20 elements: Map saxpy, Reduce of the saxpy x,
    inclusive int32 Scan of U{0..100}, 5-point binomial MapOverlap 1D;
  * 9x9 separable Gaussian (sigma 2) MapOverlap 2D on a 4096x4096 U[0,1)
    image, dot-product MapReduce of two 2^26 N(0,1) vectors, exclusive
    int32 -> int64 Scan of 2^27 U{0..1000}.

Every output is compared with the oracle (the 2D stencil and the scan in
full, not sampled).
"""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu


def test_small_plain_skeletons(skel, oracle_mod):
    n = 1 << 20
    x = si.uniform_f32(n, -1.0, 1.0, 0, 0)
    y = si.uniform_f32(n, -1.0, 1.0, 0, 1)
    cx, cy = skel.Container.from_numpy(x), skel.Container.from_numpy(y)
    skel.skel_map(skel.MAP_AXPY, [2.5], [cx, cy], cy)
    assert np.array_equal(cy.to_numpy(), oracle_mod.map_f32("axpy", [2.5], x, y)
                          .astype(np.float32))
    r = skel.Container.empty(skel.F32, 1)
    skel.skel_reduce(skel.SUM, cx, r)
    got = float(r.to_numpy()[0])
    assert abs(got - oracle_mod.reduce("sum", x)) <= 1e-5 * oracle_mod.abs_sum(x)
    xi = si.int_uniform_i32(n, 100, 0, 2)
    s = skel.Container.empty(skel.I32, n)
    skel.skel_scan(skel.Container.from_numpy(xi), s, skel.INCLUSIVE, skel.SUM)
    assert np.array_equal(s.to_numpy(), oracle_mod.scan(xi, "inclusive", "sum"))
    w = si.binomial5_weights()
    xo = si.uniform_f32(n, -1.0, 1.0, 0, 3)
    o = skel.Container.empty(skel.F32, n)
    skel.skel_mapoverlap1d(skel.Container.from_numpy(xo), o, w, 2, skel.EDGE_CLAMP)
    ref, mag = oracle_mod.mapoverlap1d(xo, w, 2)
    assert np.all(np.abs(o.to_numpy().astype(np.float64) - ref) <= 1e-6 * mag + 1e-30)
    skel.skel_sync()


def test_small_step_on_four_streams(skel, oracle_mod):
    """The small configuration's four calls are independent (the Map and the
    Reduce both only read x), and the containers order only conflicting
    accesses (Section V), so the four calls may run on four streams at once:
    eagerly, and as one captured graph whose four branches fork from one
    stream and join it again.  New inputs before every round, eager rounds
    between the replays; every result of every round matches the oracle."""
    import torch
    n = (1 << 20) + 3
    w = si.binomial5_weights()
    cx, cy, cz = (skel.Container.empty(skel.F32, n) for _ in range(3))
    cs = skel.Container.empty(skel.I32, n)
    cm, co = skel.Container.empty(skel.F32, n), skel.Container.empty(skel.F32, n)
    cr, cso = skel.Container.empty(skel.F32, 1), skel.Container.empty(skel.I32, n)
    main = torch.cuda.Stream()
    side = [torch.cuda.Stream() for _ in range(4)]
    calls = (lambda st: skel.skel_map(skel.MAP_AXPY, [2.5], [cx, cy], cm, stream=st),
             lambda st: skel.skel_reduce(skel.SUM, cx, cr, stream=st),
             lambda st: skel.skel_scan(cs, cso, skel.INCLUSIVE, skel.SUM, stream=st),
             lambda st: skel.skel_mapoverlap1d(cz, co, w, 2, skel.EDGE_CLAMP, stream=st))

    def put(rep):
        arrs = (si.uniform_f32(n, -1.0, 1.0, 9, 4 * rep), si.uniform_f32(n, -1.0, 1.0, 9, 4 * rep + 1),
                si.int_uniform_i32(n, 100, 9, 4 * rep + 2),
                si.uniform_f32(n, -1.0, 1.0, 9, 4 * rep + 3))
        for c, a in zip((cx, cy, cs, cz), arrs):
            c.write_numpy(a)
            skel.skel_container_acquire(c, skel.DEVICE, skel.READ, main)  # resident
            skel.skel_container_release(c, skel.DEVICE, main)
        return arrs

    def fork():
        for st, fn in zip(side, calls):
            st.wait_stream(main)
            fn(st)
        for st in side:
            main.wait_stream(st)

    def check(arrs, what):
        x, y, s, z = arrs
        assert np.array_equal(cm.to_numpy(), oracle_mod.map_f32("axpy", [2.5], x, y)
                              .astype(np.float32)), what
        got = float(cr.to_numpy()[0])
        assert abs(got - oracle_mod.reduce("sum", x)) <= 1e-5 * oracle_mod.abs_sum(x), what
        assert np.array_equal(cso.to_numpy(), oracle_mod.scan(s, "inclusive", "sum")), what
        ref, mag = oracle_mod.mapoverlap1d(z, w, 2)
        assert np.all(np.abs(co.to_numpy().astype(np.float64) - ref) <= 1e-6 * mag + 1e-30), what

    arrs = put(0)
    with torch.cuda.stream(main):
        fork()  # eager; also sizes every stream's workspace outside the capture
    check(arrs, "eager")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=main):
        fork()
    torch.cuda.synchronize()
    for rep in range(1, 4):
        arrs = put(2 * rep)
        with torch.cuda.stream(main):
            fork()
        check(arrs, f"eager round {rep}")
        arrs = put(2 * rep + 1)
        with torch.cuda.stream(main):
            g.replay()
        for c in (cm, cr, cso, co):
            c.mark_device_written(main)
        check(arrs, f"replay {rep}")
    skel.skel_sync()


def test_gaussian_stencil_4096(skel, oracle_mod):
    H = W = 4096
    x = si.uniform_f32(H * W, 0.0, 1.0, 1, 0).reshape(H, W)
    g = si.gaussian_weights(4, 2.0)
    ref, mag = oracle_mod.mapoverlap2d(x, 4, 4, wy=g, wx=g)
    cx = skel.Container.from_numpy(x)
    for v in (skel.VARIANT_AUTO, 0, 1, 2, 3):
        out = skel.Container.empty(skel.F32, H, W)
        skel.skel_mapoverlap2d(cx, out, wy=g, wx=g, edge=skel.EDGE_CLAMP, variant=v)
        got = out.to_numpy().astype(np.float64)
        bad = np.abs(got - ref) > 1e-6 * mag
        assert not bad.any(), (v, np.argwhere(bad)[:5])
    skel.skel_sync()


def test_dot_2_26(skel, oracle_mod):
    n = 1 << 26
    x = si.normal_f32(n, 1, 0)
    y = si.normal_f32(n, 1, 1)
    ref, mag = oracle_mod.mapreduce("mul", None, x, y)
    cx, cy = skel.Container.from_numpy(x), skel.Container.from_numpy(y)
    for v in (skel.VARIANT_AUTO, 0, 1, 2, 3):
        out = skel.Container.empty(skel.F32, 1)
        skel.skel_mapreduce(skel.MAP_MUL, None, [cx, cy], skel.SUM, out, variant=v)
        got = float(out.to_numpy()[0])
        assert abs(got - ref) <= 1e-5 * mag, (v, got, ref, mag)
    skel.skel_sync()


def test_exclusive_scan_2_27(skel, oracle_mod):
    n = 1 << 27
    x = si.int_uniform_i32(n, 1000, 1, 2)
    ref = oracle_mod.scan(x, "exclusive", "sum", np.int64)
    assert ref[-1] > 2 ** 31  # the widening matters at this size
    cx = skel.Container.from_numpy(x)
    for v in (skel.VARIANT_AUTO, 1, 2):
        out = skel.Container.empty(skel.I64, n)
        skel.skel_scan(cx, out, skel.EXCLUSIVE, skel.SUM, variant=v)
        got = out.to_numpy()
        assert np.array_equal(got, ref), (v, np.flatnonzero(got != ref)[:5])
        del out, got
    skel.skel_sync()
