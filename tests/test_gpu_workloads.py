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
