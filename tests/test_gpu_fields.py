"""GPU parity of the batched-field 2D MapOverlap and its transpose: every
field of a (fields * H) x W container is mapped on its own, so each field must
match the oracle's single-image result, for every variant and edge rule.

Bars as the single-image calls: |y - y*| <= 1e-6 * sum of |terms| per pixel."""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

EDGES = {"clamp": 0, "const": 1, "cyclic": 2}
SHAPES = [(3, 37, 45), (5, 64, 64), (2, 1, 9), (4, 130, 7)]


def weights(sep, r, seed):
    wy = si.uniform_f32(2 * r + 1, -1.0, 1.0, 22, seed)
    wx = si.uniform_f32(2 * r + 1, -1.0, 1.0, 22, seed + 1)
    if sep:
        return {"wy": wy, "wx": wx}
    return {"w2d": si.uniform_f32((2 * r + 1) ** 2, -1.0, 1.0, 22, seed + 2)
            .reshape(2 * r + 1, 2 * r + 1)}


@pytest.mark.parametrize("edge", list(EDGES))
@pytest.mark.parametrize("sep", [False, True])
@pytest.mark.parametrize("r", [1, 4])
def test_fields_forward_and_backward(skel, oracle_mod, edge, sep, r):
    w = weights(sep, r, 10 * r + sep)
    for f, h, wd in SHAPES:
        x = si.uniform_f32(f * h * wd, -1.0, 1.0, 22, f * 1000 + h).reshape(f * h, wd)
        cx = skel.Container.from_numpy(x)
        for v in range(skel.skel_variant_count(skel.SK_MAPOVERLAP2D)):
            name = skel.skel_variant_name(skel.SK_MAPOVERLAP2D, v)
            if not sep and "separable" in name:
                continue
            out = skel.Container.empty(skel.F32, f * h, wd)
            skel.skel_mapoverlap2d_fields(cx, out, f, edge=EDGES[edge], pad=0.25, variant=v,
                                          **w)
            got = out.to_numpy().reshape(f, h, wd)
            for k in range(f):
                ref, mag = oracle_mod.mapoverlap2d(x[k * h:(k + 1) * h], r, r, edge=edge,
                                                   pad=0.25, **w)
                bad = np.abs(got[k] - ref) > 1e-6 * mag + 1e-30
                assert not bad.any(), (edge, sep, r, (f, h, wd), name, k, np.argwhere(bad)[:3])
        for v in range(skel.skel_variant_count(skel.SK_MAPOVERLAP2D_BACKWARD)):
            out = skel.Container.empty(skel.F32, f * h, wd)
            skel.skel_mapoverlap2d_fields_backward(cx, out, f, edge=EDGES[edge], variant=v, **w)
            got = out.to_numpy().reshape(f, h, wd)
            for k in range(f):
                ref, mag = oracle_mod.mapoverlap2d_adjoint(x[k * h:(k + 1) * h], r, r,
                                                           edge=edge, **w)
                bad = np.abs(got[k] - ref) > 1e-6 * mag + 1e-30
                assert not bad.any(), (edge, sep, r, (f, h, wd), "adjoint", v, k,
                                       np.argwhere(bad)[:3])
    skel.skel_sync()


def test_fields_beyond_one_launch(skel, oracle_mod):
    # more fields than one launch's grid holds (65535): the launcher splits them
    f, h, wd = 70001, 2, 4
    x = si.uniform_f32(f * h * wd, -1.0, 1.0, 22, 99).reshape(f * h, wd)
    w = si.five_point_weights(0.5, 0.1, 0.2, 0.05, 0.15)
    cx = skel.Container.from_numpy(x)
    out = skel.Container.empty(skel.F32, f * h, wd)
    skel.skel_mapoverlap2d_fields(cx, out, f, w2d=w, edge=skel.EDGE_CLAMP)
    got = out.to_numpy().reshape(f, h, wd)
    back = skel.Container.empty(skel.F32, f * h, wd)
    skel.skel_mapoverlap2d_fields_backward(cx, back, f, w2d=w, edge=skel.EDGE_CLAMP)
    gb = back.to_numpy().reshape(f, h, wd)
    for k in (0, 1, 65534, 65535, 65536, f - 1):
        xf = x[k * h:(k + 1) * h]
        ref, mag = oracle_mod.mapoverlap2d(xf, 1, 1, w2d=w, edge="clamp")
        assert np.all(np.abs(got[k] - ref) <= 1e-6 * mag + 1e-30), k
        ref, mag = oracle_mod.mapoverlap2d_adjoint(xf, 1, 1, w2d=w, edge="clamp")
        assert np.all(np.abs(gb[k] - ref) <= 1e-6 * mag + 1e-30), k
    skel.skel_sync()


def test_fields_shape_errors(skel):
    x = skel.Container.from_numpy(np.zeros((10, 8), np.float32))
    out = skel.Container.empty(skel.F32, 10, 8)
    w = np.ones((3, 3), np.float32)
    for bad in (3, 0, -1):  # 3 does not divide 10 rows
        with pytest.raises(skel.SkelError) as e:
            skel.skel_mapoverlap2d_fields(x, out, bad, w2d=w)
        assert e.value.status == skel.E_SHAPE
        with pytest.raises(skel.SkelError) as e:
            skel.skel_mapoverlap2d_fields_backward(x, out, bad, w2d=w)
        assert e.value.status == skel.E_SHAPE
    skel.skel_mapoverlap2d_fields(x, out, 10, w2d=w)  # ten 1 x 8 fields
    skel.skel_sync()


from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402


@settings(max_examples=60, deadline=None, suppress_health_check=list(HealthCheck))
@given(f=st.integers(1, 5), h=st.integers(1, 40), wd=st.integers(1, 40), ry=st.integers(0, 3),
       rx=st.integers(0, 3), edge=st.sampled_from(list(EDGES)), sep=st.booleans(),
       seed=st.integers(0, 1000))
def test_fields_drawn_shapes(skel, oracle_mod, f, h, wd, ry, rx, edge, sep, seed):
    x = si.uniform_f32(f * h * wd, -1.0, 1.0, 24, seed).reshape(f * h, wd)
    wy = si.uniform_f32(2 * ry + 1, -1.0, 1.0, 24, 2000 + seed)
    wx = si.uniform_f32(2 * rx + 1, -1.0, 1.0, 24, 3000 + seed)
    w = {"wy": wy, "wx": wx} if sep else {"w2d": np.outer(wy, wx).astype(np.float32)}
    cx = skel.Container.from_numpy(x)
    out = skel.Container.empty(skel.F32, f * h, wd)
    skel.skel_mapoverlap2d_fields(cx, out, f, edge=EDGES[edge], pad=0.5, **w)
    back = skel.Container.empty(skel.F32, f * h, wd)
    skel.skel_mapoverlap2d_fields_backward(cx, back, f, edge=EDGES[edge], **w)
    got, gb = out.to_numpy().reshape(f, h, wd), back.to_numpy().reshape(f, h, wd)
    for k in range(f):
        xf = x[k * h:(k + 1) * h]
        ref, mag = oracle_mod.mapoverlap2d(xf, ry, rx, edge=edge, pad=0.5, **w)
        assert np.all(np.abs(got[k] - ref) <= 1e-6 * mag + 1e-30), k
        ref, mag = oracle_mod.mapoverlap2d_adjoint(xf, ry, rx, edge=edge, **w)
        assert np.all(np.abs(gb[k] - ref) <= 1e-6 * mag + 1e-30), k
