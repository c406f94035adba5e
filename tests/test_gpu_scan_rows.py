"""GPU parity of the row-wise Scan (every row of a matrix scanned on its own)
against the oracle, through the C ABI, for both variants.

Bars as the flat Scan: integers bit-exact; float32 sums within
|y - y*| <= 1e-5 * (sum of |x| over the terms), float32 min/max exact.
"""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

RED_OPS = {"sum": 0, "min": 1, "max": 2}
KINDS = {"inclusive": 0, "exclusive": 1, "reverse_inclusive": 2, "reverse_exclusive": 3}
# widths around the one-wavefront chunk (2048), odd widths (element accesses),
# a long row (several chunks) and many short rows
SHAPES = [(1, 1), (3, 5), (7, 64), (5, 2048), (4, 2049), (2, 5000), (300, 7), (65, 4096),
          (2, (1 << 17) + 3), (1, 1 << 17)]
SR0, SR1 = 0, 1


def aligned(cols, in_size, out_size):
    return (cols * in_size) % 16 == 0 and (cols * out_size) % 16 == 0


def ints(g, shape, din):
    if din == np.int32:
        return g.integers(-2 ** 31, 2 ** 31, shape, dtype=np.int64).astype(np.int32)
    return g.integers(-2 ** 62, 2 ** 62, shape, dtype=np.int64)


@pytest.mark.parametrize("pair", ["i32_i32", "i32_i64", "i64_i64"])
@pytest.mark.parametrize("op", list(RED_OPS))
def test_scan_rows_int_bit_exact(skel, oracle_mod, pair, op):
    din, dout, sk_in, sk_out = {"i32_i32": (np.int32, np.int32, skel.I32, skel.I32),
                                "i32_i64": (np.int32, np.int64, skel.I32, skel.I64),
                                "i64_i64": (np.int64, np.int64, skel.I64, skel.I64)}[pair]
    for shape in SHAPES:
        x = ints(si.rng(21, shape[0] * 7919 + shape[1]), shape, din)
        cx = skel.Container.from_numpy(x)
        vs = [SR1] + ([SR0] if aligned(shape[1], x.itemsize, np.dtype(dout).itemsize) else [])
        for kind, code in KINDS.items():
            ref = oracle_mod.scan_rows(x, kind, op, dout)
            for v in vs:
                out = skel.Container.empty(sk_out, *shape)
                skel.skel_scan_rows(cx, out, code, RED_OPS[op], variant=v)
                got = out.to_numpy().reshape(shape)
                assert np.array_equal(got, ref), (pair, op, shape, kind, v,
                                                  np.argwhere(got != ref)[:5])
    skel.skel_sync()


@pytest.mark.parametrize("op", list(RED_OPS))
def test_scan_rows_f32(skel, oracle_mod, op):
    for shape in SHAPES:
        x = si.normal_f32(shape[0] * shape[1], 21, shape[1]).reshape(shape)
        cx = skel.Container.from_numpy(x)
        vs = [SR1] + ([SR0] if shape[1] % 4 == 0 else [])
        for kind, code in KINDS.items():
            ref, mag = oracle_mod.scan_rows(x, kind, op)
            for v in vs:
                out = skel.Container.empty(skel.F32, *shape)
                skel.skel_scan_rows(cx, out, code, RED_OPS[op], variant=v)
                got = out.to_numpy().reshape(shape).astype(np.float64)
                bad = np.abs(got - ref) > 1e-5 * mag + 1e-30 if op == "sum" else got != ref
                assert not bad.any(), (op, shape, kind, v, np.argwhere(bad)[:5])
    skel.skel_sync()


def test_scan_rows_in_place_and_errors(skel, oracle_mod):
    for shape in [(9, 2048), (9, 2047)]:
        x = si.int_uniform_i32(shape[0] * shape[1], 100, 21, 3).reshape(shape)
        c = skel.Container.from_numpy(x)
        skel.skel_scan_rows(c, c, skel.INCLUSIVE, skel.SUM)  # in place
        assert np.array_equal(c.to_numpy().reshape(shape), oracle_mod.scan_rows(x))
    # the per-row single-pass form needs 16-byte aligned rows
    x = np.ones((3, 6), np.int32)
    out = skel.Container.empty(skel.I64, 3, 6)
    with pytest.raises(skel.SkelError) as e:
        skel.skel_scan_rows(skel.Container.from_numpy(x), out, skel.INCLUSIVE, skel.SUM,
                            variant=SR0)
    assert e.value.status == skel.E_UNSUPPORTED
    with pytest.raises(skel.SkelError) as e:
        skel.skel_scan_rows(skel.Container.from_numpy(x), skel.Container.empty(skel.I64, 2, 9),
                            skel.INCLUSIVE, skel.SUM)
    assert e.value.status == skel.E_SHAPE
    skel.skel_sync()


def test_scan_rows_many_rows(skel, oracle_mod):
    # the field layout of the batched layer: many rows of 2048, widening
    shape = (8192, 2048)
    x = si.int_uniform_i32(shape[0] * shape[1], 1000, 21, 4).reshape(shape)
    cx = skel.Container.from_numpy(x)
    for kind in ("exclusive", "reverse_inclusive"):
        ref = oracle_mod.scan_rows(x, kind, "sum", np.int64)
        for v in (SR0, SR1):
            out = skel.Container.empty(skel.I64, *shape)
            skel.skel_scan_rows(cx, out, KINDS[kind], skel.SUM, variant=v)
            assert np.array_equal(out.to_numpy().reshape(shape), ref), (kind, v)
    skel.skel_sync()


def test_scan_rows_more_rows_than_one_grid(skel, oracle_mod):
    # the kernels step over rows in a grid of at most 2^20 workgroups; sampled
    # rows around that stride are checked against the oracle one by one
    for cols in (3, 4):  # element accesses, then 16-byte vectors
        rows = (1 << 20) + 5
        x = si.int_uniform_i32(rows * cols, 1000, 21, 5 + cols).reshape(rows, cols)
        out = skel.Container.empty(skel.I64, rows, cols)
        skel.skel_scan_rows(skel.Container.from_numpy(x), out, skel.EXCLUSIVE, skel.SUM,
                            variant=SR1)
        got = out.to_numpy().reshape(rows, cols)
        for r in (0, 1, (1 << 20) - 1, 1 << 20, (1 << 20) + 1, rows - 1):
            assert np.array_equal(got[r], oracle_mod.scan(x[r], "exclusive", "sum", np.int64)), \
                (cols, r)
    skel.skel_sync()



from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402


@settings(max_examples=60, deadline=None, suppress_health_check=list(HealthCheck))
@given(rows=st.integers(1, 40), cols=st.integers(1, 5000),
       pair=st.sampled_from(["i32_i32", "i32_i64", "i64_i64"]),
       kind=st.sampled_from(list(KINDS)), op=st.sampled_from(list(RED_OPS)),
       variant=st.sampled_from([SR0, SR1]), seed=st.integers(0, 1000))
def test_scan_rows_drawn_shapes(skel, oracle_mod, rows, cols, pair, kind, op, variant, seed):
    din, dout, sk_out = {"i32_i32": (np.int32, np.int32, skel.I32),
                         "i32_i64": (np.int32, np.int64, skel.I64),
                         "i64_i64": (np.int64, np.int64, skel.I64)}[pair]
    if variant == SR0 and not aligned(cols, np.dtype(din).itemsize, np.dtype(dout).itemsize):
        variant = SR1
    x = ints(si.rng(23, seed), (rows, cols), din)
    out = skel.Container.empty(sk_out, rows, cols)
    skel.skel_scan_rows(skel.Container.from_numpy(x), out, KINDS[kind], RED_OPS[op],
                        variant=variant)
    assert np.array_equal(out.to_numpy().reshape(rows, cols),
                          oracle_mod.scan_rows(x, kind, op, dout))
