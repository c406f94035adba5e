"""GPU parity: every skeleton variant of libskel against the CPU oracle on the
same seeded inputs, called through the C ABI (via the ctypes binding).

Bars (stated per skeleton in the oracle's definitions):
  * integer Reduce / Scan: bit-exact (wrapping in the output width);
  * Map: |y - y*| <= 1e-6 * (magnitude of the terms of f);
  * Reduce / MapReduce (floating point): |r - r*| <= 1e-5 * sum |terms|;
  * MapOverlap: |y - y*| <= 1e-6 * sum_k |w_k x_k| per output;
  * floating-point Scan: |y_i - y*_i| <= 1e-5 * sum_{j<=i} |x_j|;
  * MIN / MAX: exact.
Sizes span several tiles, ragged tails, empty and one-element inputs.
"""
import math

import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 3, 4, 5, 63, 64, 65, 255, 1000, 4095, 4096, 4097, 65537, (1 << 20) + 3]
MAP_OPS = {"identity": 0, "axpy": 1, "affine": 2, "tanh": 3, "affine_tanh": 4, "mul": 5,
           "square": 6}
RED_OPS = {"sum": 0, "min": 1, "max": 2}
EDGES = {"clamp": 0, "const": 1, "cyclic": 2}


def variants(skel, sk):
    return list(range(skel.skel_variant_count(sk)))


def cont(skel, arr, dtype=None):
    return skel.Container.from_numpy(arr, dtype)


def scalar_out(skel, dtype):
    return skel.Container.empty(dtype, 1)


# ----------------------------------------------------------------------- Map
def map_mag(op, p, x, y):
    """Magnitude scale of f's terms, the reference for the 1e-6 bound."""
    x = np.abs(x.astype(np.float64))
    y = np.abs(y.astype(np.float64)) if y is not None else 0
    if op == "identity":
        return x
    if op == "axpy":
        return abs(p[0]) * x + y
    if op == "affine":
        return abs(p[0]) * x + abs(p[1])
    if op == "tanh":
        return np.maximum(1, x)
    if op == "affine_tanh":
        return np.maximum(1, abs(p[0]) * x + abs(p[1]))
    if op == "mul":
        return x * y
    return x * x


@pytest.mark.parametrize("op", list(MAP_OPS))
def test_map(skel, oracle_mod, op):
    params = {"axpy": [2.5], "affine": [-1.5, 0.25], "affine_tanh": [0.75, -0.5]}.get(op, [])
    two = op in oracle_mod.TWO_INPUT_MAP_OPS
    for n in SIZES:
        x = si.uniform_f32(n, -1.0, 1.0, 0, 0) * np.float32(3)
        y = si.uniform_f32(n, -1.0, 1.0, 0, 1) if two else None
        ref = oracle_mod.map_f32(op, [np.float32(p) for p in params], x, y)
        tol = 1e-6 * map_mag(op, params, x, y) + 1e-30
        for v in variants(skel, skel.SK_MAP):
            cx = cont(skel, x)
            out = skel.Container.empty(skel.F32, n)
            ins = [cx, cont(skel, y)] if two else [cx]
            skel.skel_map(MAP_OPS[op], params, ins, out, variant=v)
            got = out.to_numpy().astype(np.float64)
            bad = np.abs(got - ref) > tol
            assert not bad.any(), (op, n, v, np.flatnonzero(bad)[:5])


def test_map_saxpy_bit_exact_and_in_place(skel, oracle_mod):
    # x, y on the 2^-23 grid: 2.5x + y is exact in binary64, so the fused
    # multiply-add's single rounding gives exactly fp32(oracle)
    n = (1 << 20) + 7
    x = si.uniform_f32(n, -1.0, 1.0, 0, 0)
    y = si.uniform_f32(n, -1.0, 1.0, 0, 1)
    want = oracle_mod.map_f32("axpy", [2.5], x, y).astype(np.float32)
    for v in variants(skel, skel.SK_MAP):
        cx, cy = cont(skel, x), cont(skel, y)
        skel.skel_map(skel.MAP_AXPY, [2.5], [cx, cy], cy, variant=v)  # in place
        assert np.array_equal(cy.to_numpy(), want), v


# -------------------------------------------------------------------- Reduce
def check_fp(got, ref, mag, rel=1e-5):
    assert abs(float(got) - ref) <= rel * mag + 1e-30, (got, ref, mag)


@pytest.mark.parametrize("op", list(RED_OPS))
def test_reduce_f32(skel, oracle_mod, op):
    for n in SIZES:
        x = si.normal_f32(n, 1, 2)
        ref = oracle_mod.reduce(op, x)
        mag = oracle_mod.abs_sum(x)
        for v in variants(skel, skel.SK_REDUCE):
            if v in (3, 4, 5) and op != "sum":  # atomic, compensated, pairwise: sums only
                with pytest.raises(skel.SkelError) as e:
                    skel.skel_reduce(RED_OPS[op], cont(skel, x), scalar_out(skel, skel.F32),
                                     variant=v)
                assert e.value.status == skel.E_UNSUPPORTED
                continue
            out = scalar_out(skel, skel.F32)
            skel.skel_reduce(RED_OPS[op], cont(skel, x), out, variant=v)
            got = out.to_numpy()[0]
            if op == "sum":
                check_fp(got, ref, mag)
            else:
                assert float(got) == ref, (op, n, v)


@pytest.mark.parametrize("n", [1, 64, 65536, 1 << 20, 1 << 24])
def test_reduce_sum_of_indices(skel, n):
    # sum_{i<n} i = n(n-1)/2; binary32 holds every i exactly for n <= 2^24
    exact = n * (n - 1) // 2
    xi = np.arange(n, dtype=np.int32)
    for v in variants(skel, skel.SK_REDUCE):
        if v not in (4, 5):  # compensated and pairwise: floating point only
            o32, o64 = scalar_out(skel, skel.I32), scalar_out(skel, skel.I64)
            skel.skel_reduce(skel.SUM, cont(skel, xi), o32, variant=v)
            skel.skel_reduce(skel.SUM, cont(skel, xi), o64, variant=v)
            assert int(o64.to_numpy()[0]) == exact
            assert int(o32.to_numpy()[0]) == ((exact + 2 ** 31) % 2 ** 32) - 2 ** 31
        of = scalar_out(skel, skel.F32)
        skel.skel_reduce(skel.SUM, cont(skel, xi.astype(np.float32)), of, variant=v)
        assert abs(float(of.to_numpy()[0]) - exact) <= 1e-5 * exact


@pytest.mark.parametrize("pair", ["i32_i32", "i32_i64", "i64_i64"])
@pytest.mark.parametrize("op", list(RED_OPS))
def test_reduce_int_bit_exact(skel, oracle_mod, pair, op):
    din, dout = {"i32_i32": (skel.I32, skel.I32), "i32_i64": (skel.I32, skel.I64),
                 "i64_i64": (skel.I64, skel.I64)}[pair]
    for n in SIZES:
        g = si.rng(7, n)
        if din == skel.I32:
            x = g.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
        else:
            x = g.integers(-2 ** 62, 2 ** 62, n, dtype=np.int64)
        ref = oracle_mod.reduce(op, x, np.int64 if dout == skel.I64 else np.int32)
        for v in variants(skel, skel.SK_REDUCE):
            out = scalar_out(skel, dout)
            if v in (4, 5):
                with pytest.raises(skel.SkelError) as e:
                    skel.skel_reduce(RED_OPS[op], cont(skel, x), out, variant=v)
                assert e.value.status == skel.E_UNSUPPORTED
                continue
            skel.skel_reduce(RED_OPS[op], cont(skel, x), out, variant=v)
            assert int(out.to_numpy()[0]) == ref, (pair, op, n, v)


def test_reduce_deterministic_variants(skel):
    x = si.normal_f32((1 << 22) + 11, 1, 9)
    for v in (0, 1, 2, 4, 5):
        vals = set()
        for _ in range(3):
            out = scalar_out(skel, skel.F32)
            skel.skel_reduce(skel.SUM, cont(skel, x), out, variant=v)
            vals.add(out.to_numpy()[0].tobytes())
        assert len(vals) == 1, v


# ----------------------------------------------------------------- MapReduce
@pytest.mark.parametrize("mop", ["mul", "square", "identity", "axpy", "affine_tanh"])
@pytest.mark.parametrize("op", list(RED_OPS))
def test_mapreduce_f32(skel, oracle_mod, mop, op):
    params = {"axpy": [2.5], "affine_tanh": [0.5, 0.125]}.get(mop, [])
    two = mop in oracle_mod.TWO_INPUT_MAP_OPS
    for n in SIZES:
        x = si.normal_f32(n, 1, 0)
        y = si.normal_f32(n, 1, 1) if two else None
        ref, mag = oracle_mod.mapreduce(mop, params, x, y, op)
        if op != "sum":
            # min/max of f32 element results: compare with the f32-rounded values
            vals = oracle_mod.map_f32(mop, params, x, y)
            tol = 1e-6 * (np.max(map_mag(mop, params, x, y)) if n else 0)
        for v in variants(skel, skel.SK_MAPREDUCE):
            out = scalar_out(skel, skel.F32)
            ins = [cont(skel, x), cont(skel, y)] if two else [cont(skel, x)]
            if v in (4, 5) and op != "sum":  # compensated, pairwise: sums only
                with pytest.raises(skel.SkelError) as e:
                    skel.skel_mapreduce(MAP_OPS[mop], params, ins, RED_OPS[op], out,
                                        variant=v)
                assert e.value.status == skel.E_UNSUPPORTED
                continue
            skel.skel_mapreduce(MAP_OPS[mop], params, ins, RED_OPS[op], out, variant=v)
            got = float(out.to_numpy()[0])
            if op == "sum":
                check_fp(got, ref, mag)
            elif n == 0:
                assert got == ref
            else:
                assert abs(got - ref) <= tol + 1e-30, (mop, op, n, v, got, ref)


def test_mapreduce_bf16_inputs(skel, oracle_mod):
    for n in (0, 1, 7, 8, 9, 4097, (1 << 20) + 5):
        xb = si.log_uniform_signed_bf16(n, config=4, index=1)
        yb = si.log_uniform_signed_bf16(n, config=4, index=2)
        xf, yf = si.bf16_bits_to_f32(xb), si.bf16_bits_to_f32(yb)
        ref, mag = oracle_mod.mapreduce("mul", None, xf, yf)
        rsum = oracle_mod.reduce("sum", xf)
        asum = oracle_mod.abs_sum(xf)
        for v in (1, 2, 3, 4, 5):
            out = scalar_out(skel, skel.F32)
            skel.skel_mapreduce(skel.MAP_MUL, None, [cont(skel, xb, skel.BF16),
                                                     cont(skel, yb, skel.BF16)],
                                skel.SUM, out, variant=v)
            check_fp(out.to_numpy()[0], ref, mag)
        for v in variants(skel, skel.SK_REDUCE):
            out = scalar_out(skel, skel.F32)
            skel.skel_reduce(skel.SUM, cont(skel, xb, skel.BF16), out, variant=v)
            check_fp(out.to_numpy()[0], rsum, asum)
        with pytest.raises(skel.SkelError):  # the unfused form maps in f32 only
            skel.skel_mapreduce(skel.MAP_MUL, None, [cont(skel, xb, skel.BF16),
                                                     cont(skel, yb, skel.BF16)],
                                skel.SUM, scalar_out(skel, skel.F32), variant=0)


def test_mapreduce_identities(skel, oracle_mod):
    n = (1 << 20) + 1
    x = si.normal_f32(n, 1, 3)
    e = np.zeros(n, np.float32)
    e[12345] = 1
    out = scalar_out(skel, skel.F32)
    skel.skel_mapreduce(skel.MAP_MUL, None, [cont(skel, e), cont(skel, x)], skel.SUM, out)
    assert out.to_numpy()[0] == x[12345]
    out2 = scalar_out(skel, skel.F32)
    skel.skel_mapreduce(skel.MAP_MUL, None, [cont(skel, x), cont(skel, np.ones_like(x))],
                        skel.SUM, out2)
    check_fp(out2.to_numpy()[0], oracle_mod.reduce("sum", x), oracle_mod.abs_sum(x))


# ---------------------------------------------------------------- MapOverlap
@pytest.mark.parametrize("edge", list(EDGES))
@pytest.mark.parametrize("r", [0, 1, 2, 4, 7])
def test_mapoverlap1d(skel, oracle_mod, edge, r):
    w = si.uniform_f32(2 * r + 1, -1.0, 1.0, 3, r)
    for n in (1, 2, 5, 17, 1000, 1023, 1024, 1025, 4099, (1 << 20) + 2):
        x = si.uniform_f32(n, -1.0, 1.0, 0, 3)
        ref, mag = oracle_mod.mapoverlap1d(x, w, r, edge, 0.625)
        for v in variants(skel, skel.SK_MAPOVERLAP1D):
            out = skel.Container.empty(skel.F32, n)
            if v == 2 and r > 4:  # cross-lane variant reaches 4 neighbours per side
                with pytest.raises(skel.SkelError) as e:
                    skel.skel_mapoverlap1d(cont(skel, x), out, w, r, EDGES[edge], 0.625,
                                           variant=v)
                assert e.value.status == skel.E_UNSUPPORTED
                continue
            skel.skel_mapoverlap1d(cont(skel, x), out, w, r, EDGES[edge], 0.625, variant=v)
            got = out.to_numpy().astype(np.float64)
            bad = np.abs(got - ref) > 1e-6 * mag + 1e-30
            assert not bad.any(), (edge, r, n, v, np.flatnonzero(bad)[:5])


SHAPES_2D = [(1, 1), (1, 17), (13, 1), (3, 5), (64, 64), (65, 63), (100, 130), (257, 300)]
RADII_2D = [(4, 4), (1, 1), (2, 2), (3, 1), (0, 2), (8, 8)]


@pytest.mark.parametrize("edge", list(EDGES))
@pytest.mark.parametrize("ry,rx", RADII_2D)
def test_mapoverlap2d(skel, oracle_mod, edge, ry, rx):
    wy = si.uniform_f32(2 * ry + 1, 0.0, 1.0, 3, 10 + ry)
    wx = si.uniform_f32(2 * rx + 1, -1.0, 1.0, 3, 20 + rx)
    w2d = si.uniform_f32((2 * ry + 1) * (2 * rx + 1), -1.0, 1.0, 3, 30).reshape(
        2 * ry + 1, 2 * rx + 1)
    for shape in SHAPES_2D:
        x = si.uniform_f32(shape[0] * shape[1], 0.0, 1.0, 1, shape[0]).reshape(shape)
        for sep in (True, False):
            kw = dict(wy=wy, wx=wx) if sep else dict(w2d=w2d)
            ref, mag = oracle_mod.mapoverlap2d(x, ry, rx, edge=edge, pad=-0.25, **kw)
            for v in variants(skel, skel.SK_MAPOVERLAP2D):
                if v in (2, 3) and not sep:  # separable variants
                    continue
                if v == 4 and max(ry, rx) > 4:  # marching window: radii up to 4
                    continue
                out = skel.Container.empty(skel.F32, shape[0], shape[1])
                skel.skel_mapoverlap2d(cont(skel, x), out, ry=ry, rx=rx, edge=EDGES[edge],
                                       pad=-0.25, variant=v, **kw)
                got = out.to_numpy().reshape(shape).astype(np.float64)
                bad = np.abs(got - ref) > 1e-6 * mag + 1e-30
                assert not bad.any(), (edge, ry, rx, shape, sep, v, np.argwhere(bad)[:5])


# The marching-window variant's straight-line path runs for whole 256-column
# strips of images with at least 4 rows: rows beyond the image ends and the
# chunks beyond a row's two ends are mapped by the edge rule without branches.
# These shapes put strips at both row ends (widths that are multiples of 256),
# a ragged last strip (260, 772), images of 4 and 5 rows (rows wrapped or
# clamped up to 4 away) and strips that end mid-strip in height.
MARCH_SHAPES = [(4, 256), (5, 512), (37, 768), (70, 1024), (20, 260), (9, 772)]
MARCH_RADII = [(1, 1), (2, 2), (4, 4), (3, 1), (0, 2), (4, 0)]


@pytest.mark.parametrize("edge", list(EDGES))
@pytest.mark.parametrize("ry,rx", MARCH_RADII)
def test_mapoverlap2d_march_paths(skel, oracle_mod, edge, ry, rx):
    v = skel.variant_index(skel.SK_MAPOVERLAP2D, "O2e_march")
    wy = si.uniform_f32(2 * ry + 1, -1.0, 1.0, 41, 10 + ry)
    wx = si.uniform_f32(2 * rx + 1, -1.0, 1.0, 41, 20 + rx)
    w2d = si.uniform_f32((2 * ry + 1) * (2 * rx + 1), -1.0, 1.0, 41, 30).reshape(
        2 * ry + 1, 2 * rx + 1)
    for shape in MARCH_SHAPES:
        x = si.uniform_f32(shape[0] * shape[1], -1.0, 1.0, 42, shape[1]).reshape(shape)
        for kw in (dict(w2d=w2d), dict(wy=wy, wx=wx)):
            ref, mag = oracle_mod.mapoverlap2d(x, ry, rx, edge=edge, pad=0.625, **kw)
            out = skel.Container.empty(skel.F32, shape[0], shape[1])
            skel.skel_mapoverlap2d(cont(skel, x), out, ry=ry, rx=rx, edge=EDGES[edge],
                                   pad=0.625, variant=v, **kw)
            got = out.to_numpy().reshape(shape).astype(np.float64)
            bad = np.abs(got - ref) > 1e-6 * mag + 1e-30
            assert not bad.any(), (edge, ry, rx, shape, list(kw), np.argwhere(bad)[:5])


def test_mapoverlap_constant_field_and_impulse(skel):
    g = si.gaussian_weights(4, 2.0)
    sw = math.fsum(float(v) for v in g)
    c = np.float32(0.75)
    x = np.full((129, 257), c, np.float32)
    for v in variants(skel, skel.SK_MAPOVERLAP2D):
        out = skel.Container.empty(skel.F32, 129, 257)
        skel.skel_mapoverlap2d(cont(skel, x), out, wy=g, wx=g, variant=v)
        got = out.to_numpy().astype(np.float64)
        assert np.all(np.abs(got - float(c) * sw * sw) <= 1e-6), v
    # impulse: the response is W flipped in both axes (correlation orientation)
    w = np.arange(1, 16, dtype=np.float32).reshape(3, 5)
    x = np.zeros((9, 11), np.float32)
    x[4, 5] = 1
    for v in (0, 1):
        out = skel.Container.empty(skel.F32, 9, 11)
        skel.skel_mapoverlap2d(cont(skel, x), out, w2d=w, variant=v)
        got = out.to_numpy()
        assert np.array_equal(got[3:6, 3:8], w[::-1, ::-1]), v
        assert np.count_nonzero(got) == 15


# ---------------------------------------------------------------------- Scan
# tiles are 32768 elements for 4-byte inputs and 16384 for 8-byte inputs
SCAN_SIZES = [0, 1, 2, 63, 64, 65, 2047, 2049, 8193, 16383, 16384, 16385, 32767, 32768,
              32769, 3 * 32768 + 5, 70000, (1 << 20) + 3]


@pytest.mark.parametrize("pair", ["i32_i32", "i32_i64", "i64_i64"])
@pytest.mark.parametrize("kind", ["inclusive", "exclusive"])
@pytest.mark.parametrize("op", list(RED_OPS))
def test_scan_int_bit_exact(skel, oracle_mod, pair, kind, op):
    din, dout = {"i32_i32": (skel.I32, skel.I32), "i32_i64": (skel.I32, skel.I64),
                 "i64_i64": (skel.I64, skel.I64)}[pair]
    K = {"inclusive": skel.INCLUSIVE, "exclusive": skel.EXCLUSIVE}[kind]
    for n in SCAN_SIZES:
        g = si.rng(8, n)
        if din == skel.I32:
            x = g.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
        else:
            x = g.integers(-2 ** 62, 2 ** 62, n, dtype=np.int64)
        ref = oracle_mod.scan(x, kind, op, np.int64 if dout == skel.I64 else np.int32)
        for v in variants(skel, skel.SK_SCAN):
            out = skel.Container.empty(dout, n)
            skel.skel_scan(cont(skel, x), out, K, RED_OPS[op], variant=v)
            got = out.to_numpy()
            assert np.array_equal(got, ref), (pair, kind, op, n, v,
                                              np.flatnonzero(got != ref)[:5])
    skel.skel_sync()


@pytest.mark.parametrize("kind", ["inclusive", "exclusive"])
@pytest.mark.parametrize("op", list(RED_OPS))
def test_scan_f32(skel, oracle_mod, kind, op):
    K = {"inclusive": skel.INCLUSIVE, "exclusive": skel.EXCLUSIVE}[kind]
    for n in SCAN_SIZES:
        x = si.normal_f32(n, 3, 1)
        ref, mag = oracle_mod.scan(x, kind, op)
        for v in variants(skel, skel.SK_SCAN):
            out = skel.Container.empty(skel.F32, n)
            skel.skel_scan(cont(skel, x), out, K, RED_OPS[op], variant=v)
            got = out.to_numpy().astype(np.float64)
            if op == "sum":
                bad = np.abs(got - ref) > 1e-5 * mag + 1e-30
            else:
                bad = got != ref
            assert not bad.any(), (kind, op, n, v, np.flatnonzero(bad)[:5])
    skel.skel_sync()


def test_scan_in_place_and_closed_forms(skel, oracle_mod):
    n = (1 << 20) + 9
    ones = np.ones(n, np.int32)
    for v in variants(skel, skel.SK_SCAN):
        c = cont(skel, ones)
        skel.skel_scan(c, c, skel.INCLUSIVE, skel.SUM, variant=v)  # in place
        assert np.array_equal(c.to_numpy(), np.arange(1, n + 1, dtype=np.int32)), v
        x = si.int_uniform_i32(n, 100, 0, 7)
        inc, red = skel.Container.empty(skel.I64, n), scalar_out(skel, skel.I64)
        skel.skel_scan(cont(skel, x), inc, skel.INCLUSIVE, skel.SUM, variant=v)
        skel.skel_reduce(skel.SUM, cont(skel, x), red)
        assert inc.to_numpy()[-1] == red.to_numpy()[0]
    skel.skel_sync()


def test_scan_repeated_calls_reuse_descriptors(skel, oracle_mod):
    # the look-back descriptors and counters are reused across calls (a fresh
    # epoch each call): alternate sizes and the four single-pass variants
    # without clearing anything
    for k in range(24):
        n = [(1 << 20) + 1, 9000, (1 << 18) + 77][k % 3]
        x = si.int_uniform_i32(n, 1000, 5, k)
        out = skel.Container.empty(skel.I64, n)
        skel.skel_scan(cont(skel, x), out, skel.EXCLUSIVE, skel.SUM, variant=2 + (k // 3) % 4)
        assert np.array_equal(out.to_numpy(), oracle_mod.scan(x, "exclusive", "sum",
                                                              np.int64)), k
    skel.skel_sync()


# ------------------------------------------- drawn tiny shapes (hypothesis)
from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402


@settings(max_examples=40, deadline=None, suppress_health_check=list(HealthCheck))
@given(rows=st.integers(1, 90), cols=st.sampled_from([252, 255, 256, 257, 260, 512, 516, 768]),
       ry=st.integers(0, 4), rx=st.integers(0, 4), edge=st.sampled_from(list(EDGES)),
       sep=st.booleans(), seed=st.integers(0, 1000))
def test_mapoverlap2d_march_drawn_shapes(skel, oracle_mod, rows, cols, ry, rx, edge, sep, seed):
    # widths around whole 256-column strips, where the marching window
    # switches between its straight-line and general paths
    img = si.uniform_f32(rows * cols, -1.0, 1.0, 43, seed).reshape(rows, cols)
    wy = si.uniform_f32(2 * ry + 1, -1.0, 1.0, 43, 2000 + seed)
    wx = si.uniform_f32(2 * rx + 1, -1.0, 1.0, 43, 3000 + seed)
    kw = {"wy": wy, "wx": wx} if sep else {
        "w2d": (wy.astype(np.float64)[:, None] * wx.astype(np.float64)[None, :]).astype(
            np.float32)}
    ref, mag = oracle_mod.mapoverlap2d(img, ry, rx, edge=edge, pad=-0.5, **kw)
    out = skel.Container.empty(skel.F32, rows, cols)
    skel.skel_mapoverlap2d(cont(skel, img), out, ry=ry, rx=rx, edge=EDGES[edge], pad=-0.5,
                           variant=skel.variant_index(skel.SK_MAPOVERLAP2D, "O2e_march"), **kw)
    got = out.to_numpy().reshape(rows, cols).astype(np.float64)
    assert np.all(np.abs(got - ref) <= 1e-6 * mag + 1e-30), (rows, cols, ry, rx, edge, sep)


@settings(max_examples=60, deadline=None, suppress_health_check=list(HealthCheck))
@given(rows=st.integers(1, 40), cols=st.integers(1, 40), ry=st.integers(0, 8),
       rx=st.integers(0, 8), edge=st.sampled_from(list(EDGES)), sep=st.booleans(),
       seed=st.integers(0, 1000))
def test_mapoverlap2d_drawn_shapes(skel, oracle_mod, rows, cols, ry, rx, edge, sep, seed):
    img = si.uniform_f32(rows * cols, -1.0, 1.0, 13, seed).reshape(rows, cols)
    wy = si.uniform_f32(2 * ry + 1, -1.0, 1.0, 13, 2000 + seed)
    wx = si.uniform_f32(2 * rx + 1, -1.0, 1.0, 13, 3000 + seed)
    kw = {"wy": wy, "wx": wx} if sep else {
        "w2d": (wy.astype(np.float64)[:, None] * wx.astype(np.float64)[None, :]).astype(
            np.float32)}
    ref, mag = oracle_mod.mapoverlap2d(img, ry, rx, edge=edge, pad=0.375, **kw)
    for v in variants(skel, skel.SK_MAPOVERLAP2D):
        if (v in (2, 3) and not sep) or (v == 4 and max(ry, rx) > 4):
            continue
        out = skel.Container.empty(skel.F32, rows, cols)
        skel.skel_mapoverlap2d(cont(skel, img), out, ry=ry, rx=rx, edge=EDGES[edge],
                               pad=0.375, variant=v, **kw)
        got = out.to_numpy().reshape(rows, cols).astype(np.float64)
        assert np.all(np.abs(got - ref) <= 1e-6 * mag + 1e-30), (v, rows, cols, ry, rx, edge)


@settings(max_examples=60, deadline=None, suppress_health_check=list(HealthCheck))
@given(n=st.integers(1, 3000), r=st.integers(0, 9), edge=st.sampled_from(list(EDGES)),
       seed=st.integers(0, 1000))
def test_mapoverlap1d_drawn_sizes(skel, oracle_mod, n, r, edge, seed):
    x = si.uniform_f32(n, -1.0, 1.0, 14, seed)
    w = si.uniform_f32(2 * r + 1, -1.0, 1.0, 14, 2000 + seed)
    ref, mag = oracle_mod.mapoverlap1d(x, w, r, edge, -0.5)
    for v in variants(skel, skel.SK_MAPOVERLAP1D):
        if v == 2 and r > 4:
            continue
        out = skel.Container.empty(skel.F32, n)
        skel.skel_mapoverlap1d(cont(skel, x), out, w, r, EDGES[edge], -0.5, variant=v)
        assert np.all(np.abs(out.to_numpy() - ref) <= 1e-6 * mag + 1e-30), (v, n, r, edge)
    # and the adjoint on the same draw
    ga, gm = oracle_mod.mapoverlap1d_adjoint(x, w, r, edge)
    for v in range(skel.skel_variant_count(skel.SK_MAPOVERLAP1D_BACKWARD)):
        out = skel.Container.empty(skel.F32, n)
        skel.skel_mapoverlap1d_backward(cont(skel, x), out, w, r, EDGES[edge], variant=v)
        assert np.all(np.abs(out.to_numpy() - ga) <= 1e-6 * gm + 1e-30), (n, r, edge, v)
