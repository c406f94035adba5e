"""Pins of the CPU oracle against facts fixed by the mathematics.

Each skeleton definition (Section III of arXiv:1405.2915: map, reduce, scan as
higher-order functions, mapoverlap as a neighbourhood map) is checked against
hand-worked examples (tests/golden/hand_examples.json), closed forms,
invariants, library routines it reduces to (math.fsum, numpy.cumsum,
scipy.ndimage.correlate*), and exact rational brute force on tiny inputs.  The
checks are chosen so that a dropped term, a wrong sign or index, a swapped
operand or an off-by-one in inclusive/exclusive fails at least one of them.
"""
import functools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

import synth_inputs as si

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "hand_examples.json")))


# ------------------------------------------------------------------ golden --

def test_golden_map(oracle_mod):
    g = GOLD["map_axpy"]
    out = oracle_mod.map_f32("axpy", [g["p0"]], np.array(g["x"], np.float32),
                             np.array(g["y"], np.float32))
    assert out.tolist() == g["out"]
    g = GOLD["map_affine"]
    out = oracle_mod.map_f32("affine", [g["p0"], g["p1"]],
                             np.array(g["x"], np.float32))
    assert out.tolist() == g["out"]


def test_golden_reduce(oracle_mod):
    g = GOLD["reduce_sum_i32"]
    assert oracle_mod.reduce("sum", np.array(g["x"], np.int32)) == g["out"]
    assert oracle_mod.reduce("sum", np.array(g["x"], np.float32)) == g["out"]
    g = GOLD["reduce_min_max_i32"]
    x = np.array(g["x"], np.int32)
    assert oracle_mod.reduce("min", x) == g["min"]
    assert oracle_mod.reduce("max", x) == g["max"]
    assert oracle_mod.reduce("min", x, np.int64) == g["min"]
    assert oracle_mod.reduce("max", x.astype(np.int64)) == g["max"]
    assert oracle_mod.reduce("min", x.astype(np.float32)) == g["min"]
    g = GOLD["reduce_wrap_i32"]
    x = np.array(g["x"], np.int32)
    assert oracle_mod.reduce("sum", x) == g["out_i32"]
    assert oracle_mod.reduce("sum", x, np.int64) == g["out_i64"]


def test_golden_mapreduce(oracle_mod):
    g = GOLD["mapreduce_dot"]
    r, mag = oracle_mod.mapreduce("mul", None, np.array(g["x"], np.float32),
                                  np.array(g["y"], np.float32))
    assert r == g["out"]
    assert mag == 16.0  # 4 + 2 + 6 + 4


@pytest.mark.parametrize("name,op", [("scan_sum_i32", "sum"),
                                     ("scan_max_i32", "max")])
def test_golden_scan(oracle_mod, name, op):
    g = GOLD[name]
    x = np.array(g["x"], np.int32)
    for kind in ("inclusive", "exclusive", "reverse_inclusive", "reverse_exclusive"):
        assert oracle_mod.scan(x, kind, op).tolist() == g[kind]
        if op == "sum":
            assert oracle_mod.scan(x, kind, op, np.int64).tolist() == g[kind]
            assert oracle_mod.scan(x.astype(np.int64), kind, op).tolist() == g[kind]
            out, _ = oracle_mod.scan(x.astype(np.float32), kind, op)
            assert out.tolist() == g[kind]


@pytest.mark.parametrize("name,edge", [("mapoverlap1d_clamp", "clamp"),
                                       ("mapoverlap1d_const", "const"),
                                       ("mapoverlap1d_cyclic", "cyclic")])
def test_golden_mapoverlap1d(oracle_mod, name, edge):
    g = GOLD[name]
    out, _ = oracle_mod.mapoverlap1d(np.array(g["x"], np.float32),
                                     np.array(g["w"], np.float32), g["r"],
                                     edge, g.get("pad", 0.0))
    assert out.tolist() == g["out"]


@pytest.mark.parametrize("edge", ["clamp", "const", "cyclic"])
def test_golden_mapoverlap1d_adjoint(oracle_mod, edge):
    g = GOLD["mapoverlap1d_adjoint_" + edge]
    dx, mag = oracle_mod.mapoverlap1d_adjoint(np.array(g["g"], np.float32),
                                              np.array(g["w"], np.float32), g["r"], edge)
    assert dx.tolist() == g["dx"]
    assert mag.tolist() == g["dx"]  # every term is positive here


def test_golden_mapoverlap2d(oracle_mod):
    g = GOLD["mapoverlap2d_clamp"]
    out, _ = oracle_mod.mapoverlap2d(np.array(g["x"], np.float32), 1, 1,
                                     w2d=np.array(g["w"], np.float32))
    assert out.tolist() == g["out"]


# --------------------------------------------------------------------- Map --

def test_map_saxpy_exact_on_grid(oracle_mod):
    # x, y = 2U - 1 with U on the 2^-24 grid: x, y on the 2^-23 grid, so
    # 2.5 x + y is exact in binary64 and equal to the exact rational value.
    x = si.uniform_f32(4096, -1.0, 1.0, 0, 0)
    y = si.uniform_f32(4096, -1.0, 1.0, 0, 1)
    assert np.all((x.astype(np.float64) * 2 ** 23) % 1 == 0)
    out = oracle_mod.map_f32("axpy", [2.5], x, y)
    for i in range(0, 4096, 37):
        exact = Fraction(5, 2) * Fraction(float(x[i])) + Fraction(float(y[i]))
        assert Fraction(float(out[i])) == exact


def test_map_properties(oracle_mod):
    x = si.uniform_f32(1000, -1.0, 1.0, 0, 2)
    y = si.uniform_f32(1000, -1.0, 1.0, 0, 3)
    z = np.zeros_like(x)
    # x = 0 leaves y unchanged; y = 0 gives p0 * x (operand roles fixed)
    assert np.array_equal(oracle_mod.map_f32("axpy", [2.5], z, y), y)
    assert np.array_equal(oracle_mod.map_f32("axpy", [3.0], x, z),
                          3.0 * x.astype(np.float64))
    # affine with p0 = 0 is the constant p1; identity copies
    assert np.all(oracle_mod.map_f32("affine", [0.0, 1.25], x) == 1.25)
    assert np.array_equal(oracle_mod.map_f32("identity", None, x), x)
    # mul commutes, square = mul(x, x), x * 1 = x
    assert np.array_equal(oracle_mod.map_f32("mul", None, x, y),
                          oracle_mod.map_f32("mul", None, y, x))
    assert np.array_equal(oracle_mod.map_f32("square", None, x),
                          oracle_mod.map_f32("mul", None, x, x))
    assert np.array_equal(oracle_mod.map_f32("mul", None, x, np.ones_like(x)), x)


def test_map_tanh_library(oracle_mod):
    x = si.normal_f32(500, 0, 4) * np.float32(3)
    t = oracle_mod.map_f32("tanh", None, x)
    ref = np.array([math.tanh(float(v)) for v in x])
    assert np.array_equal(t, ref)
    # affine_tanh(p0, p1) = tanh(p0 x + p1); p0 = 1, p1 = 0 reduces to tanh
    assert np.array_equal(oracle_mod.map_f32("affine_tanh", [1.0, 0.0], x), t)
    at = oracle_mod.map_f32("affine_tanh", [0.5, -0.25], x)
    ref = np.array([math.tanh(0.5 * float(v) - 0.25) for v in x])
    assert np.array_equal(at, ref)
    # odd symmetry, tanh(0) = 0
    assert np.array_equal(oracle_mod.map_f32("tanh", None, -x), -t)
    assert oracle_mod.map_f32("tanh", None, np.zeros(1, np.float32))[0] == 0.0


def test_map_rejects_bad_ops(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.map_f32("axpy", [], np.ones(3, np.float32), np.ones(3, np.float32))
    with pytest.raises(ValueError):
        oracle_mod.map_f32("mul", None, np.ones(3, np.float32))


# ------------------------------------------------------------------ Reduce --

@pytest.mark.parametrize("n", [0, 1, 2, 3, 1000, 65536, 1 << 20])
def test_reduce_sum_of_indices(oracle_mod, n):
    # sum_{i<n} i = n (n - 1) / 2; binary32 holds i exactly for n <= 2^24
    i32 = np.arange(n, dtype=np.int32)
    exact = n * (n - 1) // 2
    assert oracle_mod.reduce("sum", i32.astype(np.float32)) == float(exact)
    assert oracle_mod.reduce("sum", i32, np.int64) == exact
    assert oracle_mod.reduce("sum", i32.astype(np.int64)) == exact
    wrapped = ((exact + 2 ** 31) % 2 ** 32) - 2 ** 31
    assert oracle_mod.reduce("sum", i32) == wrapped
    if n <= 65536:
        assert oracle_mod.reduce("sum", i32) == exact


def test_reduce_special_cases(oracle_mod):
    ones = np.ones(12345, np.float32)
    assert oracle_mod.reduce("sum", ones) == 12345.0
    alt = np.where(np.arange(1001) % 2 == 0, 1, -1).astype(np.float32)
    assert oracle_mod.reduce("sum", alt) == 1.0
    empty = np.zeros(0, np.float32)
    assert oracle_mod.reduce("sum", empty) == 0.0
    assert oracle_mod.reduce("min", empty) == math.inf
    assert oracle_mod.reduce("max", empty) == -math.inf
    ei = np.zeros(0, np.int32)
    assert oracle_mod.reduce("min", ei) == 2 ** 31 - 1
    assert oracle_mod.reduce("max", ei, np.int64) == -2 ** 63


def test_reduce_fsum_and_bruteforce(oracle_mod):
    x = si.normal_f32(1 << 16, 0, 5)
    s = oracle_mod.reduce("sum", x)
    exact = math.fsum(float(v) for v in x)
    # sequential binary64 error bound n * 2^-53 * sum |x|
    assert abs(s - exact) <= x.size * 2.0 ** -53 * oracle_mod.abs_sum(x)
    assert oracle_mod.abs_sum(x) == pytest.approx(float(np.abs(x.astype(np.float64)).sum()),
                                                  rel=1e-12)
    assert oracle_mod.reduce("min", x) == float(x.min())
    assert oracle_mod.reduce("max", x) == float(x.max())
    rng = si.rng(9, 0)
    for n in range(0, 65):
        xi = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
        tot = sum(int(v) for v in xi)
        assert oracle_mod.reduce("sum", xi, np.int64) == tot
        assert oracle_mod.reduce("sum", xi) == ((tot + 2 ** 31) % 2 ** 32) - 2 ** 31
        if n:
            assert oracle_mod.reduce("min", xi) == min(int(v) for v in xi)
            assert oracle_mod.reduce("max", xi) == max(int(v) for v in xi)
        xl = rng.integers(-2 ** 62, 2 ** 62, n, dtype=np.int64)
        t = sum(int(v) for v in xl)
        assert oracle_mod.reduce("sum", xl) == ((t + 2 ** 63) % 2 ** 64) - 2 ** 63


def test_reduce_segments_pins(oracle_mod):
    # segments of 0..n-1: each sum is the closed form of an arithmetic range
    n = 100000
    x = np.arange(n, dtype=np.float32)
    off = np.array([0, 0, 1, 17, 17, 5000, 65536, n], np.int64)
    out = oracle_mod.reduce_segments("sum", x, off)
    for s in range(off.size - 1):
        a, b = int(off[s]), int(off[s + 1])
        assert out[s] == (b * (b - 1) - a * (a - 1)) // 2  # sum of a..b-1
    # empty segments give the identity of each operator
    assert out[0] == 0 and out[3] == 0
    mn = oracle_mod.reduce_segments("min", x, off)
    assert mn[0] == math.inf and mn[2] == 1.0 and mn[4] == 17.0
    mx = oracle_mod.reduce_segments("max", x, off)
    assert mx[0] == -math.inf and mx[-1] == n - 1
    # one segment over everything is the plain Reduce
    y = si.normal_f32(4097, 2, 7)
    assert oracle_mod.reduce_segments("sum", y, [0, 4097])[0] == oracle_mod.reduce("sum", y)
    with pytest.raises(ValueError):
        oracle_mod.reduce_segments("sum", y, [0, 10, 5, 4097])
    with pytest.raises(ValueError):
        oracle_mod.reduce_segments("sum", y, [0, 4098])


def test_exact_sums_pins(oracle_mod):
    # the exactly rounded sum equals Python's math.fsum (the same published
    # algorithm, independently implemented) on hard inputs
    g = si.rng(12, 0)
    for trial in range(20):
        x = g.standard_normal(500) * np.exp(g.uniform(-60, 60, 500))
        x = np.concatenate([x, -x[: 200] * (1 + 2.0 ** -50)])
        g.shuffle(x)
        assert oracle_mod.fsum(x) == math.fsum(x.tolist())
    # exact cancellation, and a half-way case plain summation gets wrong
    assert oracle_mod.fsum([1e16, 1.0, -1e16]) == 1.0
    assert oracle_mod.fsum([1.0, 2.0 ** -53, 2.0 ** -106]) == 1.0 + 2.0 ** -52
    assert oracle_mod.fsum([]) == 0.0
    # bf16 sums: values on a 2^-17 grid below 2^10 sum exactly as scaled
    # integers, so the exact sum is known independently
    bits = si.log_uniform_signed_bf16(200000, config=4, index=3)
    vals = si.bf16_bits_to_f32(bits).astype(np.float64)
    scaled = sum(int(v * 2 ** 17) for v in vals)
    assert all(float(v * 2 ** 17).is_integer() for v in vals[:1000])
    assert oracle_mod.sum_bf16_exact(bits) == scaled / 2 ** 17
    # bf16 dot: products are exact in binary64; compare with math.fsum of them
    b2 = si.log_uniform_signed_bf16(200000, config=4, index=4)
    v2 = si.bf16_bits_to_f32(b2).astype(np.float64)
    assert oracle_mod.dot_bf16_exact(bits, b2) == math.fsum((vals * v2).tolist())
    # and it stays close to (but is not always equal to) the sequential sum
    assert abs(oracle_mod.sum_bf16_exact(bits) - float(np.sum(vals))) <= \
        vals.size * 2.0 ** -52 * float(np.sum(np.abs(vals)))


# --------------------------------------------------------------- MapReduce --

def test_mapreduce_identities(oracle_mod):
    x = si.normal_f32(4097, 1, 0)
    y = si.normal_f32(4097, 1, 1)
    ones = np.ones_like(x)
    # dot(x, 1) performs exactly the additions of reduce(x)
    r, _ = oracle_mod.mapreduce("mul", None, x, ones)
    assert r == oracle_mod.reduce("sum", x)
    # dot(e_k, y) = y_k
    for k in (0, 17, 4096):
        e = np.zeros_like(x)
        e[k] = 1
        assert oracle_mod.mapreduce("mul", None, e, y)[0] == float(y[k])
    # dot(x, x) = sum of squares >= 0, and equals mapreduce(square)
    rxx, mag = oracle_mod.mapreduce("mul", None, x, x)
    assert rxx >= 0 and rxx == mag
    assert rxx == oracle_mod.mapreduce("square", None, x)[0]
    # numpy binary64 dot agrees to rounding
    ref = float(np.dot(x.astype(np.float64), y.astype(np.float64)))
    r, mag = oracle_mod.mapreduce("mul", None, x, y)
    assert abs(r - ref) <= 4097 * 2.0 ** -52 * mag
    # min / max of the mapped values
    prods = x.astype(np.float64) * y.astype(np.float64)
    assert oracle_mod.mapreduce("mul", None, x, y, "max")[0] == prods.max()
    assert oracle_mod.mapreduce("mul", None, x, y, "min")[0] == prods.min()


def test_mapreduce_exact_bruteforce(oracle_mod):
    # products of binary32 values are exact in binary64; the binary64 sum of a
    # few terms stays within n ulps of the exact rational sum
    for seed in range(8):
        x = si.normal_f32(13, 7, seed)
        y = si.normal_f32(13, 8, seed)
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y))
        r, mag = oracle_mod.mapreduce("mul", None, x, y)
        assert abs(Fraction(r) - exact) <= Fraction(13 * 2.0 ** -53) * Fraction(mag)
        r, _ = oracle_mod.mapreduce("axpy", [2.5], x, y)
        exact = sum(Fraction(5, 2) * Fraction(float(a)) + Fraction(float(b))
                    for a, b in zip(x, y))
        assert abs(Fraction(r) - exact) < Fraction(1, 2 ** 40)


# -------------------------------------------------------------- MapOverlap --

def test_mapoverlap1d_constant_field(oracle_mod):
    # clamp keeps a constant field constant, so out = c * sum(w), borders too
    for w in (si.binomial5_weights(), si.gaussian_weights(4, 2.0),
              np.array([0.1, -0.7, 0.3], np.float32)):
        r = (w.size - 1) // 2
        c = np.float32(0.75)
        out, _ = oracle_mod.mapoverlap1d(np.full(300, c, np.float32), w, r)
        sw = math.fsum(float(v) for v in w)
        assert np.all(np.abs(out - float(c) * sw) <= 1e-15)
    # the binomial weights sum to 1 exactly; the 9-tap Gaussian to 1.000000011...
    assert math.fsum(float(v) for v in si.binomial5_weights()) == 1.0
    assert math.fsum(float(v) for v in si.gaussian_weights()) == pytest.approx(
        1.000000011175871, abs=1e-15)


def test_mapoverlap1d_impulse_orientation(oracle_mod):
    # correlation orientation: an impulse at m yields out[m + j] = w[r - j]
    w = np.array([1, 2, 3, 4, 5], np.float32)
    x = np.zeros(21, np.float32)
    x[10] = 1
    out, _ = oracle_mod.mapoverlap1d(x, w, 2)
    assert out[8:13].tolist() == [5, 4, 3, 2, 1]
    assert np.count_nonzero(out) == 5


@pytest.mark.parametrize("edge,mode", [("clamp", "nearest"), ("const", "constant"),
                                       ("cyclic", "wrap")])
@pytest.mark.parametrize("n,r", [(1, 2), (3, 2), (64, 1), (1000, 5), (7, 4)])
def test_mapoverlap1d_scipy(oracle_mod, edge, mode, n, r):
    x = si.uniform_f32(n, -1.0, 1.0, 3, n)
    w = si.uniform_f32(2 * r + 1, -1.0, 1.0, 3, 100 + r)
    pad = 0.375
    out, mag = oracle_mod.mapoverlap1d(x, w, r, edge, pad)
    ref = ndi.correlate1d(x.astype(np.float64), w.astype(np.float64), mode=mode,
                          cval=pad)
    assert np.all(np.abs(out - ref) <= 1e-14 * (mag + 1e-300))
    assert np.all(mag >= np.abs(out) - 1e-15)


def test_mapoverlap1d_ramp(oracle_mod):
    # symmetric weights summing to 1 reproduce a linear ramp in the interior
    x = np.arange(200, dtype=np.float32) * np.float32(0.5)
    out, _ = oracle_mod.mapoverlap1d(x, si.binomial5_weights(), 2)
    assert np.array_equal(out[2:-2], x[2:-2].astype(np.float64))


@pytest.mark.parametrize("shape", [(1, 1), (1, 17), (13, 1), (40, 33), (5, 3)])
@pytest.mark.parametrize("edge,mode", [("clamp", "nearest"), ("const", "constant"),
                                       ("cyclic", "wrap")])
def test_mapoverlap2d_scipy(oracle_mod, shape, edge, mode):
    x = si.uniform_f32(shape[0] * shape[1], 0.0, 1.0, 3, 7).reshape(shape)
    w = si.uniform_f32(5 * 7, -1.0, 1.0, 3, 8).reshape(5, 7)  # ry = 2, rx = 3
    out, mag = oracle_mod.mapoverlap2d(x, 2, 3, w2d=w, edge=edge, pad=-0.5)
    ref = ndi.correlate(x.astype(np.float64), w.astype(np.float64), mode=mode,
                        cval=-0.5)
    assert np.all(np.abs(out - ref) <= 1e-14 * mag)


def test_mapoverlap2d_impulse_and_transpose(oracle_mod):
    # W not symmetric: the impulse response is W flipped in both axes, which
    # exposes a transposed or mirrored weight index
    w = np.arange(1, 16, dtype=np.float32).reshape(3, 5)  # ry = 1, rx = 2
    x = np.zeros((9, 11), np.float32)
    x[4, 5] = 1
    out, _ = oracle_mod.mapoverlap2d(x, 1, 2, w2d=w)
    assert np.array_equal(out[3:6, 3:8], w[::-1, ::-1].astype(np.float64))
    assert np.count_nonzero(out) == 15


def test_mapoverlap2d_separable_and_constant(oracle_mod):
    g = si.gaussian_weights(4, 2.0)
    x = si.uniform_f32(37 * 29, 0.0, 1.0, 1, 0).reshape(37, 29)
    sep, mag = oracle_mod.mapoverlap2d(x, 4, 4, wy=g, wx=g)
    full = np.outer(g.astype(np.float64), g.astype(np.float64))
    # the 2D weights as binary32 products would round; the separable form uses
    # the exact binary64 outer product, equal to correlate with that W
    ref = ndi.correlate(x.astype(np.float64), full, mode="nearest")
    assert np.all(np.abs(sep - ref) <= 1e-14 * mag)
    # separable identity: rows(wx) then columns(wy) in binary64
    rows = ndi.correlate1d(x.astype(np.float64), g.astype(np.float64), axis=1,
                           mode="nearest")
    both = ndi.correlate1d(rows, g.astype(np.float64), axis=0, mode="nearest")
    assert np.all(np.abs(sep - both) <= 1e-14 * mag)
    # constant field -> c * (sum w)^2 everywhere, corners included
    c = np.float32(0.3)
    out, _ = oracle_mod.mapoverlap2d(np.full((20, 20), c, np.float32), 4, 4,
                                     wy=g, wx=g)
    sw = math.fsum(float(v) for v in g)
    assert np.all(np.abs(out - float(c) * sw * sw) <= 1e-15)
    assert sw * sw == pytest.approx(1.0000000223517418, abs=1e-15)
    # separable factors that differ: W[a][b] = wy[a] * wx[b], not wy[b] * wx[a]
    wy = np.array([0.25, 0.5, -1.0], np.float32)
    wx = np.array([2.0, -0.125, 0.75, 1.5, 3.0], np.float32)
    s2, m2 = oracle_mod.mapoverlap2d(x, 1, 2, wy=wy, wx=wx)
    ref = ndi.correlate(x.astype(np.float64),
                        np.outer(wy.astype(np.float64), wx.astype(np.float64)),
                        mode="nearest")
    assert np.all(np.abs(s2 - ref) <= 1e-14 * m2)
    # single-output form agrees with the full form
    for (i, j) in ((0, 0), (36, 28), (18, 3)):
        v, m = oracle_mod.mapoverlap2d_at(x, 4, 4, i, j, wy=g, wx=g)
        assert v == sep[i, j] and m == mag[i, j]


# -------------------------------------------------------------------- Scan --

def test_scan_closed_forms(oracle_mod):
    n = 100000
    ones = np.ones(n, np.int32)
    assert np.array_equal(oracle_mod.scan(ones, "inclusive"), np.arange(1, n + 1))
    assert np.array_equal(oracle_mod.scan(ones, "exclusive"), np.arange(n))
    x = si.int_uniform_i32(n, 1000, 1, 0)
    inc = oracle_mod.scan(x, "inclusive", "sum", np.int64)
    exc = oracle_mod.scan(x, "exclusive", "sum", np.int64)
    assert inc[-1] == oracle_mod.reduce("sum", x, np.int64)
    assert exc[0] == 0
    assert np.array_equal(np.diff(exc), x[:-1].astype(np.int64))
    assert exc[-1] + x[-1] == inc[-1]
    assert np.array_equal(inc, np.cumsum(x, dtype=np.int64))


def test_scan_wrap_and_library(oracle_mod):
    x = si.rng(2, 3).integers(-2 ** 31, 2 ** 31, 5000, dtype=np.int64).astype(np.int32)
    inc32 = oracle_mod.scan(x, "inclusive")
    inc64 = oracle_mod.scan(x, "inclusive", "sum", np.int64)
    assert np.array_equal(inc64, np.cumsum(x.astype(np.int64)))
    assert np.array_equal(inc32, inc64.astype(np.int32))  # mod 2^32
    assert np.array_equal(oracle_mod.scan(x, "inclusive", "min"),
                          np.minimum.accumulate(x))
    assert np.array_equal(oracle_mod.scan(x, "inclusive", "max", np.int64),
                          np.maximum.accumulate(x.astype(np.int64)))
    exc = oracle_mod.scan(x, "exclusive", "min")
    assert exc[0] == 2 ** 31 - 1
    assert np.array_equal(exc[1:], np.minimum.accumulate(x)[:-1])
    xl = si.rng(2, 4).integers(-2 ** 62, 2 ** 62, 3000, dtype=np.int64)
    with np.errstate(over="ignore"):
        assert np.array_equal(oracle_mod.scan(xl, "inclusive"), np.cumsum(xl))


def test_scan_f32(oracle_mod):
    x = si.normal_f32(3000, 0, 11)
    out, mag = oracle_mod.scan(x, "inclusive")
    assert np.array_equal(out, np.cumsum(x.astype(np.float64)))
    assert np.array_equal(mag, np.cumsum(np.abs(x.astype(np.float64))))
    exc, emag = oracle_mod.scan(x, "exclusive")
    assert exc[0] == 0.0 and emag[0] == 0.0
    assert np.array_equal(exc[1:], out[:-1])
    assert out[-1] == oracle_mod.reduce("sum", x)
    mx, _ = oracle_mod.scan(x, "inclusive", "max")
    assert np.array_equal(mx, np.maximum.accumulate(x.astype(np.float64)))


def test_scan_bruteforce_tiny(oracle_mod):
    rng = si.rng(5, 5)
    for n in range(0, 65):
        x = rng.integers(-50, 51, n, dtype=np.int32)
        for op, fn in (("sum", lambda a, b: a + b), ("min", min), ("max", max)):
            acc = None
            inc, exc = [], []
            ident = {"sum": 0, "min": 2 ** 31 - 1, "max": -2 ** 31}[op]
            for v in x:
                exc.append(ident if acc is None else acc)
                acc = int(v) if acc is None else fn(acc, int(v))
                inc.append(acc)
            assert oracle_mod.scan(x, "inclusive", op).tolist() == inc
            assert oracle_mod.scan(x, "exclusive", op).tolist() == exc
            # suffix forms, brute force from the definition
            rinc = [functools.reduce(fn, [int(v) for v in x[i:]]) for i in range(n)]
            rexc = [functools.reduce(fn, [int(v) for v in x[i + 1:]], ident)
                    for i in range(n)]
            assert oracle_mod.scan(x, "reverse_inclusive", op).tolist() == rinc
            assert oracle_mod.scan(x, "reverse_exclusive", op).tolist() == rexc


# ------------------------------------------------------------ generators --

def test_generators_reproducible_and_on_grid():
    a = si.uniform_f32(1000, -1.0, 1.0, 0, 0)
    b = si.uniform_f32(1000, -1.0, 1.0, 0, 0)
    assert np.array_equal(a, b) and a.dtype == np.float32
    assert a.min() >= -1 and a.max() < 1
    assert np.all((a.astype(np.float64) * 2 ** 23) % 1 == 0)
    g = si.gaussian_weights()
    assert g.dtype == np.float32 and g.size == 9
    assert g[4] == np.float32(0.20416368544101715)
    assert g[0] == g[8] == np.float32(0.027630550786852837)
    lens = si.log_uniform_lengths(4096, 32, 1 << 20)
    assert lens.min() >= 32 and lens.max() <= 1 << 20
    h = si.bf16_bits_from_f32(np.array([1.0, -2.5, 3.0e-3, 1.00390625], np.float32))
    assert h.tolist() == [0x3F80, 0xC020, 0x3B45, 0x3F80]  # last: tie to even


# ------------------------------------------------------------- adjoints --

def test_reverse_scan_f32_and_widening(oracle_mod):
    x = si.normal_f32(2000, 0, 12)
    xd = x.astype(np.float64)
    ri, rmag = oracle_mod.scan(x, "reverse_inclusive")
    assert np.array_equal(ri, np.cumsum(xd[::-1])[::-1])
    assert np.array_equal(rmag, np.cumsum(np.abs(xd[::-1]))[::-1])
    re_, _ = oracle_mod.scan(x, "reverse_exclusive")
    assert re_[-1] == 0.0 and np.array_equal(re_[:-1], ri[1:])
    xi = si.rng(5, 6).integers(-2 ** 31, 2 ** 31, 500, dtype=np.int64).astype(np.int32)
    wide = oracle_mod.scan(xi, "reverse_inclusive", "sum", np.int64)
    exact = np.cumsum(xi.astype(object)[::-1])[::-1]
    assert wide.tolist() == [int(v) for v in exact]
    narrow = oracle_mod.scan(xi, "reverse_inclusive", "sum")
    assert narrow.tolist() == [((int(v) + 2 ** 31) % 2 ** 32) - 2 ** 31 for v in exact]


def test_scan_rows_library_forms(oracle_mod):
    # a row-wise scan is numpy's cumsum along the last axis (exact in int64;
    # the float32 case against a float64 cumsum of the stored values)
    g = si.rng(5, 7)
    x = g.integers(-1000, 1000, (7, 301), dtype=np.int64).astype(np.int32)
    c = np.cumsum(x.astype(np.int64), axis=1)
    assert np.array_equal(oracle_mod.scan_rows(x, "inclusive", "sum", np.int64), c)
    assert np.array_equal(oracle_mod.scan_rows(x, "exclusive", "sum", np.int64), c - x)
    rc = np.cumsum(x[:, ::-1].astype(np.int64), axis=1)[:, ::-1]
    assert np.array_equal(oracle_mod.scan_rows(x, "reverse_inclusive", "sum", np.int64), rc)
    assert np.array_equal(oracle_mod.scan_rows(x, "reverse_exclusive", "sum", np.int64), rc - x)
    assert np.array_equal(oracle_mod.scan_rows(x, "inclusive", "max"),
                          np.maximum.accumulate(x, axis=1))
    xf = si.normal_f32(5 * 64, 0, 13).reshape(5, 64)
    out, mag = oracle_mod.scan_rows(xf, "inclusive")
    assert np.array_equal(out, np.cumsum(xf.astype(np.float64), axis=1))
    assert np.array_equal(mag, np.cumsum(np.abs(xf.astype(np.float64)), axis=1))
    # rows do not leak into each other: a row of ones after a row of large values
    y = np.array([[10 ** 6] * 5, [1] * 5], np.int32)
    assert oracle_mod.scan_rows(y, "inclusive", "sum").tolist()[1] == [1, 2, 3, 4, 5]
    assert oracle_mod.scan_rows(np.zeros((3, 0), np.int32)).shape == (3, 0)


def _dense_1d(oracle_mod, n, w, r, edge):
    """The forward map as a dense matrix, column j = forward(e_j) (pad 0)."""
    a = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n, np.float32)
        e[j] = 1.0
        a[:, j], _ = oracle_mod.mapoverlap1d(e, w, r, edge, 0.0)
    return a


@pytest.mark.parametrize("edge", ["clamp", "const", "cyclic"])
@pytest.mark.parametrize("n,r", [(1, 0), (1, 2), (3, 2), (7, 2), (12, 3), (5, 4)])
def test_mapoverlap1d_adjoint_is_transpose(oracle_mod, edge, n, r):
    w = si.uniform_f32(2 * r + 1, -1.0, 1.0, 6, r)
    g = si.uniform_f32(n, -1.0, 1.0, 6, 10 + n)
    a = _dense_1d(oracle_mod, n, w, r, edge)
    dx, _ = oracle_mod.mapoverlap1d_adjoint(g, w, r, edge)
    np.testing.assert_allclose(dx, a.T @ g.astype(np.float64), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("edge", ["clamp", "const", "cyclic"])
def test_mapoverlap1d_adjoint_inner_products(oracle_mod, edge):
    # <A x, g> = <x, A^T g> with A x from the forward map (the pad term of the
    # constant border is affine, so it is zero here)
    n, r = 4099, 3
    w = si.uniform_f32(2 * r + 1, -1.0, 1.0, 6, 40)
    x = si.normal_f32(n, 6, 41)
    g = si.normal_f32(n, 6, 42)
    ax, _ = oracle_mod.mapoverlap1d(x, w, r, edge, 0.0)
    atg, _ = oracle_mod.mapoverlap1d_adjoint(g, w, r, edge)
    lhs = math.fsum(ax * g.astype(np.float64))
    rhs = math.fsum(x.astype(np.float64) * atg)
    assert abs(lhs - rhs) <= 1e-12 * math.fsum(np.abs(ax * g))


@pytest.mark.parametrize("edge", ["clamp", "const", "cyclic"])
@pytest.mark.parametrize("shape,ry,rx", [((1, 1), 1, 1), ((5, 4), 2, 1), ((6, 9), 1, 3),
                                         ((3, 3), 0, 2)])
def test_mapoverlap2d_adjoint_is_transpose(oracle_mod, edge, shape, ry, rx):
    rows, cols = shape
    w2d = si.uniform_f32((2 * ry + 1) * (2 * rx + 1), -1.0, 1.0, 6, 50).reshape(
        2 * ry + 1, 2 * rx + 1)
    g = si.uniform_f32(rows * cols, -1.0, 1.0, 6, 51).reshape(rows, cols)
    a = np.zeros((rows * cols, rows * cols))
    for s in range(rows * cols):
        e = np.zeros(rows * cols, np.float32)
        e[s] = 1.0
        col, _ = oracle_mod.mapoverlap2d(e.reshape(rows, cols), ry, rx, w2d=w2d, edge=edge)
        a[:, s] = col.reshape(-1)
    dx, _ = oracle_mod.mapoverlap2d_adjoint(g, ry, rx, w2d=w2d, edge=edge)
    np.testing.assert_allclose(dx.reshape(-1), a.T @ g.reshape(-1).astype(np.float64),
                               rtol=1e-13, atol=1e-15)
    # separable factors give the same map as their outer product
    wy = si.uniform_f32(2 * ry + 1, -1.0, 1.0, 6, 52)
    wx = si.uniform_f32(2 * rx + 1, -1.0, 1.0, 6, 53)
    d1, _ = oracle_mod.mapoverlap2d_adjoint(g, ry, rx, wy=wy, wx=wx, edge=edge)
    outer = (wy.astype(np.float64)[:, None] * wx.astype(np.float64)[None, :])
    d2 = np.zeros_like(d1)
    for s in range(rows * cols):  # A^T g for the outer-product weights, by columns
        e = np.zeros(rows * cols, np.float32)
        e[s] = 1.0
        col, _ = oracle_mod.mapoverlap2d(e.reshape(rows, cols), ry, rx, wy=wy, wx=wx,
                                         edge=edge)
        d2.reshape(-1)[s] = float(col.reshape(-1) @ g.reshape(-1).astype(np.float64))
    np.testing.assert_allclose(d1, d2, rtol=1e-13, atol=1e-15)
    assert outer.shape == (2 * ry + 1, 2 * rx + 1)


MAP_GRAD_CASES = [("identity", []), ("axpy", [2.5]), ("affine", [0.75, -0.5]),
                  ("tanh", []), ("affine_tanh", [1.5, 0.25]), ("mul", []), ("square", [])]


@pytest.mark.parametrize("op,params", MAP_GRAD_CASES)
def test_map_grad_finite_differences(oracle_mod, op, params):
    # central differences of the forward oracle in binary64: inputs on a
    # 2^-8 grid in [-1, 1), step 2^-12, so x +- h is exact in binary32
    n = 64
    rng = si.rng(6, 60)
    x = (rng.integers(-256, 256, n) / 256.0).astype(np.float32)
    y = (rng.integers(-256, 256, n) / 256.0).astype(np.float32)
    g = si.uniform_f32(n, -1.0, 1.0, 6, 61)
    two = op in oracle_mod.TWO_INPUT_MAP_OPS
    dx, dy, dp, _ = oracle_mod.map_grad(op, params, x, g, y if two else None)
    h = 2.0 ** -12

    def f(xx, yy, pp):
        return oracle_mod.map_f32(op, pp, xx, yy if two else None)

    fd_x = (f(x + np.float32(h), y, params) - f(x - np.float32(h), y, params)) / (2 * h)
    np.testing.assert_allclose(dx, g.astype(np.float64) * fd_x, rtol=1e-5, atol=1e-7)
    if two:
        fd_y = (f(x, y + np.float32(h), params) - f(x, y - np.float32(h), params)) / (2 * h)
        np.testing.assert_allclose(dy, g.astype(np.float64) * fd_y, rtol=1e-5, atol=1e-7)
    for k in range(len(params)):
        pp, pm = list(params), list(params)
        pp[k] += h
        pm[k] -= h
        fd_p = (f(x, y, pp) - f(x, y, pm)) / (2 * h)
        assert abs(dp[k] - math.fsum(g.astype(np.float64) * fd_p)) <= 1e-5 * (
            math.fsum(np.abs(g.astype(np.float64) * fd_p)) + 1e-12), (op, k)


def test_map_grad_rejects_bad_ops(oracle_mod):
    x = np.ones(4, np.float32)
    with pytest.raises(ValueError):
        oracle_mod.map_grad("affine", [1.0], x, x)  # needs two parameters


def test_oracle_threads_do_not_change_results(oracle_mod):
    """The element-parallel loops (map, stencils) give bit-identical results on
    one thread and on several (each output is computed alone, in a fixed
    order)."""
    x = si.normal_f32(10007, 7, 0)
    y = si.normal_f32(10007, 7, 1)
    img = si.uniform_f32(97 * 101, 0.0, 1.0, 7, 2).reshape(97, 101)
    w5, g9 = si.binomial5_weights(), si.gaussian_weights(4, 2.0)
    before = oracle_mod.get_threads()
    try:
        res = []
        for th in (1, 8):
            oracle_mod.set_threads(th)
            res.append((oracle_mod.map_f32("affine_tanh", [1.5, 0.25], x),
                        oracle_mod.map_f32("axpy", [2.5], x, y),
                        oracle_mod.mapoverlap1d(x, w5, 2, "cyclic")[0],
                        oracle_mod.mapoverlap2d(img, 4, 4, wy=g9, wx=g9, edge="clamp")[0]))
        for a, b in zip(*res):
            assert np.array_equal(a, b)
    finally:
        oracle_mod.set_threads(before)


# --------------------------------------------------------------- call chain --
# Map -> MapOverlap 2D -> Reduce SUM (a composition of skeleton calls)

CHAIN_MAPS = {"identity": ([], lambda x, p: x),
              "affine_tanh": ([0.75, -0.25], lambda x, p: np.tanh(p[0] * x + p[1])),
              "square": ([], lambda x, p: x * x)}


def _asym5():
    """asymmetric 5-point weights (C .5, N .1, S .2, W .05, E .15): a flipped
    or transposed tap changes the result"""
    return si.five_point_weights(0.5, 0.1, 0.2, 0.05, 0.15)


@pytest.mark.parametrize("edge,mode", [("clamp", "nearest"), ("const", "constant"),
                                       ("cyclic", "wrap")])
@pytest.mark.parametrize("shape,ry,rx", [((1, 1, 1), 1, 1), ((2, 3, 4), 1, 1),
                                         ((2, 16, 16), 1, 1), ((1, 7, 5), 2, 3),
                                         ((3, 4, 9), 0, 2)])
@pytest.mark.parametrize("op", sorted(CHAIN_MAPS))
def test_chain_scipy(oracle_mod, edge, mode, shape, ry, rx, op):
    """The chain equals scipy's correlation of the mapped fields, summed."""
    params, fn = CHAIN_MAPS[op]
    x = si.normal_f32(int(np.prod(shape)), 6, 70).reshape(shape)
    if (ry, rx) == (1, 1):
        w2d = _asym5()
    else:
        w2d = si.uniform_f32((2 * ry + 1) * (2 * rx + 1), -1.0, 1.0, 6, 71).reshape(
            2 * ry + 1, 2 * rx + 1)
    pad = 0.375
    t = fn(x.astype(np.float64), params)
    ref = math.fsum(ndi.correlate(t[f], w2d.astype(np.float64), mode=mode, cval=pad).sum()
                    for f in range(shape[0]))
    got, mag = oracle_mod.chain(op, params, x, ry, rx, w2d=w2d, edge=edge, pad=pad)
    assert abs(got - ref) <= 1e-12 * mag


@pytest.mark.parametrize("op", sorted(CHAIN_MAPS))
def test_chain_closed_forms(oracle_mod, op):
    params, fn = CHAIN_MAPS[op]
    w5 = _asym5()
    wsum = math.fsum(w5.astype(np.float64).reshape(-1))
    x = si.normal_f32(3 * 11 * 13, 6, 72).reshape(3, 11, 13)
    # cyclic borders: every mapped element is read once per tap
    got, mag = oracle_mod.chain(op, params, x, 1, 1, w2d=w5, edge="cyclic")
    want = wsum * math.fsum(fn(x.astype(np.float64), params).reshape(-1))
    assert abs(got - want) <= 1e-12 * mag
    # a constant field stays constant under clamped borders
    c = np.full((2, 5, 6), 0.625, np.float32)
    got, mag = oracle_mod.chain(op, params, c, 1, 1, w2d=w5, edge="clamp")
    want = 2 * 5 * 6 * wsum * float(fn(np.float64(0.625), params))
    assert abs(got - want) <= 1e-12 * mag
    # separable factors act as their exact (binary64) outer product
    wy, wx = si.gaussian_weights(2, 1.0), si.binomial5_weights()
    got, mag = oracle_mod.chain(op, params, x, 2, 2, wy=wy, wx=wx, edge="clamp")
    outer = wy.astype(np.float64)[:, None] * wx.astype(np.float64)[None, :]
    t = fn(x.astype(np.float64), params)
    want = math.fsum(ndi.correlate(t[f], outer, mode="nearest").sum() for f in range(3))
    assert abs(got - want) <= 1e-12 * mag
    # identity map: the chain is the fsum of the MapOverlap oracle's outputs
    if op == "identity":
        for edge in ("clamp", "const", "cyclic"):
            got, mag = oracle_mod.chain(op, params, x, 1, 1, w2d=w5, edge=edge, pad=0.5)
            parts = [oracle_mod.mapoverlap2d(x[f], 1, 1, w2d=w5, edge=edge, pad=0.5)[0]
                     for f in range(3)]
            assert abs(got - math.fsum(np.concatenate([p.reshape(-1) for p in parts]))) \
                <= 1e-12 * mag


@pytest.mark.parametrize("edge", ["clamp", "const", "cyclic"])
def test_chain_grad_finite_differences_16x16(oracle_mod, edge):
    """Central differences of the chain's binary64 forward at 16 x 16 (the
    size the differentiation workload checks at): every element of dx at the
    corners, edges and inside, and both parameters."""
    params = [0.75, -0.25]
    w5 = _asym5()
    rng = si.rng(6, 73)
    # inputs on a 2^-8 grid so that x +- 2^-12 is exact in binary32
    x = (rng.integers(-512, 512, (2, 16, 16)) / 256.0).astype(np.float32)
    g1 = 1.5
    dx, dxm, dp, dpm = oracle_mod.chain_grad("affine_tanh", params, x, 1, 1, g1, w2d=w5,
                                             edge=edge)
    h = 2.0 ** -12
    for f, i, j in [(0, 0, 0), (0, 0, 15), (1, 15, 0), (1, 15, 15), (0, 0, 7), (1, 9, 0),
                    (0, 15, 4), (1, 6, 15), (0, 7, 8), (1, 1, 1), (0, 14, 13)]:
        xp, xm = x.copy(), x.copy()
        xp[f, i, j] += np.float32(h)
        xm[f, i, j] -= np.float32(h)
        lp, _ = oracle_mod.chain("affine_tanh", params, xp, 1, 1, w2d=w5, edge=edge)
        lm, _ = oracle_mod.chain("affine_tanh", params, xm, 1, 1, w2d=w5, edge=edge)
        fd = g1 * (lp - lm) / (2 * h)
        assert abs(dx[f, i, j] - fd) <= 1e-6 * max(1.0, abs(fd)), (f, i, j, dx[f, i, j], fd)
    hp = 1e-6
    for k in range(2):
        pp, pm = list(params), list(params)
        pp[k] += hp
        pm[k] -= hp
        lp, _ = oracle_mod.chain("affine_tanh", pp, x, 1, 1, w2d=w5, edge=edge)
        lm, _ = oracle_mod.chain("affine_tanh", pm, x, 1, 1, w2d=w5, edge=edge)
        fd = g1 * (lp - lm) / (2 * hp)
        assert abs(dp[k] - fd) <= 1e-6 * max(1.0, dpm[k]), (k, dp[k], fd)


@pytest.mark.parametrize("edge", ["clamp", "const", "cyclic"])
def test_chain_grad_composes_the_pinned_adjoints(oracle_mod, edge):
    """The chain's gradient is the MapOverlap adjoint of the broadcast upstream
    gradient, pushed through the Map adjoint (both pinned above)."""
    w5 = _asym5()
    x = si.normal_f32(2 * 9 * 7, 6, 74).reshape(2, 9, 7)
    g1 = -0.75
    for op, params in (("identity", []), ("affine_tanh", [0.75, -0.25])):
        dx, _, dp, _ = oracle_mod.chain_grad(op, params, x, 1, 1, g1, w2d=w5, edge=edge)
        for f in range(2):
            gt, _ = oracle_mod.mapoverlap2d_adjoint(np.full((9, 7), g1, np.float32), 1, 1,
                                                    w2d=w5, edge=edge)
            # the Map adjoint oracle takes g in binary32: gt rounded once (2^-24)
            want, _, _, _ = oracle_mod.map_grad(op, params, x[f], gt.astype(np.float32))
            np.testing.assert_allclose(dx[f].reshape(-1), want, rtol=2e-7, atol=1e-12)
