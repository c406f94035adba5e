"""Skeleton oracle: the plain CPU definition of every skeleton result.

TEST INFRASTRUCTURE ONLY.  The product package never imports this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It loads ``liboracle.so``, which is built from
``oracle.c`` by gcc (``oracle/build.py``) and shares no code with the HIP
library.  Floating point is binary64, integers are exact modular arithmetic of
the output width; the definitions follow the skeleton list of Section III of
Kessler, Dastgeer & Li (arXiv:1405.2915): map, reduce, scan (higher-order
functions) and mapoverlap (a neighbourhood map), plus map-then-reduce.

Operations are named by strings here so that no numeric constant is shared with
the library under test.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SKEL_ORACLE_LIB lets the mutation test load a deliberately broken build
LIB_PATH = os.environ.get("SKEL_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

MAP_OPS = {"identity": 0, "axpy": 1, "affine": 2, "tanh": 3,
           "affine_tanh": 4, "mul": 5, "square": 6}
TWO_INPUT_MAP_OPS = {"axpy", "mul"}
REDUCE_OPS = {"sum": 0, "min": 1, "max": 2}
SCAN_KINDS = {"inclusive": 0, "exclusive": 1, "reverse_inclusive": 2,
              "reverse_exclusive": 3}
EDGES = {"clamp": 0, "const": 1, "cyclic": 2}

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    vp = C.c_void_p
    I64 = C.c_int64
    lib.oracle_set_threads.argtypes = [C.c_int]
    lib.oracle_get_threads.restype = C.c_int
    lib.oracle_map_f32.argtypes = [C.c_int, vp, C.c_int, f32p, vp, I64, f64p]
    lib.oracle_map_f32.restype = C.c_int
    lib.oracle_reduce_f32.argtypes = [C.c_int, f32p, I64]
    lib.oracle_reduce_f32.restype = C.c_double
    lib.oracle_reduce_segments_f32.argtypes = [C.c_int, f32p, I64, i64p, I64, f64p]
    lib.oracle_reduce_segments_f32.restype = C.c_int
    u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
    lib.oracle_fsum_f64.argtypes = [f64p, I64]
    lib.oracle_fsum_f64.restype = C.c_double
    lib.oracle_sum_bf16_exact.argtypes = [u16p, I64]
    lib.oracle_sum_bf16_exact.restype = C.c_double
    lib.oracle_dot_bf16_exact.argtypes = [u16p, u16p, I64]
    lib.oracle_dot_bf16_exact.restype = C.c_double
    lib.oracle_abs_sum_f32.argtypes = [f32p, I64]
    lib.oracle_abs_sum_f32.restype = C.c_double
    lib.oracle_reduce_i32_i32.argtypes = [C.c_int, i32p, I64]
    lib.oracle_reduce_i32_i32.restype = C.c_int32
    lib.oracle_reduce_i32_i64.argtypes = [C.c_int, i32p, I64]
    lib.oracle_reduce_i32_i64.restype = C.c_int64
    lib.oracle_reduce_i64_i64.argtypes = [C.c_int, i64p, I64]
    lib.oracle_reduce_i64_i64.restype = C.c_int64
    lib.oracle_mapreduce_f32.argtypes = [C.c_int, vp, C.c_int, f32p, vp, I64,
                                         C.c_int, C.POINTER(C.c_double)]
    lib.oracle_mapreduce_f32.restype = C.c_double
    lib.oracle_map_grad_f32.argtypes = [C.c_int, vp, C.c_int, f32p, vp, f32p, I64,
                                        f64p, vp, vp, vp]
    lib.oracle_map_grad_f32.restype = C.c_int
    lib.oracle_mapoverlap1d_adjoint_f32.argtypes = [f32p, I64, f32p, C.c_int, C.c_int,
                                                    f64p, vp]
    lib.oracle_mapoverlap1d_adjoint_f32.restype = C.c_int
    lib.oracle_mapoverlap2d_adjoint_f32.argtypes = [f32p, I64, I64, vp, vp, vp, C.c_int,
                                                    C.c_int, C.c_int, f64p, vp]
    lib.oracle_mapoverlap2d_adjoint_f32.restype = C.c_int
    lib.oracle_mapoverlap1d_f32.argtypes = [f32p, I64, f32p, C.c_int, C.c_int,
                                            C.c_float, f64p, vp]
    lib.oracle_mapoverlap1d_f32.restype = C.c_int
    lib.oracle_mapoverlap2d_f32.argtypes = [f32p, I64, I64, vp, vp, vp, C.c_int,
                                            C.c_int, C.c_int, C.c_float, f64p,
                                            vp]
    lib.oracle_mapoverlap2d_f32.restype = C.c_int
    lib.oracle_mapoverlap2d_at_f32.argtypes = [f32p, I64, I64, vp, vp, vp,
                                               C.c_int, C.c_int, C.c_int,
                                               C.c_float, I64, I64,
                                               C.POINTER(C.c_double)]
    lib.oracle_mapoverlap2d_at_f32.restype = C.c_double
    for nm, tin, tout in (("oracle_scan_i32_i32", i32p, i32p),
                          ("oracle_scan_i32_i64", i32p, i64p),
                          ("oracle_scan_i64_i64", i64p, i64p)):
        fn = getattr(lib, nm)
        fn.argtypes = [tin, I64, C.c_int, C.c_int, tout]
        fn.restype = C.c_int
    lib.oracle_chain_f32.argtypes = [C.c_int, vp, C.c_int, f32p, I64, I64, I64, vp, vp, vp,
                                     C.c_int, C.c_int, C.c_int, C.c_float,
                                     C.POINTER(C.c_double)]
    lib.oracle_chain_f32.restype = C.c_double
    lib.oracle_chain_grad_f32.argtypes = [C.c_int, vp, C.c_int, f32p, I64, I64, I64, vp, vp,
                                          vp, C.c_int, C.c_int, C.c_int, C.c_double, f64p,
                                          vp, vp, vp]
    lib.oracle_chain_grad_f32.restype = C.c_int
    lib.oracle_scan_f32.argtypes = [f32p, I64, C.c_int, C.c_int, f64p, vp]
    lib.oracle_scan_f32.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _params(params):
    p = np.ascontiguousarray(np.asarray(params if params is not None else [],
                                        dtype=np.float64))
    return p, len(p)


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def map_f32(op: str, params, x, y=None) -> np.ndarray:
    """out[i] = f(x[i], y[i]) in binary64."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    if y is not None:
        y = np.ascontiguousarray(y, dtype=np.float32)
        assert y.shape == x.shape
    p, np_ = _params(params)
    out = np.empty(x.size, dtype=np.float64)
    rc = lib.oracle_map_f32(MAP_OPS[op], _ptr(p), np_, x.reshape(-1),
                            _ptr(y), x.size, out)
    if rc != 0:
        raise ValueError(f"oracle map: bad op/operands ({op})")
    return out.reshape(x.shape)


def reduce(op: str, x, out_dtype=None):
    """Reduce x with op.  float32 input -> Python float (binary64 sum);
    int32 -> int32 (wrapping) or int64 if out_dtype is int64; int64 -> int64."""
    lib = _load()
    x = np.ascontiguousarray(x).reshape(-1)
    code = REDUCE_OPS[op]
    if x.dtype == np.float32:
        return float(lib.oracle_reduce_f32(code, x, x.size))
    if x.dtype == np.int32:
        if out_dtype is None or np.dtype(out_dtype) == np.int32:
            return int(lib.oracle_reduce_i32_i32(code, x, x.size))
        return int(lib.oracle_reduce_i32_i64(code, x, x.size))
    if x.dtype == np.int64:
        return int(lib.oracle_reduce_i64_i64(code, x, x.size))
    raise TypeError(f"oracle reduce: unsupported dtype {x.dtype}")


def reduce_segments(op: str, x, offsets) -> np.ndarray:
    """out[s] = reduce of x[offsets[s]:offsets[s+1]] in binary64."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    off = np.ascontiguousarray(offsets, dtype=np.int64).reshape(-1)
    out = np.empty(max(off.size - 1, 0), dtype=np.float64)
    rc = lib.oracle_reduce_segments_f32(REDUCE_OPS[op], x, x.size, off, out.size, out)
    if rc != 0:
        raise ValueError("oracle reduce_segments: offsets must be nondecreasing in [0, n]")
    return out


def fsum(x) -> float:
    """Exactly rounded binary64 sum of binary64 values."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    return float(_load().oracle_fsum_f64(x, x.size))


def sum_bf16_exact(bits) -> float:
    """Exactly rounded sum of bfloat16 values given as uint16 bit patterns."""
    b = np.ascontiguousarray(bits, dtype=np.uint16).reshape(-1)
    return float(_load().oracle_sum_bf16_exact(b, b.size))


def dot_bf16_exact(xbits, ybits) -> float:
    """Exactly rounded sum of the products of two bfloat16 vectors."""
    a = np.ascontiguousarray(xbits, dtype=np.uint16).reshape(-1)
    b = np.ascontiguousarray(ybits, dtype=np.uint16).reshape(-1)
    assert a.size == b.size
    return float(_load().oracle_dot_bf16_exact(a, b, a.size))


def abs_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    return float(_load().oracle_abs_sum_f32(x, x.size))


def mapreduce(map_op: str, params, x, y=None, reduce_op: str = "sum"):
    """(r, sum |f|) with r = reduce_op over f(x[i], y[i]), binary64."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    if y is not None:
        y = np.ascontiguousarray(y, dtype=np.float32).reshape(-1)
        assert y.size == x.size
    p, np_ = _params(params)
    mag = C.c_double(0.0)
    r = lib.oracle_mapreduce_f32(MAP_OPS[map_op], _ptr(p), np_, x, _ptr(y),
                                 x.size, REDUCE_OPS[reduce_op], C.byref(mag))
    if np.isnan(r) and not np.isnan(x).any():
        raise ValueError("oracle mapreduce: bad op/operands")
    return float(r), float(mag.value)


def mapoverlap1d(x, w, r: int, edge: str = "clamp", pad: float = 0.0):
    """(out, mag): out[i] = sum_k w[k] x[e(i+k-r)], mag = sum_k |term|."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    w = np.ascontiguousarray(w, dtype=np.float32)
    assert w.size == 2 * r + 1
    out = np.empty(x.size, dtype=np.float64)
    mag = np.empty(x.size, dtype=np.float64)
    rc = lib.oracle_mapoverlap1d_f32(x, x.size, w, r, EDGES[edge], pad, out,
                                     _ptr(mag))
    if rc != 0:
        raise ValueError("oracle mapoverlap1d: bad arguments")
    return out, mag


def _weights2d(w2d, wy, wx, ry, rx):
    if w2d is not None:
        w2d = np.ascontiguousarray(w2d, dtype=np.float32)
        assert w2d.shape == (2 * ry + 1, 2 * rx + 1)
        return w2d, None, None
    wy = np.ascontiguousarray(wy, dtype=np.float32)
    wx = np.ascontiguousarray(wx, dtype=np.float32)
    assert wy.size == 2 * ry + 1 and wx.size == 2 * rx + 1
    return None, wy, wx


def mapoverlap2d(x, ry: int, rx: int, w2d=None, wy=None, wx=None,
                 edge: str = "clamp", pad: float = 0.0):
    """(out, mag) of the 2D neighbourhood map over a rows x cols image."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    assert x.ndim == 2
    w2d, wy, wx = _weights2d(w2d, wy, wx, ry, rx)
    out = np.empty(x.shape, dtype=np.float64)
    mag = np.empty(x.shape, dtype=np.float64)
    rc = lib.oracle_mapoverlap2d_f32(x.reshape(-1), x.shape[0], x.shape[1],
                                     _ptr(w2d), _ptr(wy), _ptr(wx), ry, rx,
                                     EDGES[edge], pad, out.reshape(-1),
                                     _ptr(mag))
    if rc != 0:
        raise ValueError("oracle mapoverlap2d: bad arguments")
    return out, mag


def mapoverlap2d_at(x, ry: int, rx: int, i: int, j: int, w2d=None, wy=None,
                    wx=None, edge: str = "clamp", pad: float = 0.0):
    """(value, mag) of the single output (i, j)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    w2d, wy, wx = _weights2d(w2d, wy, wx, ry, rx)
    mag = C.c_double(0.0)
    v = lib.oracle_mapoverlap2d_at_f32(x.reshape(-1), x.shape[0], x.shape[1],
                                       _ptr(w2d), _ptr(wy), _ptr(wx), ry, rx,
                                       EDGES[edge], pad, int(i), int(j),
                                       C.byref(mag))
    return float(v), float(mag.value)


def map_grad(map_op: str, params, x, g, y=None):
    """Reverse-mode derivative of Map: (dx, dy or None, dparams, dparams_mag),
    binary64, with g = dL/d(out) of the same length as x."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    g = np.ascontiguousarray(g, dtype=np.float32).reshape(-1)
    assert g.size == x.size
    two = map_op in TWO_INPUT_MAP_OPS
    if two:
        y = np.ascontiguousarray(y, dtype=np.float32).reshape(-1)
        assert y.size == x.size
    p, np_ = _params(params)
    dx = np.empty(x.size, dtype=np.float64)
    dy = np.empty(x.size, dtype=np.float64) if two else None
    dp = np.zeros(max(np_, 1), dtype=np.float64)
    dpm = np.zeros(max(np_, 1), dtype=np.float64)
    rc = lib.oracle_map_grad_f32(MAP_OPS[map_op], _ptr(p), np_, x, _ptr(y if two else None),
                                 g, x.size, dx, _ptr(dy), _ptr(dp), _ptr(dpm))
    if rc != 0:
        raise ValueError("oracle map_grad: bad op/operands")
    return dx, dy, dp[:np_], dpm[:np_]


def mapoverlap1d_adjoint(g, w, r: int, edge: str = "clamp"):
    """(dx, mag): the transpose of the 1D neighbourhood map applied to g."""
    lib = _load()
    g = np.ascontiguousarray(g, dtype=np.float32).reshape(-1)
    w = np.ascontiguousarray(w, dtype=np.float32)
    assert w.size == 2 * r + 1
    dx = np.empty(g.size, dtype=np.float64)
    mag = np.empty(g.size, dtype=np.float64)
    if lib.oracle_mapoverlap1d_adjoint_f32(g, g.size, w, r, EDGES[edge], dx, _ptr(mag)):
        raise ValueError("oracle mapoverlap1d_adjoint: bad arguments")
    return dx, mag


def mapoverlap2d_adjoint(g, ry: int, rx: int, w2d=None, wy=None, wx=None,
                         edge: str = "clamp"):
    """(dx, mag): the transpose of the 2D neighbourhood map applied to g."""
    lib = _load()
    g = np.ascontiguousarray(g, dtype=np.float32)
    assert g.ndim == 2
    w2d, wy, wx = _weights2d(w2d, wy, wx, ry, rx)
    dx = np.empty(g.shape, dtype=np.float64)
    mag = np.empty(g.shape, dtype=np.float64)
    if lib.oracle_mapoverlap2d_adjoint_f32(g.reshape(-1), g.shape[0], g.shape[1], _ptr(w2d),
                                           _ptr(wy), _ptr(wx), ry, rx, EDGES[edge],
                                           dx.reshape(-1), _ptr(mag)):
        raise ValueError("oracle mapoverlap2d_adjoint: bad arguments")
    return dx, mag


def scan(x, kind: str = "inclusive", op: str = "sum", out_dtype=None):
    """Prefix combination.  int32 -> int32 (or int64 if out_dtype is int64),
    int64 -> int64, float32 -> (binary64 out, mag)."""
    lib = _load()
    x = np.ascontiguousarray(x).reshape(-1)
    k, o = SCAN_KINDS[kind], REDUCE_OPS[op]
    if x.dtype == np.float32:
        out = np.empty(x.size, dtype=np.float64)
        mag = np.empty(x.size, dtype=np.float64)
        rc = lib.oracle_scan_f32(x, x.size, k, o, out, _ptr(mag))
        if rc:
            raise ValueError("oracle scan: bad kind/op")
        return out, mag
    if x.dtype == np.int32:
        if out_dtype is None or np.dtype(out_dtype) == np.int32:
            out = np.empty(x.size, dtype=np.int32)
            rc = lib.oracle_scan_i32_i32(x, x.size, k, o, out)
        else:
            out = np.empty(x.size, dtype=np.int64)
            rc = lib.oracle_scan_i32_i64(x, x.size, k, o, out)
    elif x.dtype == np.int64:
        out = np.empty(x.size, dtype=np.int64)
        rc = lib.oracle_scan_i64_i64(x, x.size, k, o, out)
    else:
        raise TypeError(f"oracle scan: unsupported dtype {x.dtype}")
    if rc:
        raise ValueError("oracle scan: bad kind/op")
    return out


def scan_rows(x, kind: str = "inclusive", op: str = "sum", out_dtype=None):
    """The scan of Section III applied to every row of a 2D array on its own:
    row r of the result is scan(x[r]).  Same types and returns as scan (for
    float32 input: (binary64 out, mag), both shaped like x)."""
    x = np.asarray(x)
    if x.ndim != 2:
        raise ValueError("oracle scan_rows: x must be 2D")
    res = [scan(x[r], kind, op, out_dtype) for r in range(x.shape[0])]
    if x.dtype == np.float32:
        if not res:
            return np.empty(x.shape), np.empty(x.shape)
        return (np.stack([o for o, _ in res]).reshape(x.shape),
                np.stack([m for _, m in res]).reshape(x.shape))
    if not res:
        return np.empty(x.shape, dtype=np.int64 if out_dtype is not None else x.dtype)
    return np.stack(res).reshape(x.shape)


def chain(map_op: str, params, x, ry: int, rx: int, w2d=None, wy=None, wx=None,
          edge: str = "clamp", pad: float = 0.0):
    """(loss, mag) of the call chain Map -> MapOverlap 2D -> Reduce SUM over
    x of shape (fields, rows, cols) (or (rows, cols): one field), binary64."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    if x.ndim == 2:
        x = x.reshape(1, *x.shape)
    assert x.ndim == 3
    w2d, wy, wx = _weights2d(w2d, wy, wx, ry, rx)
    p, np_ = _params(params)
    mag = C.c_double(0.0)
    v = lib.oracle_chain_f32(MAP_OPS[map_op], _ptr(p), np_, x.reshape(-1), x.shape[0],
                             x.shape[1], x.shape[2], _ptr(w2d), _ptr(wy), _ptr(wx), ry, rx,
                             EDGES[edge], pad, C.byref(mag))
    if np.isnan(v) and not np.isnan(x).any():
        raise ValueError("oracle chain: bad arguments")
    return float(v), float(mag.value)


def chain_grad(map_op: str, params, x, ry: int, rx: int, g1: float = 1.0, w2d=None, wy=None,
               wx=None, edge: str = "clamp"):
    """Reverse mode through the chain: (dx, dx_mag, dparams, dparams_mag),
    binary64, dx shaped like x."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    shape = x.shape
    if x.ndim == 2:
        x = x.reshape(1, *x.shape)
    assert x.ndim == 3
    w2d, wy, wx = _weights2d(w2d, wy, wx, ry, rx)
    p, np_ = _params(params)
    dx = np.empty(x.size, dtype=np.float64)
    dxm = np.empty(x.size, dtype=np.float64)
    dp = np.zeros(max(np_, 1), dtype=np.float64)
    dpm = np.zeros(max(np_, 1), dtype=np.float64)
    rc = lib.oracle_chain_grad_f32(MAP_OPS[map_op], _ptr(p), np_, x.reshape(-1), x.shape[0],
                                   x.shape[1], x.shape[2], _ptr(w2d), _ptr(wy), _ptr(wx), ry,
                                   rx, EDGES[edge], float(g1), dx, _ptr(dxm), _ptr(dp),
                                   _ptr(dpm))
    if rc != 0:
        raise ValueError("oracle chain_grad: bad arguments")
    return dx.reshape(shape), dxm.reshape(shape), dp[:np_], dpm[:np_]
