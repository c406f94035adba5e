"""The host table of the fused call chain Map -> MapOverlap 2D -> Reduce SUM:
for every element of a field, how often (weighted) the neighbourhood map
reads it.  Checked on the CPU, element by element, against the oracle's
reverse mode of the chain with the identity map and a unit upstream gradient,
which is exactly that column sum (A^T 1) in binary64; and the constant pad
term against the oracle chain of a zero field."""
import ctypes as C
import os

import numpy as np
import pytest

import synth_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# SKEL_HOSTTEST_LIB selects another build (the sanitizer build, for one)
LIB = os.environ.get("SKEL_HOSTTEST_LIB") or os.path.join(ROOT, "paper_1405_2915_amd",
                                                          "libskel_hosttest.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libskel_hosttest.so not built (paper_1405_2915_amd/build_lib.py)")
    L = C.CDLL(LIB)
    vp = C.c_void_p
    L.skel_hosttest_chain_weights.argtypes = [C.c_int64, C.c_int64, C.c_int64, vp, vp, vp,
                                              C.c_int, C.c_int, C.c_int, C.c_float, vp,
                                              C.POINTER(C.c_double)]
    return L


EDGES = {"clamp": 0, "const": 1, "cyclic": 2}


def _weights(ry, rx, sep, seed):
    if sep:
        return (None, si.uniform_f32(2 * ry + 1, -1.0, 1.0, 6, seed),
                si.uniform_f32(2 * rx + 1, -1.0, 1.0, 6, seed + 1))
    w = si.uniform_f32((2 * ry + 1) * (2 * rx + 1), -1.0, 1.0, 6, seed)
    return w.reshape(2 * ry + 1, 2 * rx + 1), None, None


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@pytest.mark.parametrize("edge", ["clamp", "const", "cyclic"])
@pytest.mark.parametrize("rows,cols,ry,rx", [(1, 1, 1, 1), (2, 3, 1, 1), (16, 16, 1, 1),
                                             (5, 9, 2, 3), (3, 17, 4, 0), (40, 7, 8, 3),
                                             (9, 9, 4, 4), (1, 50, 0, 8)])
@pytest.mark.parametrize("sep", [False, True])
def test_chain_table_is_the_column_sum(lib, oracle_mod, edge, rows, cols, ry, rx, sep):
    w2d, wy, wx = _weights(ry, rx, sep, 80)
    out = np.empty(rows * cols, np.float32)
    pad_total = C.c_double()
    lib.skel_hosttest_chain_weights(rows, cols, 3, _ptr(w2d), _ptr(wy), _ptr(wx), ry, rx,
                                    EDGES[edge], C.c_float(0.625), _ptr(out),
                                    C.byref(pad_total))
    x = np.zeros((1, rows, cols), np.float32)
    colsum, mag, _, _ = oracle_mod.chain_grad("identity", [], x, ry, rx, 1.0, w2d=w2d, wy=wy,
                                              wx=wx, edge=edge)
    # the table holds the binary64 sum rounded once to binary32
    assert np.all(np.abs(out.astype(np.float64) - colsum.reshape(-1))
                  <= 2.0 ** -24 * mag.reshape(-1) + 1e-30)
    # pad reads: the chain of a zero field over 3 fields is the pad term alone
    want, wmag = oracle_mod.chain("identity", [], np.zeros((3, rows, cols), np.float32), ry, rx,
                                  w2d=w2d, wy=wy, wx=wx, edge=edge, pad=0.625)
    assert abs(pad_total.value - want) <= 1e-12 * wmag
