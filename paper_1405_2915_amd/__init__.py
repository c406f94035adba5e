"""Python binding of libskel: data-parallel skeletons over smart containers on
one MI355X (gfx950).

Each ``skel_*`` function below marshals its arguments and calls the C entry
point of the same name in ``libskel.so`` (declared in ``include/skel.h``);
every step of the computation runs in the library's HIP kernels.  PyTorch is
used only as plumbing: its caching allocator provides device memory and its
current stream orders the calls.  If ``libskel.so`` has not been built, import
of the library fails loudly -- there is no fallback.

Concepts (Kessler, Dastgeer, Li, arXiv:1405.2915): skeletons with several
implementation variants and an execution plan (Section III), smart containers
with lazy host/device coherence (Section IV), asynchronous calls ordered by
container dependences (Section V).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

try:
    # torch ships its own HIP runtime (same soname, libamdhip64.so.7).  Loading
    # it before libskel.so makes the library bind to that one runtime; loaded
    # the other way round, the process would hold two HIP runtimes.
    import torch  # noqa: F401
except ImportError:
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
# SKEL_LIBRARY selects another build of the library (the shrunk-tile scan
# build of the stress test, for one)
LIB_PATH = os.environ.get("SKEL_LIBRARY") or os.path.join(_HERE, "libskel.so")

# ------------------------------------------------------------- skel.h enums
OK, E_INVAL, E_DTYPE, E_SHAPE, E_NOMEM, E_STATE, E_UNSUPPORTED, E_HIP, E_NOINIT, \
    E_TIMEOUT = range(10)
STATUS_NAMES = {0: "SKEL_OK", 1: "SKEL_E_INVAL", 2: "SKEL_E_DTYPE", 3: "SKEL_E_SHAPE",
                4: "SKEL_E_NOMEM", 5: "SKEL_E_STATE", 6: "SKEL_E_UNSUPPORTED",
                7: "SKEL_E_HIP", 8: "SKEL_E_NOINIT", 9: "SKEL_E_TIMEOUT"}
F32, BF16, I32, I64 = 0, 1, 2, 3
HOST, DEVICE = 0, 1
READ, WRITE, RW = 1, 2, 3
EDGE_CLAMP, EDGE_CONST, EDGE_CYCLIC = 0, 1, 2
INCLUSIVE, EXCLUSIVE, REVERSE_INCLUSIVE, REVERSE_EXCLUSIVE = 0, 1, 2, 3
SUM, MIN, MAX = 0, 1, 2
MAP_IDENTITY, MAP_AXPY, MAP_AFFINE, MAP_TANH, MAP_AFFINE_TANH, MAP_MUL, MAP_SQUARE = range(7)
SK_MAP, SK_REDUCE, SK_MAPREDUCE, SK_MAPOVERLAP1D, SK_MAPOVERLAP2D, SK_SCAN, \
    SK_REDUCE_SEGMENTS, SK_MAPOVERLAP1D_BACKWARD, SK_MAPOVERLAP2D_BACKWARD, SK_SCAN_ROWS, \
    SK_MAP_OVERLAP2D_REDUCE = range(11)
VARIANT_AUTO = -1
MAX_RADIUS_1D, MAX_RADIUS_2D = 64, 8

NP_DTYPE = {F32: np.dtype(np.float32), BF16: np.dtype(np.uint16), I32: np.dtype(np.int32),
            I64: np.dtype(np.int64)}
DTYPE_OF_NP = {np.dtype(np.float32): F32, np.dtype(np.int32): I32,
               np.dtype(np.int64): I64}


class SkelError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


class _XferStats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in
                ("h2d", "d2h", "h2d_bytes", "d2h_bytes", "eager_equiv", "acquires")]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


_lib = None
_live = weakref.WeakSet()
_keepalive = []
# handles of containers collected while a graph capture was running on the
# current stream: destroying one may wait for the device and frees pinned host
# memory, which would invalidate the capture, so they are destroyed afterwards
_deferred = []
_shutting_down = False
_device = 0


def load_library(path: str = LIB_PATH):
    """Load libskel.so and declare its C signatures.  Raises ImportError with
    the build command when the library is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1405_2915_amd.build_lib`"
                          " (the HIP library is required, there is no fallback)")
    try:
        lib = C.CDLL(path)
    except OSError as e:  # e.g. an undefined symbol: linked from sources of different ages
        raise ImportError(f"{path} cannot be loaded ({e}): it is older than the sources or "
                          "half rebuilt; rebuild it with "
                          "`python -m paper_1405_2915_amd.build_lib`") from e
    st, vp, i64, i = C.c_int, C.c_void_p, C.c_int64, C.c_int
    dp = C.POINTER(C.c_double)
    fp = C.POINTER(C.c_float)
    sig = {
        "skel_init": (st, [i, C.POINTER(_Allocator)]),
        "skel_finalize": (st, []),
        "skel_sync": (st, [vp]),
        "skel_last_error": (C.c_char_p, []),
        "skel_container_create": (st, [i, i64, i64, vp, C.POINTER(vp)]),
        "skel_container_destroy": (st, [vp]),
        "skel_container_acquire": (st, [vp, i, i, vp, C.POINTER(vp)]),
        "skel_container_release": (st, [vp, i, vp]),
        "skel_container_stats": (st, [vp, C.POINTER(_XferStats)]),
        "skel_container_info": (st, [vp, C.POINTER(i), C.POINTER(i64), C.POINTER(i64)]),
        "skel_map": (st, [i, dp, i, C.POINTER(vp), i, vp, i, vp]),
        "skel_reduce": (st, [i, vp, vp, i, vp]),
        "skel_mapreduce": (st, [i, dp, i, C.POINTER(vp), i, i, vp, i, vp]),
        "skel_mapoverlap1d": (st, [vp, vp, fp, i, i, C.c_float, i, vp]),
        "skel_mapoverlap2d": (st, [vp, vp, fp, fp, fp, i, i, i, C.c_float, i, vp]),
        "skel_scan": (st, [vp, vp, i, i, i, vp]),
        "skel_scan_rows": (st, [vp, vp, i, i, i, vp]),
        "skel_scan_noalloc": (st, [vp, i, vp, i, i64, i, i, vp]),
        "skel_reduce_segments": (st, [i, vp, vp, vp, i, vp]),
        "skel_container_wrap_device": (st, [i, i64, i64, vp, vp, C.POINTER(vp)]),
        "skel_container_acquire_range": (st, [vp, i, i, i64, i64, vp, C.POINTER(vp)]),
        "skel_container_valid_ranges": (st, [vp, i, C.POINTER(i64), i64, C.POINTER(i64)]),
        "skel_map_backward": (st, [i, dp, i, C.POINTER(vp), i, vp, C.POINTER(vp), vp, vp]),
        "skel_mapoverlap1d_backward": (st, [vp, vp, fp, i, i, i, vp]),
        "skel_mapoverlap2d_backward": (st, [vp, vp, fp, fp, fp, i, i, i, i, vp]),
        "skel_mapoverlap2d_fields": (st, [vp, vp, i64, fp, fp, fp, i, i, i, C.c_float, i, vp]),
        "skel_mapoverlap2d_fields_backward": (st, [vp, vp, i64, fp, fp, fp, i, i, i, i, vp]),
        "skel_map_overlap2d_reduce": (st, [i, dp, i, vp, i64, fp, fp, fp, i, i, i, C.c_float,
                                           vp, i, vp]),
        "skel_map_overlap2d_reduce_backward": (st, [i, dp, i, vp, i64, fp, fp, fp, i, i, i, vp,
                                                    vp, vp, i, vp]),
        "skel_variant_count": (i, [i]),
        "skel_variant_name": (C.c_char_p, [i, i]),
        "skel_select_variant": (i, [i, i, i64, i64, i64, i]),
        "skel_load_plan": (st, [C.c_char_p]),
        "skel_clear_plan": (st, []),
    }
    for name, (res, args) in sig.items():
        try:
            fn = getattr(lib, name)
        except AttributeError as e:
            raise ImportError(f"{path} lacks {name}: it is older than the sources; rebuild it "
                              "with `python -m paper_1405_2915_amd.build_lib`") from e
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _L():
    return _lib if _lib is not None else load_library()


def _check(status: int, where: str) -> None:
    if status != OK:
        msg = _lib.skel_last_error()
        raise SkelError(status, where, msg.decode() if msg else "")


# torch's raw current-stream query (no Stream object per call), when present
_RAW_STREAM = getattr(getattr(torch, "_C", None), "_cuda_getCurrentRawStream", None)


def _current_stream() -> int:
    if torch is not None and torch.cuda.is_initialized():
        if _RAW_STREAM is not None:
            return _RAW_STREAM(_device)
        return torch.cuda.current_stream().cuda_stream
    return 0


def _stream(stream) -> int:
    if stream is None:
        return _current_stream()
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


# ----------------------------------------------------------------- runtime
DEFAULT_PLAN = os.path.join(_HERE, "plans", "gfx950.plan")


def skel_init(device: int = 0, allocator: str = "torch", plan: str | None = "default") -> None:
    """Bind the library to `device`.  allocator="torch" routes device memory
    through torch's caching allocator; "hip" uses hipMalloc/hipFree.
    plan: "default" loads the execution plan tuned for this GPU model
    (plans/gfx950.plan, written by paper_1405_2915_amd.autotune) unless
    SKEL_PLAN_FILE names another; a path loads that table; None uses the
    static rules only."""
    _init_device(device, allocator)
    if plan == "default":
        if not os.environ.get("SKEL_PLAN_FILE") and os.path.exists(DEFAULT_PLAN):
            skel_load_plan(DEFAULT_PLAN)
    elif plan is None:
        skel_clear_plan()
    else:
        skel_load_plan(plan)


def _init_device(device: int, allocator: str) -> None:
    global _device
    lib = load_library()
    _device = device
    if allocator == "torch":
        import torch
        torch.cuda.init()
        torch.cuda.set_device(device)

        def _alloc(nbytes, stream, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream or 0))
            except Exception:  # out of memory: report NULL to the library
                return None

        def _free(ptr, stream, ctx):
            if not _shutting_down:
                torch.cuda.caching_allocator_delete(ptr)

        a = _Allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None)
        _keepalive[:] = [a]
        _check(lib.skel_init(device, C.byref(a)), "skel_init")
    elif allocator == "hip":
        _check(lib.skel_init(device, None), "skel_init")
    else:
        raise ValueError(f"unknown allocator {allocator!r}")


def skel_finalize() -> None:
    _check(load_library().skel_finalize(), "skel_finalize")


def _capturing() -> bool:
    return (torch is not None and torch.cuda.is_initialized()
            and torch.cuda.is_current_stream_capturing())


def _destroy_deferred() -> None:
    if _deferred and _lib is not None and not _capturing():
        handles = _deferred[:]
        del _deferred[:]
        for h in handles:
            _lib.skel_container_destroy(C.c_void_p(h))


def skel_sync(stream=None) -> None:
    _destroy_deferred()
    _check(load_library().skel_sync(_stream(stream)), "skel_sync")


def skel_last_error() -> str:
    m = load_library().skel_last_error()
    return m.decode() if m else ""


# -------------------------------------------------------------- containers
class Container:
    """A smart container (Section IV): library-owned host and device copies
    with lazy coherence.  Wraps the opaque skel_container handle."""

    def __init__(self, handle: int, dtype: int, rows: int, cols: int):
        _destroy_deferred()
        self.handle = handle
        self.dtype = dtype
        self.rows = rows
        self.cols = cols
        _live.add(self)

    @property
    def shape(self):
        return (self.rows, self.cols)

    @property
    def n(self) -> int:
        return self.rows * self.cols

    @classmethod
    def from_numpy(cls, arr: np.ndarray, dtype: int | None = None) -> "Container":
        arr = np.ascontiguousarray(arr)
        if dtype is None:
            dtype = DTYPE_OF_NP[arr.dtype]
        if arr.dtype != NP_DTYPE[dtype]:
            raise TypeError(f"array dtype {arr.dtype} does not store skel dtype {dtype}")
        rows, cols = (1, arr.size) if arr.ndim <= 1 else (arr.shape[0], arr.size // arr.shape[0])
        return skel_container_create(dtype, rows, cols, arr)

    @classmethod
    def empty(cls, dtype: int, rows: int, cols: int | None = None) -> "Container":
        if cols is None:
            rows, cols = 1, rows
        return skel_container_create(dtype, rows, cols, None)

    def to_numpy(self) -> np.ndarray:
        """Host acquire for READ (copies from the device only if the host copy
        is stale), copy out, release."""
        ptr = skel_container_acquire(self, HOST, READ)
        try:
            dt = NP_DTYPE[self.dtype]
            out = np.empty(self.n, dtype=dt)
            if self.n:
                C.memmove(out.ctypes.data, ptr, self.n * dt.itemsize)
        finally:
            skel_container_release(self, HOST)
        return out.reshape(self.shape) if self.rows > 1 else out

    def write_numpy(self, arr: np.ndarray) -> None:
        """Host acquire for WRITE (invalidates the device copy), fill, release."""
        dt = NP_DTYPE[self.dtype]
        arr = np.ascontiguousarray(arr, dtype=dt).reshape(-1)
        if arr.size != self.n:
            raise ValueError("size mismatch")
        ptr = skel_container_acquire(self, HOST, WRITE)
        try:
            if self.n:
                C.memmove(ptr, arr.ctypes.data, self.n * dt.itemsize)
        finally:
            skel_container_release(self, HOST)

    def write_range(self, first: int, arr: np.ndarray) -> None:
        """Host WRITE of elements [first, first + len(arr)): only that range
        becomes stale on the device."""
        dt = NP_DTYPE[self.dtype]
        arr = np.ascontiguousarray(arr, dtype=dt).reshape(-1)
        ptr = skel_container_acquire_range(self, HOST, WRITE, first, arr.size)
        try:
            if arr.size:
                C.memmove(ptr, arr.ctypes.data, arr.size * dt.itemsize)
        finally:
            skel_container_release(self, HOST)

    def read_range(self, first: int, count: int) -> np.ndarray:
        """Host READ of elements [first, first + count): copies from the
        device only the stale parts of that range."""
        dt = NP_DTYPE[self.dtype]
        ptr = skel_container_acquire_range(self, HOST, READ, first, count)
        try:
            out = np.empty(count, dtype=dt)
            if count:
                C.memmove(out.ctypes.data, ptr, count * dt.itemsize)
        finally:
            skel_container_release(self, HOST)
        return out

    def valid_ranges(self, place: int):
        return skel_container_valid_ranges(self, place)

    def stats(self) -> dict:
        return skel_container_stats(self)

    def mark_device_written(self, stream=None) -> None:
        """Tell the coherence protocol that the device copy was written outside
        a skeleton call (e.g. by replaying a captured graph): a device write
        acquire/release pair, which makes the host copy stale."""
        skel_container_acquire(self, DEVICE, WRITE, stream)
        skel_container_release(self, DEVICE, stream)

    def destroy(self) -> None:
        if self.handle:
            h, self.handle = self.handle, None
            _check(_L().skel_container_destroy(C.c_void_p(h)), "skel_container_destroy")

    def __del__(self):
        if self.handle and not _shutting_down and _lib is not None:
            if _capturing():  # collected during a graph capture: destroy it afterwards
                _deferred.append(self.handle)
                self.handle = None
                return
            try:
                self.destroy()
            except Exception:
                pass


def _h(c):
    if c is None:
        return None
    if c.__class__ is not Container or not c.handle:
        if not isinstance(c, Container) or not c.handle:
            raise TypeError("expected a live Container")
    return c.handle


def skel_container_create(dtype: int, rows: int, cols: int, host_src=None) -> Container:
    lib = load_library()
    out = C.c_void_p()
    src = None
    if host_src is not None:
        host_src = np.ascontiguousarray(host_src)
        if host_src.size != rows * cols:
            raise ValueError("host_src size does not match rows*cols")
        src = C.c_void_p(host_src.ctypes.data)
    _check(lib.skel_container_create(dtype, rows, cols, src, C.byref(out)),
           "skel_container_create")
    return Container(out.value, dtype, rows, cols)


def skel_container_destroy(c: Container) -> None:
    c.destroy()


def skel_container_wrap_device(dtype: int, rows: int, cols: int, dev_ptr: int,
                               stream=None) -> Container:
    """A container over caller-owned device memory (its valid device copy);
    the library never frees it."""
    out = C.c_void_p()
    _check(load_library().skel_container_wrap_device(dtype, rows, cols, C.c_void_p(dev_ptr),
                                                     _stream(stream),
                                                     C.byref(out)),
           "skel_container_wrap_device")
    return Container(out.value, dtype, rows, cols)


_TORCH_DTYPE = None


def wrap_tensor(t, stream=None) -> Container:
    """A container viewing a contiguous CUDA tensor's memory (f32, bf16 bits as
    int16/bfloat16, int32, int64); the tensor must outlive the container."""
    import torch
    global _TORCH_DTYPE
    if _TORCH_DTYPE is None:
        _TORCH_DTYPE = {torch.float32: F32, torch.bfloat16: BF16, torch.int32: I32,
                        torch.int64: I64}
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("wrap_tensor needs a contiguous CUDA tensor")
    if t.dtype not in _TORCH_DTYPE:
        raise TypeError(f"unsupported tensor dtype {t.dtype}")
    # leading axis = rows; an empty tensor (any shape) is a 1 x 0 container
    rows, cols = ((1, t.numel()) if t.dim() <= 1 or t.numel() == 0
                  else (t.shape[0], t.numel() // t.shape[0]))
    return skel_container_wrap_device(_TORCH_DTYPE[t.dtype], rows, cols, t.data_ptr(), stream)


def skel_container_acquire(c: Container, place: int, access: int, stream=None) -> int:
    ptr = C.c_void_p()
    _check(_L().skel_container_acquire(_h(c), place, access, _stream(stream),
                                       C.byref(ptr)), "skel_container_acquire")
    return ptr.value or 0


def skel_container_acquire_range(c: Container, place: int, access: int, first: int,
                                 count: int, stream=None) -> int:
    """Acquire elements [first, first + count) only; returns the address of
    element `first` of the copy at `place`."""
    ptr = C.c_void_p()
    _check(_L().skel_container_acquire_range(_h(c), place, access, int(first), int(count),
                                             _stream(stream), C.byref(ptr)),
           "skel_container_acquire_range")
    return ptr.value or 0


def skel_container_valid_ranges(c: Container, place: int):
    """[(first, last), ...] element ranges that are current at `place`."""
    cnt = C.c_int64()
    _check(_L().skel_container_valid_ranges(_h(c), place, None, 0, C.byref(cnt)),
           "skel_container_valid_ranges")
    buf = (C.c_int64 * (2 * max(cnt.value, 1)))()
    _check(_L().skel_container_valid_ranges(_h(c), place, buf, cnt.value, C.byref(cnt)),
           "skel_container_valid_ranges")
    return [(buf[2 * k], buf[2 * k + 1]) for k in range(cnt.value)]


def skel_container_release(c: Container, place: int, stream=None) -> None:
    _check(_L().skel_container_release(_h(c), place, _stream(stream)),
           "skel_container_release")


def skel_container_stats(c: Container) -> dict:
    s = _XferStats()
    _check(_L().skel_container_stats(_h(c), C.byref(s)), "skel_container_stats")
    return {k: int(getattr(s, k)) for k, _ in _XferStats._fields_}


def skel_container_info(c: Container):
    dt, r, cc = C.c_int(), C.c_int64(), C.c_int64()
    _check(_L().skel_container_info(_h(c), C.byref(dt), C.byref(r), C.byref(cc)),
           "skel_container_info")
    return dt.value, r.value, cc.value


# --------------------------------------------------------------- skeletons
_PARAM_ARRAYS = {}  # parameter lists of plain Python numbers -> their ctypes arrays


def _params(params):
    """(keep-alive object, pointer argument, count) for a parameter list."""
    if params is None or len(params) == 0:
        return None, None, 0
    key = tuple(params)
    hit = _PARAM_ARRAYS.get(key)
    if hit is not None:
        return hit
    vals = [float(v) for v in key]
    arr = (C.c_double * len(vals))(*vals)
    hit = (arr, arr, len(vals))
    # only plain numbers are keys (a tensor would hash by identity, not value);
    # the library copies the values at call time, so a shared array is safe
    if len(_PARAM_ARRAYS) < 256 and all(v.__class__ in (int, float) for v in key):
        _PARAM_ARRAYS[key] = hit
    return hit


_HANDLE_ARRAYS = {k: C.c_void_p * k for k in range(1, 9)}


def _handles(cs):
    hs = [_h(c) for c in cs]
    k = len(hs)
    arr = (_HANDLE_ARRAYS.get(k) or (C.c_void_p * k))(*hs)
    return arr, k


def _floats(w):
    if w is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(w, dtype=np.float32)).reshape(-1)
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def skel_map(op: int, params, ins, out: Container, variant: int = VARIANT_AUTO,
             stream=None) -> None:
    """Map: out[i] = f(ins[0][i], ins[1][i])."""
    arr, nin = _handles(ins)
    ho = _h(out)
    p, pp, np_ = _params(params)
    _check(_L().skel_map(op, pp, np_, arr, nin, ho, variant, _stream(stream)), "skel_map")


def skel_reduce(op: int, inp: Container, out1: Container, variant: int = VARIANT_AUTO,
                stream=None) -> None:
    _check(_L().skel_reduce(op, _h(inp), _h(out1), variant, _stream(stream)),
           "skel_reduce")


def skel_mapreduce(map_op: int, params, ins, op: int, out1: Container,
                   variant: int = VARIANT_AUTO, stream=None) -> None:
    arr, nin = _handles(ins)
    p, pp, np_ = _params(params)
    _check(_L().skel_mapreduce(map_op, pp, np_, arr, nin, op, _h(out1), variant,
                               _stream(stream)), "skel_mapreduce")


def skel_mapoverlap1d(inp: Container, out: Container, w, radius: int,
                      edge: int = EDGE_CLAMP, pad: float = 0.0,
                      variant: int = VARIANT_AUTO, stream=None) -> None:
    wa, wp = _floats(w)
    if wa is None or wa.size != 2 * radius + 1:
        raise ValueError("w must hold 2*radius+1 weights")
    _check(_L().skel_mapoverlap1d(_h(inp), _h(out), wp, radius, edge, pad, variant,
                                  _stream(stream)), "skel_mapoverlap1d")


def _weights_2d(w2d, wy, wx, ry, rx):
    """ctypes pointers for the 2D weights (and the arrays they point into,
    which the caller keeps alive for the call) and the radii."""
    a2, p2 = _floats(w2d)
    ay, py = _floats(wy)
    ax, px = _floats(wx)
    if w2d is not None:
        shp = np.shape(w2d)
        ry = (shp[0] - 1) // 2 if ry is None else ry
        rx = (shp[1] - 1) // 2 if rx is None else rx
        if a2.size != (2 * ry + 1) * (2 * rx + 1):
            raise ValueError("w2d must be (2ry+1) x (2rx+1)")
    else:
        if ay is None or ax is None:
            raise ValueError("need w2d or both wy and wx")
        ry = (ay.size - 1) // 2 if ry is None else ry
        rx = (ax.size - 1) // 2 if rx is None else rx
        if ay.size != 2 * ry + 1 or ax.size != 2 * rx + 1:
            raise ValueError("wy / wx sizes must be 2r+1")
    return (p2, py, px), (a2, ay, ax), ry, rx


def skel_mapoverlap2d(inp: Container, out: Container, w2d=None, wy=None, wx=None,
                      ry: int | None = None, rx: int | None = None,
                      edge: int = EDGE_CLAMP, pad: float = 0.0,
                      variant: int = VARIANT_AUTO, stream=None) -> None:
    (p2, py, px), keep, ry, rx = _weights_2d(w2d, wy, wx, ry, rx)
    _check(_L().skel_mapoverlap2d(_h(inp), _h(out), p2, py, px, ry, rx, edge, pad, variant,
                                  _stream(stream)), "skel_mapoverlap2d")


def skel_mapoverlap2d_fields(inp: Container, out: Container, fields: int, w2d=None, wy=None,
                             wx=None, ry: int | None = None, rx: int | None = None,
                             edge: int = EDGE_CLAMP, pad: float = 0.0,
                             variant: int = VARIANT_AUTO, stream=None) -> None:
    """The 2D map on each of `fields` equally shaped images stored back to back
    in (fields * H, W) containers."""
    (p2, py, px), keep, ry, rx = _weights_2d(w2d, wy, wx, ry, rx)
    _check(_L().skel_mapoverlap2d_fields(_h(inp), _h(out), fields, p2, py, px, ry, rx, edge,
                                         pad, variant, _stream(stream)),
           "skel_mapoverlap2d_fields")


def skel_scan(inp: Container, out: Container, kind: int = INCLUSIVE, op: int = SUM,
              variant: int = VARIANT_AUTO, stream=None) -> None:
    _check(_L().skel_scan(_h(inp), _h(out), kind, op, variant, _stream(stream)),
           "skel_scan")


def skel_scan_noalloc(in_ptr: int, din: int, out_ptr: int, dout: int, n: int,
                      kind: int = INCLUSIVE, op: int = SUM, stream=None) -> None:
    """Scan of n elements at device address in_ptr into out_ptr (caller-owned
    device memory, e.g. tensors' data_ptr()) that allocates nothing: the
    library's fixed per-GPU array holds the tile totals.  Forward kinds only;
    at most 2^30 elements (2^29 for int64 input)."""
    _check(_L().skel_scan_noalloc(C.c_void_p(in_ptr), din, C.c_void_p(out_ptr), dout, int(n),
                                  kind, op, _stream(stream)), "skel_scan_noalloc")


def skel_scan_rows(inp: Container, out: Container, kind: int = INCLUSIVE, op: int = SUM,
                   variant: int = VARIANT_AUTO, stream=None) -> None:
    """Scan every row of a (rows, cols) container on its own."""
    _check(_L().skel_scan_rows(_h(inp), _h(out), kind, op, variant,
                               _stream(stream)), "skel_scan_rows")


def skel_reduce_segments(op: int, inp: Container, offsets: Container, out: Container,
                         variant: int = VARIANT_AUTO, stream=None) -> None:
    """out[s] = op over inp[offsets[s]:offsets[s+1]] for every segment s."""
    _check(_L().skel_reduce_segments(op, _h(inp), _h(offsets), _h(out), variant,
                                     _stream(stream)), "skel_reduce_segments")


def skel_map_backward(map_op: int, params, ins, g: Container, grad_ins,
                      grad_params: Container | None = None, stream=None) -> None:
    """grad_ins[k] = g * df/d(input k); grad_params[k] = sum_i g df/dp_k.
    g has n elements or one (broadcast)."""
    arr, nin = _handles(ins)
    garr, ng = _handles(grad_ins)
    p, pp, np_ = _params(params)
    if ng != nin:
        raise ValueError("one gradient output per input")
    _check(_L().skel_map_backward(map_op, pp, np_, arr, nin, _h(g), garr, _h(grad_params),
                                  _stream(stream)), "skel_map_backward")


def skel_mapoverlap1d_backward(g: Container, grad_in: Container, w, radius: int,
                               edge: int = EDGE_CLAMP, variant: int = VARIANT_AUTO,
                               stream=None) -> None:
    wa, wp = _floats(w)
    if wa is None or wa.size != 2 * radius + 1:
        raise ValueError("w must hold 2*radius+1 weights")
    _check(_L().skel_mapoverlap1d_backward(_h(g), _h(grad_in), wp, radius, edge, variant,
                                           _stream(stream)),
           "skel_mapoverlap1d_backward")


def skel_mapoverlap2d_backward(g: Container, grad_in: Container, w2d=None, wy=None, wx=None,
                               ry: int | None = None, rx: int | None = None,
                               edge: int = EDGE_CLAMP, variant: int = VARIANT_AUTO,
                               stream=None) -> None:
    (p2, py, px), keep, ry, rx = _weights_2d(w2d, wy, wx, ry, rx)
    _check(_L().skel_mapoverlap2d_backward(_h(g), _h(grad_in), p2, py, px, ry, rx, edge,
                                           variant, _stream(stream)),
           "skel_mapoverlap2d_backward")


def skel_mapoverlap2d_fields_backward(g: Container, grad_in: Container, fields: int, w2d=None,
                                      wy=None, wx=None, ry: int | None = None,
                                      rx: int | None = None, edge: int = EDGE_CLAMP,
                                      variant: int = VARIANT_AUTO, stream=None) -> None:
    """The 2D transpose on each of `fields` equally shaped images."""
    (p2, py, px), keep, ry, rx = _weights_2d(w2d, wy, wx, ry, rx)
    _check(_L().skel_mapoverlap2d_fields_backward(_h(g), _h(grad_in), fields, p2, py, px, ry,
                                                  rx, edge, variant,
                                                  _stream(stream)),
           "skel_mapoverlap2d_fields_backward")


def skel_map_overlap2d_reduce(map_op: int, params, inp: Container, fields: int, out1: Container,
                              w2d=None, wy=None, wx=None, ry: int | None = None,
                              rx: int | None = None, edge: int = EDGE_CLAMP, pad: float = 0.0,
                              variant: int = VARIANT_AUTO, stream=None) -> None:
    """out1[0] = sum of the 2D neighbourhood map of f(inp) over every field (the
    chain Map -> MapOverlap 2D -> Reduce SUM as one call)."""
    (p2, py, px), keep, ry, rx = _weights_2d(w2d, wy, wx, ry, rx)
    p, pp, np_ = _params(params)
    _check(_L().skel_map_overlap2d_reduce(map_op, pp, np_, _h(inp), fields, p2, py, px, ry, rx,
                                          edge, pad, _h(out1), variant, _stream(stream)),
           "skel_map_overlap2d_reduce")


def skel_map_overlap2d_reduce_backward(map_op: int, params, inp: Container, fields: int,
                                       g1: Container, grad_in: Container,
                                       grad_params: Container | None = None, w2d=None, wy=None,
                                       wx=None, ry: int | None = None, rx: int | None = None,
                                       edge: int = EDGE_CLAMP, variant: int = VARIANT_AUTO,
                                       stream=None) -> None:
    """grad_in = g1 * d(chain)/d(inp), grad_params = g1 * d(chain)/d(params)."""
    (p2, py, px), keep, ry, rx = _weights_2d(w2d, wy, wx, ry, rx)
    p, pp, np_ = _params(params)
    _check(_L().skel_map_overlap2d_reduce_backward(map_op, pp, np_, _h(inp), fields, p2, py, px,
                                                   ry, rx, edge, _h(g1), _h(grad_in),
                                                   _h(grad_params), variant, _stream(stream)),
           "skel_map_overlap2d_reduce_backward")


def skel_variant_count(skeleton: int) -> int:
    return load_library().skel_variant_count(skeleton)


def skel_variant_name(skeleton: int, variant: int):
    n = load_library().skel_variant_name(skeleton, variant)
    return n.decode() if n else None


def skel_select_variant(skeleton: int, dtype: int, n: int, rows: int = 1, cols: int | None = None,
                        aux: int = 0) -> int:
    """aux: the radius for MapOverlap1D; for MapOverlap2D, separable + 2 * max(ry, rx)
    (separable: 1 when the weights are given as factors); 1 for reverse scans."""
    return load_library().skel_select_variant(skeleton, dtype, n, rows,
                                              n if cols is None else cols, aux)


def skel_load_plan(path: str) -> None:
    _check(load_library().skel_load_plan(path.encode()), "skel_load_plan")


def skel_clear_plan() -> None:
    _check(load_library().skel_clear_plan(), "skel_clear_plan")


def variant_index(skeleton: int, name: str) -> int:
    for v in range(skel_variant_count(skeleton)):
        if skel_variant_name(skeleton, v) == name:
            return v
    raise KeyError(name)


@atexit.register
def _shutdown():
    global _shutting_down
    if _lib is None:
        return
    for c in list(_live):
        try:
            c.destroy()
        except Exception:
            pass
    for h in _deferred:
        _lib.skel_container_destroy(C.c_void_p(h))
    del _deferred[:]
    try:
        _L().skel_finalize()
    except Exception:
        pass
    _shutting_down = True


# Load eagerly when built, so a broken library fails at import.  When it is not
# built, or was built from older sources, the package still imports (build_lib
# lives in it) and every call raises ImportError until it is rebuilt.
if os.path.exists(LIB_PATH):
    try:
        load_library()
    except ImportError as _e:
        if "older than the sources" not in str(_e):
            raise
