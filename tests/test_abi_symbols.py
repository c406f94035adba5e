"""libskel.so loads without a GPU and exports every function include/skel.h
declares; the Python binding mirrors each of them by name."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skel.h")
LIB = os.path.join(ROOT, "paper_1405_2915_amd", "libskel.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(skel_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("skel_init", "skel_container_create", "skel_container_acquire",
                 "skel_container_release", "skel_container_destroy", "skel_map",
                 "skel_reduce", "skel_mapreduce", "skel_mapoverlap1d",
                 "skel_mapoverlap2d", "skel_scan", "skel_sync", "skel_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libskel.so not built"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (skel_\w+)", out))
    assert set(declared_functions()) <= exported


def test_library_is_gfx950_code_object():
    # the embedded offload bundle names its target; only gfx950 is built
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data
    for other in (b"--gfx942", b"--gfx90a", b"--gfx1100"):
        assert other not in data


def test_binding_mirrors_names():
    import paper_1405_2915_amd as skel
    for n in declared_functions():
        assert hasattr(skel, n), n


def test_calls_without_init_fail_cleanly():
    import paper_1405_2915_amd as skel
    lib = skel.load_library()
    out = ctypes.c_void_p()
    st = lib.skel_container_create(skel.F32, 1, 4, None, ctypes.byref(out))
    assert st == skel.E_NOINIT
    assert b"skel_init" in lib.skel_last_error()
    assert lib.skel_reduce(0, None, None, -1, None) == skel.E_NOINIT


def test_unloadable_library_raises_import_error(tmp_path):
    """A library the dynamic loader refuses (here: an undefined symbol, as a
    half-finished rebuild leaves it) turns into ImportError, which the package
    import tolerates so that the build step inside it can still run."""
    import paper_1405_2915_amd as skel
    src = tmp_path / "stale.c"
    src.write_text("extern int symbol_from_elsewhere(void);\n"
                   "int skel_init(void) { return symbol_from_elsewhere(); }\n")
    so = tmp_path / "libstale.so"
    subprocess.run(["gcc", "-shared", "-fPIC", "-Wl,-z,now", "-o", str(so), str(src)],
                   check=True)
    saved = skel._lib
    skel._lib = None
    try:
        with pytest.raises(ImportError, match="older than the sources"):
            skel.load_library(str(so))
    finally:
        skel._lib = saved
