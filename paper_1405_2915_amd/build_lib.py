"""Build libskel.so (HIP, gfx950) in-tree, and the CPU-only host-logic test
library used by the container-protocol tests.

    python -m paper_1405_2915_amd.build_lib [-v]

Every HIP source is compiled by hipcc for gfx950 only, with packed-FP32
instruction generation disabled.  The container protocol, the execution plan
and error reporting are plain C++ and are also compiled by g++, together with
a host-memory fake of the copy backend, into libskel_hosttest.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libskel.so")
HOSTTEST_LIB = os.path.join(PKG, "libskel_hosttest.so")

HIP_SOURCES = ["common.cpp", "container.cpp", "dispatch.cpp", "runtime.cpp", "chain_table.cpp",
               "skeletons.cpp", "k_map.hip", "k_reduce.hip", "k_scan.hip",
               "k_overlap.hip", "k_segments.hip", "k_grad.hip", "k_chain.hip"]
HOST_SOURCES = ["common.cpp", "container.cpp", "dispatch.cpp", "chain_table.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Wall", "-Wno-unused-function",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{INC}", f"-I{CSRC}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n"
                           f"{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)


def build_hip(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    cmds = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([HIPCC] + HIP_FLAGS + lang + ["-c", os.path.join(CSRC, src),
                                                  "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
         verbose)
    os.replace(tmp, LIB)
    return LIB


HOSTTEST_SAN_LIB = os.path.join(PKG, "libskel_hosttest_san.so")
# AddressSanitizer and UndefinedBehaviorSanitizer for the host-only builds
SANITIZE = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
            "-fno-sanitize-recover=undefined"]


def build_hosttest(verbose: bool = False, sanitize: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in HOST_SOURCES]
    srcs.append(os.path.join(ROOT, "tests", "host", "fake_backend.cpp"))
    out = HOSTTEST_SAN_LIB if sanitize else HOSTTEST_LIB
    tmp = out + ".tmp"
    _run(["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-Wall"] +
         (SANITIZE if sanitize else []) + [f"-I{INC}", f"-I{CSRC}", "-o", tmp] + srcs, verbose)
    os.replace(tmp, out)
    return out


SCAN_STRESS_LIB = os.path.join(PKG, "libskel_scan_w2.so")


def build_scan_stress(verbose: bool = False) -> str:
    """libskel_scan_w2.so: the library with the scan tiles shrunk to two
    wavefronts (4096 elements for 4-byte inputs instead of 32768), eight times
    as many tiles and a deeper decoupled look-back, for the look-back stress
    test.  The other objects are those of the product build."""
    obj = os.path.join(BUILD, "k_scan.hip.w2.o")
    _run([HIPCC] + HIP_FLAGS + ["-DSKEL_SCAN_WAVES=2", "-x", "hip", "-c",
                                os.path.join(CSRC, "k_scan.hip"), "-o", obj], verbose)
    objs = [os.path.join(BUILD, s + ".o") for s in HIP_SOURCES if s != "k_scan.hip"] + [obj]
    tmp = SCAN_STRESS_LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, SCAN_STRESS_LIB)
    return SCAN_STRESS_LIB


def build(verbose: bool = False) -> None:
    build_hip(verbose)
    build_scan_stress(verbose)
    build_hosttest(verbose)


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        # the container protocol, plan and chain table (and the oracle) built
        # with the sanitizers; see sanitize_env() for running the CPU tests
        print(build_hosttest("-v" in sys.argv, sanitize=True))
        sys.path.insert(0, ROOT)
        from oracle import build as oracle_build
        print(oracle_build.build("-v" in sys.argv, sanitize=True))
    else:
        build(verbose="-v" in sys.argv)
        print(LIB)
