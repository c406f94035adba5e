"""Benchmark of the skeleton hot path on one MI355X.

One step = one pass over every skeleton on a fixed, HBM-resident synthetic
workload (the large configuration; every call goes through the execution
plan, and every operand through the container protocol, which copies nothing
once the device copies are valid):

  Map        saxpy y <- 2.5 x + y, in place          x, y  f32[2^26]
  MapOverlap 1D 5-point binomial, clamp             z     f32[2^26]
  Scan       exclusive, int32 -> int64               s     i32[2^27]
  MapReduce  dot(x, y)                               x, y  f32[2^26]
  MapOverlap 2D 9x9 separable Gaussian (sigma 2)     img   f32[4096][4096]
  Reduce     sum of the 1D stencil's output          f32[2^26]

The order keeps consecutive calls on different data, so no call finds its
inputs in the 256 MiB Infinity Cache.  Reported: whole-step throughput in
algorithmic GB/s (inputs read once + outputs written once), each skeleton's
kernel time from HIP events on the launch stream, the roofline of the
dominant kernel (the scan), a measured copy-kernel ceiling, the speedup over
the fixed plain variants, and the CPU oracle timed on a sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_VEC = 1 << 26
N_SCAN = 1 << 27
IMG = 4096

# algorithmic bytes per call
BYTES = {
    "map_saxpy": 12 * N_VEC,
    "mapoverlap1d_5pt": 8 * N_VEC,
    "scan_excl_i32_i64": 12 * N_SCAN,
    "mapreduce_dot": 8 * N_VEC,
    "mapoverlap2d_9x9": 8 * IMG * IMG,
    "reduce_sum": 4 * N_VEC,
}
ORDER = list(BYTES)
PLAIN = {"map_saxpy": "M0_scalar", "mapoverlap1d_5pt": "O1a_direct",
         "scan_excl_i32_i64": "S1_reduce_then_scan", "mapreduce_dot": "MR0_unfused",
         "mapoverlap2d_9x9": "O2a_direct", "reduce_sum": "R1_two_pass"}
DOMINANT = "scan_excl_i32_i64"
# variants bulk selection may give each call of the step (the single-workgroup
# forms, which would take one CU at these sizes, the order-dependent atomic
# Reduce and the slow direct 2D stencils are left out)
STEP_SITES = {
    "map_saxpy": ["M0_scalar", "M1_vec4", "M2_vec4x4_nt"],
    "mapoverlap1d_5pt": ["O1a_direct", "O1b_lds_tile", "O1c_shuffle"],
    "scan_excl_i32_i64": ["S1_reduce_then_scan", "S2_decoupled_lookback",
                          "S3_persistent_lookback"],
    "mapreduce_dot": ["MR1_fused_two_pass", "MR2_fused_ticket", "MR4_compensated",
                      "MR5_pairwise", "MR6_fused_gather"],
    "mapoverlap2d_9x9": ["O2c_lds_separable", "O2d_separable_l1", "O2e_march"],
    "reduce_sum": ["R1_two_pass", "R2_ticket", "R4_compensated", "R5_pairwise", "R6_gather"],
}
# kernels of each Scan variant (int32 -> int64, exclusive sum)
SCAN_KERNELS = {
    "S0_single_wg": "scan_single<int32 -> int64, exclusive sum>",
    "S1_reduce_then_scan": "scan_tile_totals + scan_tile_offsets + scan_tile_apply",
    "S2_decoupled_lookback": "scan_lookback<int32 -> int64, exclusive sum>",
    "S3_persistent_lookback": "scan_lookback_persist<int32 -> int64, exclusive sum>",
}
# device sources of the dominant kernel: its traffic figure holds only while
# their combined hash is the one the counters were taken on
KERNEL_SRC = {"scan_excl_i32_i64": ("k_scan.hip", "kcommon.hpp", "kepoch.hpp")}


def source_hash(name):
    """sha256 over the named kernel's device sources, in the listed order."""
    h = hashlib.sha256()
    for src in KERNEL_SRC[name]:
        with open(os.path.join(ROOT, "paper_1405_2915_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    model = platform.processor() or "?"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


class Workload:
    def __init__(self, skel):
        import synth_inputs as si
        self.skel = skel
        log("generating inputs")
        self.x_h = si.normal_f32(N_VEC, 1, 0)
        self.y_h = si.normal_f32(N_VEC, 1, 1)
        self.z_h = si.uniform_f32(N_VEC, -1.0, 1.0, 0, 3)
        self.s_h = si.int_uniform_i32(N_SCAN, 1000, 1, 2)
        self.img_h = si.uniform_f32(IMG * IMG, 0.0, 1.0, 1, 0).reshape(IMG, IMG)
        self.w5 = si.binomial5_weights()
        self.g9 = si.gaussian_weights(4, 2.0)
        C = skel.Container
        self.x, self.y = C.from_numpy(self.x_h), C.from_numpy(self.y_h)
        self.z = C.from_numpy(self.z_h)
        self.o1 = C.empty(skel.F32, N_VEC)
        self.s = C.from_numpy(self.s_h)
        self.so = C.empty(skel.I64, N_SCAN)
        self.img = C.from_numpy(self.img_h)
        self.imo = C.empty(skel.F32, IMG, IMG)
        self.r_dot = C.empty(skel.F32, 1)
        self.r_sum = C.empty(skel.F32, 1)

    def calls(self, variants=None):
        """(name, thunk) for one step; variants maps name -> forced variant."""
        sk = self.skel
        v = lambda name: -1 if variants is None else variants[name]
        return [
            ("map_saxpy", lambda: sk.skel_map(sk.MAP_AXPY, [2.5], [self.x, self.y], self.y,
                                              variant=v("map_saxpy"))),
            ("mapoverlap1d_5pt", lambda: sk.skel_mapoverlap1d(
                self.z, self.o1, self.w5, 2, sk.EDGE_CLAMP, variant=v("mapoverlap1d_5pt"))),
            ("scan_excl_i32_i64", lambda: sk.skel_scan(self.s, self.so, sk.EXCLUSIVE, sk.SUM,
                                                       variant=v("scan_excl_i32_i64"))),
            ("mapreduce_dot", lambda: sk.skel_mapreduce(sk.MAP_MUL, None, [self.x, self.y],
                                                        sk.SUM, self.r_dot,
                                                        variant=v("mapreduce_dot"))),
            ("mapoverlap2d_9x9", lambda: sk.skel_mapoverlap2d(
                self.img, self.imo, wy=self.g9, wx=self.g9, edge=sk.EDGE_CLAMP,
                variant=v("mapoverlap2d_9x9"))),
            ("reduce_sum", lambda: sk.skel_reduce(sk.SUM, self.o1, self.r_sum,
                                                  variant=v("reduce_sum"))),
        ]

    def selected(self):
        sk = self.skel
        return {
            "map_saxpy": sk.skel_select_variant(sk.SK_MAP, sk.F32, N_VEC),
            "mapoverlap1d_5pt": sk.skel_select_variant(sk.SK_MAPOVERLAP1D, sk.F32, N_VEC, aux=2),
            "scan_excl_i32_i64": sk.skel_select_variant(sk.SK_SCAN, sk.I32, N_SCAN),
            "mapreduce_dot": sk.skel_select_variant(sk.SK_MAPREDUCE, sk.F32, N_VEC),
            "mapoverlap2d_9x9": sk.skel_select_variant(sk.SK_MAPOVERLAP2D, sk.F32, IMG * IMG,
                                                       IMG, IMG, aux=1 + 2 * 4),
            "reduce_sum": sk.skel_select_variant(sk.SK_REDUCE, sk.F32, N_VEC),
        }


def run_steps(torch, calls, steps, with_events):
    """Run `steps` steps; return (elapsed seconds, {name: [kernel ms, ...]}).
    with_events: False, True (every call), or a set of call names to bracket
    with HIP events on the launch stream (each event marker costs GPU time,
    so the timed region brackets only the kernel it reports)."""
    stream = torch.cuda.current_stream()
    ev = {name: [] for name, _ in calls}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for name, fn in calls:
            if with_events is True or (with_events and name in with_events):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn()
                b.record(stream)
                ev[name].append((a, b))
            else:
                fn()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = {k: [a.elapsed_time(b) for a, b in v] for k, v in ev.items()}
    return el, ms


def copy_ceiling(skel, torch, reps=10):
    """Plain device copy (Map identity, 16-byte vectors) of 2^27 floats."""
    n = 1 << 27
    a = skel.Container.from_numpy(np.ones(n, np.float32))
    b = skel.Container.empty(skel.F32, n)
    v = skel.variant_index(skel.SK_MAP, "M2_vec4x4_nt")
    skel.skel_map(skel.MAP_IDENTITY, None, [a], b, variant=v)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        skel.skel_map(skel.MAP_IDENTITY, None, [a], b, variant=v)
        e1.record(st)
        times.append((e0, e1))
    torch.cuda.synchronize()
    ms = float(np.median([x.elapsed_time(y) for x, y in times]))
    a.destroy()
    b.destroy()
    return 8 * n / (ms * 1e-3) / 1e9, ms


def isolated(skel, torch, wl, name, reps, before):
    """One skeleton of the step alone, `reps` times, each call preceded by a
    pass over a separate 1 GiB buffer that replaces the Infinity Cache's
    contents: `before` = "read" (plain loads, torch's sum: the cache holds
    clean lines; the library's Reduce kernels load non-temporally and leave
    most of the cache in place) or "write" (a Map writing it with plain
    stores: the cache holds dirty lines, as after the step's scan).  Kernel
    time from HIP events around the call on the launch stream."""
    n = 1 << 28
    buf = skel.Container.from_numpy(np.zeros(n, np.float32)) if before == "write" else None
    flush = torch.zeros(n, dtype=torch.float32, device="cuda") if before == "read" else None
    dst = skel.Container.empty(skel.F32, n) if before == "write" else None
    m1 = skel.variant_index(skel.SK_MAP, "M1_vec4")  # plain 16-byte stores
    calls = wl.calls()
    for _, c in calls:  # one whole step first: every operand then holds valid data
        c()
    call = dict(calls)[name]
    st = torch.cuda.current_stream()
    evs = []
    for _ in range(reps + 1):
        if before == "write":
            skel.skel_map(skel.MAP_IDENTITY, None, [buf], dst, variant=m1)
        else:
            flush.sum()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        call()
        e1.record(st)
        evs.append((e0, e1))
    torch.cuda.synchronize()
    us = float(np.median([a.elapsed_time(b) for a, b in evs[1:]])) * 1e3
    for c in (buf, dst):
        if c is not None:
            c.destroy()
    return us


def traffic_from_profile(name, per_launch_bytes, variant):
    """HBM bytes per launch measured by rocprofv3 counters, from the committed
    summary in profiles/, or None when the kernel source changed since or the
    counters were taken on another variant than the one the plan picks."""
    src = KERNEL_SRC.get(name)
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.txt")
    if not src or not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    m_bytes = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    m_var = re.search(r"variant:\s*(\S+)", text)
    if not m_hash or not m_bytes or not m_var or m_var.group(1) != variant:
        return None
    if source_hash(name) != m_hash.group(1):
        return None
    return float(m_bytes.group(1))


def time_call(torch, fn, reps):
    """Median kernel time (ms) of fn() from HIP events on the launch stream."""
    st = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    ev = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        ev.append((a, b))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def batched_reduce(skel, torch):
    """4096 float32 N(0, 1) vectors with log-uniform lengths in [32, 2^20) (about
    4.1e8 elements): one persistent launch (B1) against one reduction launch
    pair per vector (B0, the per-vector loop)."""
    import synth_inputs as si
    lens = si.log_uniform_lengths(4096, 32, 1 << 20, config=3, index=10)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    n = int(off[-1])
    x = skel.Container.from_numpy(si.normal_f32(n, 3, 0))
    offs = skel.Container.from_numpy(off)
    out = skel.Container.empty(skel.F32, len(lens))
    res = {"segments": len(lens), "elements": n, "bytes": 4 * n + 8 * len(off)}
    for name, reps in (("B1_persistent", 10), ("B0_per_segment", 3)):
        v = skel.variant_index(skel.SK_REDUCE_SEGMENTS, name)
        ms = time_call(torch, lambda: skel.skel_reduce_segments(skel.SUM, x, offs, out,
                                                                variant=v), reps)
        res[name] = {"us": round(ms * 1e3, 1), "GBps": round(res["bytes"] / (ms * 1e-3) / 1e9, 1)}
    res["speedup_persistent_vs_per_segment"] = round(
        res["B0_per_segment"]["us"] / res["B1_persistent"]["us"], 2)
    for c in (x, offs, out):
        c.destroy()
    return res


def bf16_sums(skel, torch, with_errors=True):
    """2^28 bfloat16 values, |x| log-uniform in [1e-3, 1e3] with random signs:
    plain (R2 / MR2) against compensated (R4 / MR4) and pairwise (R5 / MR5)
    Reduce and dot.  Each result's error is stated against the exactly rounded
    sum of the same stored values (the oracle, on the host, after the timing),
    with the bars the precision tests hold it to: 1e-5 sum|x| for every
    variant, 2u|s| + 2^-36 sum|x| for the compensated ones, 64u sum|x| (65u for
    the dot) for the pairwise ones (u = 2^-24)."""
    import synth_inputs as si
    n = 1 << 28
    xh = si.log_uniform_signed_bf16(n, config=5, index=0)
    yh = si.log_uniform_signed_bf16(n, config=5, index=1)
    xb = skel.Container.from_numpy(xh, skel.BF16)
    yb = skel.Container.from_numpy(yh, skel.BF16)
    out = skel.Container.empty(skel.F32, 1)
    res = {"elements": n}
    got = {}
    for name in ("R2_ticket", "R4_compensated", "R5_pairwise"):
        v = skel.variant_index(skel.SK_REDUCE, name)
        ms = time_call(torch, lambda: skel.skel_reduce(skel.SUM, xb, out, variant=v), 10)
        got["reduce_" + name] = float(out.to_numpy()[0])
        res["reduce_" + name] = {"us": round(ms * 1e3, 1),
                                 "GBps": round(2 * n / (ms * 1e-3) / 1e9, 1)}
    for name in ("MR2_fused_ticket", "MR4_compensated", "MR5_pairwise"):
        v = skel.variant_index(skel.SK_MAPREDUCE, name)
        ms = time_call(torch, lambda: skel.skel_mapreduce(skel.MAP_MUL, None, [xb, yb],
                                                          skel.SUM, out, variant=v), 10)
        got["dot_" + name] = float(out.to_numpy()[0])
        res["dot_" + name] = {"us": round(ms * 1e3, 1),
                              "GBps": round(4 * n / (ms * 1e-3) / 1e9, 1)}
    for c in (xb, yb, out):
        c.destroy()
    if with_errors:
        import oracle
        log("exact bf16 sums on the host (oracle)")
        xf, yf = si.bf16_bits_to_f32(xh), si.bf16_bits_to_f32(yh)
        ref = {"reduce": (oracle.sum_bf16_exact(xh), oracle.abs_sum(xf)),
               "dot": (oracle.dot_bf16_exact(xh, yh), oracle.abs_sum(xf * yf))}
        u = 2.0 ** -24
        for key, val in got.items():
            kind = key.split("_")[0]
            exact, mag = ref[kind]
            err = abs(val - exact)
            bar = (2 * u * abs(exact) + 2.0 ** -36 * mag if "compensated" in key
                   else (64 + (kind == "dot")) * u * mag if "pairwise" in key else 1e-5 * mag)
            res[key].update({"result": val, "abs_err": float(f"{err:.4g}"),
                             "rel_err": float(f"{err / abs(exact):.4g}"),
                             "err_over_abs_sum": float(f"{err / mag:.4g}"),
                             "bar": float(f"{bar:.4g}"), "within_bar": bool(err <= bar)})
        res["exact"] = {k: {"sum": v[0], "abs_sum": v[1]} for k, v in ref.items()}
    return res


def backward_kernels(skel, torch, wl):
    """The adjoints at the large sizes: Map backward of saxpy (x, g read; dx,
    dy written; the parameter gradient summed), the 1D and 2D stencil
    transposes in both variants, and the reverse scan."""
    n, res = N_VEC, {}
    g = skel.Container.from_numpy(wl.z_h)
    dx, dy = skel.Container.empty(skel.F32, n), skel.Container.empty(skel.F32, n)
    dp = skel.Container.empty(skel.F32, 1)
    ms = time_call(torch, lambda: skel.skel_map_backward(skel.MAP_AXPY, [2.5], [wl.x, wl.y], g,
                                                         [dx, dy], dp), 10)
    res["map_backward_saxpy"] = {"us": round(ms * 1e3, 1),
                                 "GBps": round(16 * n / (ms * 1e-3) / 1e9, 1)}
    for v in range(skel.skel_variant_count(skel.SK_MAPOVERLAP1D_BACKWARD)):
        name = skel.skel_variant_name(skel.SK_MAPOVERLAP1D_BACKWARD, v)
        ms = time_call(torch, lambda: skel.skel_mapoverlap1d_backward(
            g, dx, wl.w5, 2, skel.EDGE_CLAMP, variant=v), 10)
        res["mapoverlap1d_5pt_backward_" + name] = {"us": round(ms * 1e3, 1),
                                                    "GBps": round(8 * n / (ms * 1e-3) / 1e9, 1)}
    gi = skel.Container.from_numpy(wl.img_h)
    di = skel.Container.empty(skel.F32, IMG, IMG)
    for v in range(skel.skel_variant_count(skel.SK_MAPOVERLAP2D_BACKWARD)):
        name = skel.skel_variant_name(skel.SK_MAPOVERLAP2D_BACKWARD, v)
        ms = time_call(torch, lambda: skel.skel_mapoverlap2d_backward(
            gi, di, wy=wl.g9, wx=wl.g9, edge=skel.EDGE_CLAMP, variant=v), 10)
        res["mapoverlap2d_9x9_backward_" + name] = {
            "us": round(ms * 1e3, 1), "GBps": round(8 * IMG * IMG / (ms * 1e-3) / 1e9, 1)}
    ms = time_call(torch, lambda: skel.skel_scan(wl.s, wl.so, skel.REVERSE_EXCLUSIVE, skel.SUM),
                   10)
    res["scan_reverse_excl_i32_i64"] = {"us": round(ms * 1e3, 1),
                                        "GBps": round(12 * N_SCAN / (ms * 1e-3) / 1e9, 1)}
    for c in (g, dx, dy, dp, gi, di):
        c.destroy()
    return res


FIELDS, FIELD_H, FIELD_W = 64, 2048, 2048  # the batched layer: 2^28 f32 per tensor


def field_layer(skel, torch, reps=5):
    """The differentiable layer on a batch of fields (64 x 2048 x 2048 f32,
    N(0, 1) from torch's seeded generator on the device): a 5-point stencil on
    every field (clamped borders), then prefix sums along every field row.
    Forward: one batched-field stencil call and one row-wise Scan; backward
    from an upstream gradient: one reverse row-wise Scan and one batched-field
    stencil transpose.  Each part is captured once into a HIP graph and
    replayed (HIP events on the replay stream); every part moves 8 algorithmic
    bytes per element (f32 in, f32 out).  For comparison, the forward stencil
    is also timed with the LDS-tile variant forced (`compare_*`, not part of
    the pass totals)."""
    import synth_inputs as si
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(si.BASE_SEED + 1000 * 4)
    shape = (FIELDS, FIELD_H, FIELD_W)
    x = torch.randn(shape, generator=gen, device=dev)
    gz = torch.randn(shape, generator=gen, device=dev)
    y, z, gy, gx = (torch.empty_like(x) for _ in range(4))
    w5 = si.five_point_weights()
    stream = torch.cuda.Stream()
    res, made = {}, []
    with torch.cuda.stream(stream):
        def wrap(t):
            made.append(skel.wrap_tensor(t, stream))
            return made[-1]
        rows = lambda t: wrap(t.view(-1, FIELD_W))
        cx, cy, cz, cgz, cgy, cgx = (rows(t) for t in (x, y, z, gz, gy, gx))
        parts = {
            "forward_stencil": lambda: skel.skel_mapoverlap2d_fields(
                cx, cy, FIELDS, w2d=w5, edge=skel.EDGE_CLAMP),
            "forward_scan_rows": lambda: skel.skel_scan_rows(cy, cz, skel.INCLUSIVE, skel.SUM),
            "backward_scan_rows": lambda: skel.skel_scan_rows(cgz, cgy, skel.REVERSE_INCLUSIVE,
                                                              skel.SUM),
            "backward_stencil": lambda: skel.skel_mapoverlap2d_fields_backward(
                cgy, cgx, FIELDS, w2d=w5, edge=skel.EDGE_CLAMP),
            "compare_forward_stencil_O2b_lds_tile": lambda: skel.skel_mapoverlap2d_fields(
                cx, cy, FIELDS, w2d=w5, edge=skel.EDGE_CLAMP,
                variant=skel.variant_index(skel.SK_MAPOVERLAP2D, "O2b_lds_tile")),
        }
        for fn in parts.values():  # sizes the stream's workspace outside the captures
            fn()
        torch.cuda.synchronize()
        graphs = {}
        for name, fn in parts.items():
            graphs[name] = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graphs[name], stream=stream):
                fn()
        torch.cuda.synchronize()
        nbytes = 8 * x.numel()
        for name, g in graphs.items():
            g.replay()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                g.replay()
            b.record(stream)
            b.synchronize()
            ms = a.elapsed_time(b) / reps
            res[name] = {"us": round(ms * 1e3, 1), "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1)}
    skel.skel_sync(stream)
    for c in made:
        c.destroy()
    for p in ("forward", "backward"):
        us = sum(v["us"] for k, v in res.items() if k.startswith(p))
        res[p] = {"us": round(us, 1), "GBps": round(2 * 8 * x.numel() / (us * 1e-6) / 1e9, 1)}
    res["fields"] = [FIELDS, FIELD_H, FIELD_W]
    n = x.numel()
    res["forward_stencil_variant"] = skel.skel_variant_name(
        skel.SK_MAPOVERLAP2D, skel.skel_select_variant(skel.SK_MAPOVERLAP2D, skel.F32, n,
                                                       FIELD_H, FIELD_W, aux=2 * 1))
    return res


def chain_layer(skel, torch, reps=5):
    """The differentiation workload's loss as one call: loss = sum over 64
    fields of 2048 x 2048 (N(0, 1) from torch's seeded generator on the
    device) of the 5-point MapOverlap2D (clamped) of tanh(w x + b), w = 0.75,
    b = -0.25, and its backward (dx, dw, db) from dL/dloss = 1.  Fused (C1:
    one pass reading x; the backward reads x and writes dx) against composed
    (C0: Map, batched-field stencil and Reduce with stored intermediates; the
    backward broadcasts, transposes the stencil and runs the Map adjoint).
    Algorithmic bytes: 4 per element forward, 8 backward."""
    import synth_inputs as si
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(si.BASE_SEED + 1000 * 4)
    x = torch.randn((FIELDS, FIELD_H, FIELD_W), generator=gen, device=dev)
    dx = torch.empty_like(x)
    w5 = si.five_point_weights()
    params = [0.75, -0.25]
    cx = skel.wrap_tensor(x.view(-1, FIELD_W))
    cdx = skel.wrap_tensor(dx.view(-1, FIELD_W))
    out = skel.Container.empty(skel.F32, 1)
    g1 = skel.Container.from_numpy(np.ones(1, np.float32))
    dp = skel.Container.empty(skel.F32, 2)
    n = x.numel()
    res = {"fields": [FIELDS, FIELD_H, FIELD_W], "map": "tanh(0.75 x - 0.25)",
           "stencil": "5-point, C 0.5, N S W E 0.125, clamp"}
    for v in range(skel.skel_variant_count(skel.SK_MAP_OVERLAP2D_REDUCE)):
        name = skel.skel_variant_name(skel.SK_MAP_OVERLAP2D_REDUCE, v)
        fwd = time_call(torch, lambda: skel.skel_map_overlap2d_reduce(
            skel.MAP_AFFINE_TANH, params, cx, FIELDS, out, w2d=w5, variant=v), reps)
        loss = float(out.to_numpy()[0])
        bwd = time_call(torch, lambda: skel.skel_map_overlap2d_reduce_backward(
            skel.MAP_AFFINE_TANH, params, cx, FIELDS, g1, cdx, dp, w2d=w5, variant=v), reps)
        res[name] = {
            "forward_us": round(fwd * 1e3, 1),
            "forward_GBps": round(4 * n / (fwd * 1e-3) / 1e9, 1),
            "forward_frac_hbm": round(4 * n / (fwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "backward_us": round(bwd * 1e3, 1),
            "backward_GBps": round(8 * n / (bwd * 1e-3) / 1e9, 1),
            "backward_frac_hbm": round(8 * n / (bwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "loss": loss, "dparams": [float(v_) for v_ in dp.to_numpy()]}
    fused, comp = res["C1_fused"], res["C0_composed"]
    res["speedup_fused_vs_composed"] = {
        "forward": round(comp["forward_us"] / fused["forward_us"], 2),
        "backward": round(comp["backward_us"] / fused["backward_us"], 2)}
    for c in (cx, cdx, out, g1, dp):
        c.destroy()
    return res


def dispatch_overhead(skel, torch):
    """Host cost of the execution plan and of a whole skeleton call (argument
    checks, plan, container protocol, launch), from Python through the C ABI,
    on a tiny operand so the GPU never holds the host back."""
    import ctypes
    lib = skel.load_library()
    reps = 20000
    t0 = time.perf_counter()
    for _ in range(reps):
        lib.skel_select_variant(skel.SK_REDUCE, skel.F32, 1 << 20, 1, 1 << 20, 0)
    sel_ns = (time.perf_counter() - t0) / reps * 1e9
    x = skel.Container.from_numpy(np.ones(256, np.float32))
    y = skel.Container.empty(skel.F32, 256)
    skel.skel_map(skel.MAP_AFFINE, [2.0, 1.0], [x], y)
    torch.cuda.synchronize()
    calls = 5000
    t0 = time.perf_counter()
    for _ in range(calls):
        skel.skel_map(skel.MAP_AFFINE, [2.0, 1.0], [x], y)
    host_us = (time.perf_counter() - t0) / calls * 1e6
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lib.skel_variant_count(skel.SK_MAP)  # a bare ctypes round trip, for comparison
    ctypes_ns = (time.perf_counter() - t0) / reps * 1e9
    x.destroy()
    y.destroy()
    return {"plan_lookup_ns": round(sel_ns, 1), "ctypes_call_ns": round(ctypes_ns, 1),
            "map_call_host_us": round(host_us, 2)}


def graph_replay(skel, torch, wl, steps):
    """One step captured into a HIP graph (torch.cuda.CUDAGraph) and replayed,
    against the same step issued call by call on the same stream."""
    calls = wl.calls()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _, fn in calls:  # sizes this stream's workspace outside the capture
            fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for _, fn in calls:
                fn()
        torch.cuda.synchronize()

        def timed(body):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            t0 = time.perf_counter()
            for _ in range(steps):
                body()
            b.record(stream)
            b.synchronize()
            return a.elapsed_time(b) / steps, (time.perf_counter() - t0) / steps * 1e3

        eager_gpu, eager_wall = timed(lambda: [fn() for _, fn in calls])
        graph_gpu, graph_wall = timed(g.replay)
    skel.skel_sync(stream)
    return {"eager_ms_per_step": round(eager_gpu, 4), "graph_ms_per_step": round(graph_gpu, 4),
            "eager_host_ms_per_step": round(eager_wall, 4),
            "graph_host_ms_per_step": round(graph_wall, 4)}


def cpu_baseline(wl):
    """The oracle (as it is, not tuned) over full steps on the host: on all
    of the process's cores (about 8 s), and on one thread (one step)."""
    import oracle
    model, ncpu = host_info()
    threads = min(ncpu, 64)

    def step():
        oracle.map_f32("axpy", [2.5], wl.x_h, wl.y_h)
        o1, _ = oracle.mapoverlap1d(wl.z_h, wl.w5, 2)
        oracle.scan(wl.s_h, "exclusive", "sum", np.int64)
        oracle.mapreduce("mul", None, wl.x_h, wl.y_h)
        oracle.mapoverlap2d(wl.img_h, 4, 4, wy=wl.g9, wx=wl.g9)
        oracle.reduce("sum", o1.astype(np.float32))

    oracle.set_threads(threads)
    reps, el = 0, 0.0
    while reps < 20 and (reps == 0 or el < 8.0):  # bounded: about 8 s of host work
        t0 = time.perf_counter()
        step()
        el += time.perf_counter() - t0
        reps += 1
    oracle.set_threads(1)
    t0 = time.perf_counter()
    step()
    el1 = time.perf_counter() - t0
    total = sum(BYTES.values())
    return {"value": round(total * reps / el / 1e9, 3), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} full step(s) (all six skeletons, same sizes) in {el:.2f} s; "
                      f"binary64/exact C oracle, OpenMP over independent outputs "
                      f"(map, stencils), sequential reductions and scans; host {model}",
            "one_thread": {"value": round(total / el1 / 1e9, 3), "unit": "GB/s",
                           "sample": f"1 full step on 1 thread in {el1:.2f} s"}}


def small_config(skel, torch):
    """The small configuration (2^20 elements, resident in the 256 MiB
    Infinity Cache, latency-bound): device time per call from bursts of 50
    back-to-back calls between one event pair, enqueued behind a spin kernel
    so that host issue gaps stay out (the plan's variant for each call), every
    Reduce and single-pass Scan variant on its own, and the four calls as one
    step: issued call by call, replayed as a captured graph, and forked onto
    four streams (eagerly and as a graph with four branches)."""
    import synth_inputs as si
    n = 1 << 20
    x = skel.Container.from_numpy(si.uniform_f32(n, -1.0, 1.0, 0, 0))
    y = skel.Container.from_numpy(si.uniform_f32(n, -1.0, 1.0, 0, 1))
    s = skel.Container.from_numpy(si.int_uniform_i32(n, 100, 0, 2))
    so = skel.Container.empty(skel.I32, n)
    z = skel.Container.from_numpy(si.uniform_f32(n, -1.0, 1.0, 0, 3))
    o = skel.Container.empty(skel.F32, n)
    r = skel.Container.empty(skel.F32, 1)
    w5 = si.binomial5_weights()
    calls = {
        "map_saxpy": (12 * n, skel.SK_MAP, skel.F32,
                      lambda v=-1: skel.skel_map(skel.MAP_AXPY, [2.5], [x, y], y, variant=v)),
        "reduce_sum": (4 * n, skel.SK_REDUCE, skel.F32,
                       lambda v=-1: skel.skel_reduce(skel.SUM, x, r, variant=v)),
        "scan_incl_i32": (8 * n, skel.SK_SCAN, skel.I32,
                          lambda v=-1: skel.skel_scan(s, so, skel.INCLUSIVE, skel.SUM,
                                                      variant=v)),
        "mapoverlap1d_5pt": (8 * n, skel.SK_MAPOVERLAP1D, skel.F32,
                             lambda v=-1: skel.skel_mapoverlap1d(z, o, w5, 2, skel.EDGE_CLAMP,
                                                                 variant=v)),
    }
    from paper_1405_2915_amd.autotune import SpinCalibration, burst_us
    burst = 50
    stream = torch.cuda.Stream()

    def per_call_us(body, reps=burst):
        body()
        return burst_us(torch, body, reps, spin)

    res = {"elements": n,
           "timing": f"bursts of {burst} back-to-back calls per event pair, enqueued behind "
                     "a spin kernel (device time, no host issue gaps)"}
    with torch.cuda.stream(stream):
        spin = SpinCalibration(torch)
        for name, (nbytes, sk, dt, fn) in calls.items():
            us = per_call_us(fn)
            v = skel.skel_select_variant(sk, dt, n, aux=2 if sk == skel.SK_MAPOVERLAP1D else 0)
            res[name] = {"variant": skel.skel_variant_name(sk, v), "us": round(us, 2),
                         "GBps": round(nbytes / (us * 1e-6) / 1e9, 1)}
        # the latency-bound variants one by one (the single-workgroup forms
        # and the order-dependent atomic finish left out)
        for name, sk, keep in (("reduce_sum", skel.SK_REDUCE,
                                ("R1_two_pass", "R2_ticket", "R6_gather")),
                               ("scan_incl_i32", skel.SK_SCAN,
                                ("S1_reduce_then_scan", "S2_decoupled_lookback",
                                 "S3_persistent_lookback", "S4_small_tile_lookback",
                                 "S5_flat_lookback"))):
            fn = calls[name][3]
            res[name]["variants_us"] = {
                vn: round(per_call_us(lambda: fn(skel.variant_index(sk, vn))), 2) for vn in keep}
        # the four calls as one step (launch-bound work is where the graph pays)
        for _, _, _, fn in calls.values():  # sizes this stream's workspace outside the capture
            fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for _, _, _, fn in calls.values():
                fn()
        torch.cuda.synchronize()
        eager = per_call_us(lambda: [fn() for _, _, _, fn in calls.values()], 25)
        graph = per_call_us(g.replay, 25)
        # ten steps in one graph: what a replay costs beyond its kernels
        g10 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g10, stream=stream):
            for _ in range(10):
                for _, _, _, fn in calls.values():
                    fn()
        torch.cuda.synchronize()
        graph10 = per_call_us(g10.replay, 10) / 10
        # The four calls are independent, and the containers order only
        # conflicting accesses (the Map and the Reduce both only read x): the
        # same step with three calls forked onto their own streams and the
        # fourth on this one, joined again, eagerly and as one captured graph
        # with four branches.
        fns = [fn for _, _, _, fn in calls.values()]
        side = [torch.cuda.Stream() for _ in fns[1:]]

        def fork():
            for st, fn in zip(side, fns[1:]):
                st.wait_stream(stream)
                with torch.cuda.stream(st):
                    fn()
            fns[0]()
            for st in side:
                stream.wait_stream(st)

        fork()  # outside capture: sizes every stream's workspace
        torch.cuda.synchronize()
        g4 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g4, stream=stream):
            fork()
        torch.cuda.synchronize()
        eager4 = per_call_us(fork, 25)
        graph4 = per_call_us(g4.replay, 25)
    skel.skel_sync(stream)
    res["step_of_four"] = {"eager_us": round(eager, 2), "graph_us": round(graph, 2),
                           "graph_of_ten_steps_us_per_step": round(graph10, 2),
                           "four_streams_eager_us": round(eager4, 2),
                           "four_streams_graph_us": round(graph4, 2)}
    for c in (x, y, s, so, z, o, r):
        c.destroy()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-variant pass")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the batched, bf16 and graph-replay measurements")
    ap.add_argument("--no-bulk", action="store_true",
                    help="time the step with the per-call plan's variants only (no bulk "
                         "selection over the whole step)")
    ap.add_argument("--small", action="store_true",
                    help="time only the small configuration (2^20 elements) and print its "
                         "JSON")
    ap.add_argument("--isolate", choices=ORDER, default=None,
                    help="time this one skeleton of the step alone (--steps calls) and exit")
    ap.add_argument("--before", choices=["read", "write"], default="read",
                    help="with --isolate: a 1 GiB read (clean cache) or plain write (dirty "
                         "cache) before every call")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the skeletons run on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU partitioning of the containers is not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1405_2915_amd as skel

    skel.skel_init(0, "torch")
    if args.small:
        res = small_config(skel, torch)
        res["dispatch"] = dispatch_overhead(skel, torch)
        print(json.dumps({"small_config": res}), flush=True)
        return
    wl = Workload(skel)
    if args.isolate:
        name = args.isolate
        us = isolated(skel, torch, wl, name, max(args.steps, 3), args.before)
        sk_id = {"map_saxpy": skel.SK_MAP, "mapoverlap1d_5pt": skel.SK_MAPOVERLAP1D,
                 "scan_excl_i32_i64": skel.SK_SCAN, "mapreduce_dot": skel.SK_MAPREDUCE,
                 "mapoverlap2d_9x9": skel.SK_MAPOVERLAP2D, "reduce_sum": skel.SK_REDUCE}[name]
        env_key = {skel.SK_MAP: "MAP", skel.SK_MAPOVERLAP1D: "MAPOVERLAP1D",
                   skel.SK_SCAN: "SCAN", skel.SK_MAPREDUCE: "MAPREDUCE",
                   skel.SK_MAPOVERLAP2D: "MAPOVERLAP2D", skel.SK_REDUCE: "REDUCE"}[sk_id]
        var = os.environ.get("SKEL_VARIANT_" + env_key)
        gbs = BYTES[name] / (us * 1e-6) / 1e9
        print(json.dumps({"isolated": name, "before": args.before,
                          "variant": var or skel.skel_variant_name(sk_id, wl.selected()[name]),
                          "us": round(us, 2), "GBps": round(gbs, 1),
                          "frac_hbm": round(gbs / HBM_PEAK_GBS, 4), "calls": args.steps}),
              flush=True)
        return
    calls = wl.calls()
    log(f"warmup {args.warmup} (first call copies every operand to HBM once)")
    run_steps(torch, calls, max(args.warmup, 1), with_events=False)
    skel.skel_sync()
    ids = {"map_saxpy": skel.SK_MAP, "mapoverlap1d_5pt": skel.SK_MAPOVERLAP1D,
           "scan_excl_i32_i64": skel.SK_SCAN, "mapreduce_dot": skel.SK_MAPREDUCE,
           "mapoverlap2d_9x9": skel.SK_MAPOVERLAP2D, "reduce_sum": skel.SK_REDUCE}
    plan_sel = wl.selected()
    names = lambda a: {k: skel.skel_variant_name(ids[k], v) for k, v in a.items()}

    def time_chain(assign, steps=8, samples=3):
        cl = wl.calls(assign)
        run_steps(torch, cl, 2, with_events=False)
        return float(np.median([run_steps(torch, cl, steps, with_events=False)[0] / steps * 1e3
                                for _ in range(samples)]))
    selection = {"per_call_plan": names(plan_sel)}
    sel = plan_sel
    if not args.no_bulk:
        # global composition over the step (Section V): the variants of all six
        # calls chosen together by whole-step time, from the plan's choices
        from paper_1405_2915_amd import compose
        log("bulk selection of the step's variants (whole-step timings)")
        sites = {k: [skel.variant_index(ids[k], nm) for nm in v] for k, v in STEP_SITES.items()}
        sel, rep = compose.bulk_select(time_chain, sites, plan_sel)
        skel.skel_sync()
        selection.update({"bulk": names(sel), "per_call_plan_ms_per_step": round(rep["start_ms"], 4),
                          "bulk_ms_per_step": round(rep["final_ms"], 4),
                          "whole_step_trials": len(rep["trials"])})
        calls = wl.calls(sel)
        run_steps(torch, calls, 2, with_events=False)
        skel.skel_sync()
    xfer_before = {k: getattr(wl, k).stats() for k in ("x", "y", "z", "s", "img")}
    log(f"timing {args.steps} steps")
    el, ms_dom = run_steps(torch, calls, args.steps, with_events={DOMINANT})
    skel.skel_sync()
    for k, before in xfer_before.items():
        after = getattr(wl, k).stats()
        assert after["h2d"] == before["h2d"], "no host-device copy inside the timed region"
    ms_step = el / args.steps * 1e3
    total_bytes = sum(BYTES.values())
    value = total_bytes / (el / args.steps) / 1e9
    log("per-skeleton breakdown (HIP events around every call, outside the timed region)")
    _, ms = run_steps(torch, calls, max(5, args.steps // 2), with_events=True)
    skel.skel_sync()

    per = {}
    for name in ORDER:
        avg = float(np.mean(ms[name]))
        gbs = BYTES[name] / (avg * 1e-3) / 1e9
        sk_id = {"map_saxpy": skel.SK_MAP, "mapoverlap1d_5pt": skel.SK_MAPOVERLAP1D,
                 "scan_excl_i32_i64": skel.SK_SCAN, "mapreduce_dot": skel.SK_MAPREDUCE,
                 "mapoverlap2d_9x9": skel.SK_MAPOVERLAP2D, "reduce_sum": skel.SK_REDUCE}[name]
        per[name] = {"variant": skel.skel_variant_name(sk_id, sel[name]),
                     "bytes": BYTES[name], "us": round(avg * 1e3, 2),
                     "GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}

    speedup = None
    if not args.no_plain:
        log("timing the fixed plain variants")
        ids = {"map_saxpy": skel.SK_MAP, "mapoverlap1d_5pt": skel.SK_MAPOVERLAP1D,
               "scan_excl_i32_i64": skel.SK_SCAN, "mapreduce_dot": skel.SK_MAPREDUCE,
               "mapoverlap2d_9x9": skel.SK_MAPOVERLAP2D, "reduce_sum": skel.SK_REDUCE}
        pv = {k: skel.variant_index(ids[k], PLAIN[k]) for k in ORDER}
        pcalls = wl.calls(pv)
        run_steps(torch, pcalls, 1, with_events=False)
        pel, pms = run_steps(torch, pcalls, max(3, args.steps // 4), with_events=True)
        skel.skel_sync()
        speedup = {"step": round((pel / max(3, args.steps // 4)) / (el / args.steps), 3)}
        for name in ORDER:
            p = float(np.mean(pms[name]))
            speedup[name] = round(p / (per[name]["us"] * 1e-3), 3)
            per[name]["plain_variant"] = PLAIN[name]
            per[name]["plain_us"] = round(p * 1e3, 2)

    ceil_gbs, ceil_ms = copy_ceiling(skel, torch)
    dom_variant = per[DOMINANT]["variant"]
    dom_kernel = SCAN_KERNELS.get(dom_variant, dom_variant)
    dom_us = float(np.mean(ms_dom[DOMINANT])) * 1e3  # timed region, launch stream
    achieved = BYTES[DOMINANT] / (dom_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_from_profile(DOMINANT, BYTES[DOMINANT], dom_variant),
                "kernel": dom_kernel,
                "kernel_us": round(dom_us, 2),
                "algorithmic_bytes_per_launch": BYTES[DOMINANT]}
    out = {
        "metric": "skeleton GB/s & % of HBM peak; autotuned/fused vs fixed-variant speedup",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32/i64", "data": "synthetic",
        "config": {"workload": "plain skeleton step on the large configuration: 9x9 "
                               "separable Gaussian MapOverlap2D 4096x4096 f32, dot "
                               "MapReduce 2^26 f32, exclusive Scan 2^27 i32->i64, plus "
                               "saxpy Map, 5-pt MapOverlap1D and sum Reduce on 2^26 f32",
                   "bytes_per_step": total_bytes, "parallelism": "single GPU"},
        "frac_hbm_step": round(value / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "copy_ceiling_GBps": round(ceil_gbs, 1),
        "per_skeleton": per,
        "speedup_vs_plain": speedup,
        "selection": selection,
    }
    if not args.no_next:
        log("graph replay of one step")
        nxt = {"graph_step": graph_replay(skel, torch, wl, max(args.steps, 5))}
        log("batched Reduce over 4096 uneven vectors")
        nxt["batched_reduce"] = batched_reduce(skel, torch)
        log("bf16 plain, compensated and pairwise sums, 2^28")
        nxt["bf16_sums"] = bf16_sums(skel, torch)
        out["next_rows"] = nxt
        log("backward kernels")
        nxt["backward"] = backward_kernels(skel, torch, wl)
        log("batched field layer, 64 x 2048^2: forward and backward")
        nxt["field_layer"] = field_layer(skel, torch)
        log("loss chain Map -> MapOverlap2D -> Reduce, 64 x 2048^2: fused and composed")
        nxt["chain_loss"] = chain_layer(skel, torch)
        log("small configuration, 2^20")
        out["small_config"] = small_config(skel, torch)
        out["small_config"]["dispatch"] = dispatch_overhead(skel, torch)
    if not args.no_cpu:
        log("timing the CPU oracle on one step")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
