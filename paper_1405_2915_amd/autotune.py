"""Off-line tuning of the execution plan.

Section II of the paper: besides on-line models, composition can use off-line
tuning that precomputes a dispatch structure, looked up at run time, from
sample executions; Section III: an execution plan attached to a skeleton gives
the expected best implementation for a call context and is recomputed once per
target system.  This module is that off-line step for one GPU:

    python -m paper_1405_2915_amd.autotune [--out FILE] [--min 10] [--max 28]
                                           [--reps 7] [--report FILE.json]

For each tuned skeleton (sum Reduce, dot MapReduce, inclusive int32 Scan,
saxpy Map, 5-point MapOverlap1D, 9x9 separable MapOverlap2D on a near-square
image) and each size n = 2^k it times every selectable variant (forced) with
HIP events on the launch stream.  Above 2^22 elements: the median of `reps`
single calls, each after the 256 MiB Infinity Cache was evicted by a pass of
plain loads over a 1 GiB buffer (non-temporal loads, which the Reduce kernels
use, leave most of the cache's contents in place: a 2^24-element copy takes
the same time after such a pass as back to back).  Up to 2^22 elements, where one call lasts a few
microseconds: after one eviction, `burst` calls back to back between one
event pair, the time per call being their span divided by `burst` (median of
`reps` bursts).  A spin kernel ahead of the pair holds the stream until the
host has enqueued the whole burst, so the calls run back to back at the
device's pace: the figure is the kernels' time on the device, not the host's
issue time of a call (a few microseconds through Python and the C ABI, as
long as a small kernel), and later calls of a burst find their operands in
the caches, as calls of that size do in a loop.  It writes the fastest variant per
(skeleton, dtype, log2 n) as a plan table (the text format of skel_load_plan)
and a JSON report of every timing.  Single-workgroup variants are not timed
above 2^22 elements (they use one CU of 256).  The atomic-finish Reduce (R3),
whose floating-point result depends on the order the workgroups finish in, is
left out of the plan unless --allow-order-dependent is given: a tuned plan
keeps every automatic call deterministic.

--adaptive samples sizes adaptively instead of all of them (adaptive
sampling, cited in Section II as a way to spend fewer off-line sample
executions at a small loss of precision): per skeleton, both ends of the
range are timed first, and a size interval is bisected only while the
variant chosen at its lower end is more than the tolerance slower than the
fastest variant at its upper end.  Unsampled sizes take the choice of the
nearest sampled size below, as the plan table does.  --compare FULL.json
states, for every size of a full sweep, how much slower the adaptive plan's
choice is than that sweep's fastest variant.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_PLAN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plans", "gfx950.plan")
SINGLE_WG_MAX_LOG2 = 22


BURST_MAX_LOG2 = 22  # sizes timed as bursts of back-to-back calls
BURST = 20


class SpinCalibration:
    """Cycles of torch.cuda._sleep (a spin kernel) per microsecond, measured
    once with events."""

    def __init__(self, torch):
        st = torch.cuda.current_stream()
        torch.cuda._sleep(1000)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        cycles = 1 << 22
        a.record(st)
        torch.cuda._sleep(cycles)
        b.record(st)
        b.synchronize()
        self.cycles_per_us = cycles / max(a.elapsed_time(b) * 1e3, 1e-3)


def burst_us(torch, fn, burst, spin, before=None):
    """Device time per call (us) of `burst` back-to-back calls of fn.  A spin
    kernel holds the stream while the host enqueues the burst (it spins for
    three times the host's measured issue time of one burst, plus 100 us), so
    the calls then run back to back at the device's pace and the event pair
    around them sees no host issue gaps: small calls are timed by the GPU, not
    by the Python and C-ABI cost of issuing them.  `before` (e.g. a cache
    eviction pass) runs ahead of the spin."""
    import time
    st = torch.cuda.current_stream()
    t0 = time.perf_counter()
    for _ in range(burst):
        fn()
    host_us = (time.perf_counter() - t0) * 1e6
    torch.cuda.synchronize()
    if before is not None:
        before()
    torch.cuda._sleep(int(spin.cycles_per_us * (3.0 * host_us + 100.0)))
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(burst):
        fn()
    b.record(st)
    b.synchronize()
    return a.elapsed_time(b) * 1e3 / burst


def _timed(torch, fn, evict, reps, burst=1, spin=None):
    """Median over `reps` of the device time per call in microseconds, the
    Infinity Cache evicted before each timing: one call per event pair, or
    (burst > 1) a burst of back-to-back calls behind a spin kernel."""
    st = torch.cuda.current_stream()
    fn()  # sizes the stream's workspace; first-use costs stay out of the timing
    times = []
    for _ in range(reps):
        if burst > 1:
            times.append(burst_us(torch, fn, burst, spin, before=evict))
            continue
        evict()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        times.append(a.elapsed_time(b) * 1e3)
    return float(np.median(times))


ORDER_DEPENDENT = {"R3_atomic"}


class Bisection:
    """Adaptive choice of the sizes (log2 n) to sample for one skeleton.

    Starts from both ends of [lo, hi]; after each round of measurements an
    open interval [a, b] is settled when the fastest variant at a is within
    `tol` of the fastest at b (the plan then keeps it across the interval),
    and is otherwise split at its midpoint, until intervals are one size
    wide.  `res` maps every sampled size to its {variant: us}."""

    def __init__(self, lo, hi, tol=0.05, exclude=()):
        self.tol = tol
        self.exclude = set(exclude)
        self.res = {}
        self.pending = {lo, hi}
        self.open = [(lo, hi)] if hi > lo else []

    def _best(self, k):
        r = {a: b for a, b in self.res[k].items() if a not in self.exclude}
        return min(r, key=r.get), r

    def settled(self, a, b):
        wa, _ = self._best(a)
        _, rb = self._best(b)
        return wa in rb and rb[wa] <= (1 + self.tol) * min(rb.values())

    def wanted(self):
        return sorted(self.pending - set(self.res))

    def add(self, k, res):
        self.res[k] = res

    def step(self):
        """Split the unsettled intervals; True while sizes remain to sample."""
        nxt = []
        for a, b in self.open:
            if b - a <= 1 or self.settled(a, b):
                continue
            m = (a + b) // 2
            self.pending.add(m)
            nxt += [(a, m), (m, b)]
        self.open = nxt
        return bool(self.wanted())


class _Timer:
    """Containers of one size and the timed calls of every tuned skeleton."""

    CASES = ("REDUCE", "MAPREDUCE", "SCAN", "MAP", "MAPOVERLAP1D", "MAPOVERLAP2D")

    def __init__(self, torch, skel, si, reps, log):
        self.torch, self.skel, self.si, self.reps, self.log = torch, skel, si, reps, log
        # plain-load read of 1 GiB: replaces the Infinity Cache's contents with
        # clean lines of another buffer
        self.flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
        self.evict()
        torch.cuda.synchronize()
        self.spin = SpinCalibration(torch)
        self.single = {skel.SK_REDUCE: "R0_single_wg", skel.SK_MAPREDUCE: "MR3_fused_single_wg",
                       skel.SK_SCAN: "S0_single_wg"}
        self.w5 = si.binomial5_weights()
        self.g9 = si.gaussian_weights(4, 2.0)

    def evict(self):
        self.flush.sum()

    def time_size(self, k, names):
        """{name: {variant: us}} for the named skeletons at n = 2^k."""
        skel, si = self.skel, self.si
        n = 1 << k
        x = skel.Container.from_numpy(si.normal_f32(n, 2, 0))
        y = skel.Container.from_numpy(si.normal_f32(n, 2, 1))
        s = skel.Container.from_numpy(si.int_uniform_i32(n, 100, 2, 2))
        so = skel.Container.empty(skel.I32, n)
        out1 = skel.Container.empty(skel.F32, 1)
        o1 = skel.Container.empty(skel.F32, n)
        rows = 1 << (k // 2)  # the 2D cases: a rows x (n / rows) image
        img = skel.Container.from_numpy(si.uniform_f32(n, 0.0, 1.0, 2, 3).reshape(rows,
                                                                                   n // rows))
        imo = skel.Container.empty(skel.F32, rows, n // rows)
        w5, g9 = self.w5, self.g9
        cases = {
            "REDUCE": (skel.SK_REDUCE,
                       lambda v: skel.skel_reduce(skel.SUM, x, out1, variant=v)),
            "MAPREDUCE": (skel.SK_MAPREDUCE,
                          lambda v: skel.skel_mapreduce(skel.MAP_MUL, None, [x, y], skel.SUM,
                                                        out1, variant=v)),
            "SCAN": (skel.SK_SCAN,
                     lambda v: skel.skel_scan(s, so, skel.INCLUSIVE, skel.SUM, variant=v)),
            "MAP": (skel.SK_MAP,
                    lambda v: skel.skel_map(skel.MAP_AXPY, [2.5], [x, y], y, variant=v)),
            "MAPOVERLAP1D": (skel.SK_MAPOVERLAP1D,
                             lambda v: skel.skel_mapoverlap1d(x, o1, w5, 2, skel.EDGE_CLAMP,
                                                              variant=v)),
            "MAPOVERLAP2D": (skel.SK_MAPOVERLAP2D,
                             lambda v: skel.skel_mapoverlap2d(img, imo, wy=g9, wx=g9,
                                                              edge=skel.EDGE_CLAMP, variant=v)),
        }
        out = {}
        for name in names:
            sk, call = cases[name]
            res = {}
            for v in range(skel.skel_variant_count(sk)):
                vname = skel.skel_variant_name(sk, v)
                if vname == self.single.get(sk) and k > SINGLE_WG_MAX_LOG2:
                    continue
                burst = BURST if k <= BURST_MAX_LOG2 else 1
                try:
                    res[vname] = round(_timed(self.torch, lambda: call(v), self.evict,
                                              self.reps, burst, self.spin), 3)
                except skel.SkelError as err:
                    if err.status != skel.E_UNSUPPORTED:
                        raise
                    # not selectable at this size (e.g. S5 beyond 1024 tiles)
            out[name] = res
            self.log(f"{name:12s} 2^{k:2d}: " + "  ".join(f"{a}={b:.1f}" for a, b in res.items()))
        for c in (x, y, s, so, out1, o1, img, imo):
            c.destroy()
        return out


def tune(lo=10, hi=28, reps=7, log=print, allow_order_dependent=False, adaptive=False,
         tol=0.05):
    import torch

    import paper_1405_2915_amd as skel
    import synth_inputs as si

    skel.skel_init(0, "torch", plan=None)  # time the variants, not a previous plan
    timer = _Timer(torch, skel, si, reps, log)
    report = {"lo": lo, "hi": hi, "reps": reps, "unit": "us", "results": {},
              "mode": "adaptive" if adaptive else "full"}
    if not adaptive:
        for k in range(lo, hi + 1):
            for name, res in timer.time_size(k, _Timer.CASES).items():
                report["results"].setdefault(name, {})[str(k)] = res
    else:
        excl = () if allow_order_dependent else ORDER_DEPENDENT
        bis = {name: Bisection(lo, hi, tol, excl) for name in _Timer.CASES}
        rounds = 0
        while True:
            want = {}
            for name, b in bis.items():
                for k in b.wanted():
                    want.setdefault(k, []).append(name)
            if not want:
                break
            rounds += 1
            for k in sorted(want):
                for name, res in timer.time_size(k, want[k]).items():
                    bis[name].add(k, res)
            for b in bis.values():
                b.step()
        for name, b in bis.items():
            report["results"][name] = {str(k): b.res[k] for k in sorted(b.res)}
        report["rounds"] = rounds
        report["sampled"] = {name: sorted(b.res) for name, b in bis.items()}
    report["dtypes"] = {"REDUCE": "f32", "MAPREDUCE": "f32", "SCAN": "i32", "MAP": "f32",
                        "MAPOVERLAP1D": "f32", "MAPOVERLAP2D": "f32"}
    report["timing"] = {"burst_max_log2": BURST_MAX_LOG2, "burst": BURST,
                        "spin_cycles_per_us": round(timer.spin.cycles_per_us, 1)}
    # the stencil class each MapOverlap entry was tuned on: radius 2 (the
    # 5-point binomial) in 1D, separable 9 x 9 (1 + 2 * 4) in 2D
    report["classes"] = {"MAPOVERLAP1D": 2, "MAPOVERLAP2D": 1 + 2 * 4}
    return plan_from_report(report, tol=tol, allow_order_dependent=allow_order_dependent), report


def plan_choice(table, name, k):
    """The plan's variant for skeleton `name` at log2 n = k: the entry of the
    nearest sampled size at or below k (None below the first)."""
    best = None
    for nm, _dt, kk, v, _c in sorted(table, key=lambda e: e[2]):
        if nm == name and kk <= k:
            best = v
    return best


def compare_with_full(table, full_report, allow_order_dependent=False):
    """For every skeleton and size of a full sweep: the chosen variant's time
    over the fastest there.  Returns {name: {"sizes": N, "worst": x,
    "mean": x, "over_tol": count}} and the per-size ratios."""
    out, ratios = {}, {}
    for name, per_k in full_report["results"].items():
        rs = []
        for k, res in per_k.items():
            res = {a: b for a, b in res.items()
                   if allow_order_dependent or a not in ORDER_DEPENDENT}
            pick = plan_choice(table, name, int(k))
            if pick is None or pick not in res:
                continue
            r = res[pick] / min(res.values())
            rs.append(r)
            ratios[(name, int(k))] = r
        if rs:
            out[name] = {"sizes": len(rs), "worst": round(max(rs), 3),
                         "mean": round(float(np.mean(rs)), 4),
                         "over_tol": sum(r > 1.05 for r in rs)}
    return out, ratios


def plan_from_report(report, tol=0.05, allow_order_dependent=False):
    """Plan entries (skeleton, dtype, log2 n, variant, stencil class or None)
    from measured times.

    Sizes are visited in increasing order and the previous size's choice is
    kept while it stays within `tol` of the fastest variant, so timing noise
    between near-equal variants does not make the plan flip back and forth."""
    table = []
    for name, per_k in report["results"].items():
        dt = report.get("dtypes", {}).get(name, "f32")
        cls = report.get("classes", {}).get(name)
        prev = None
        for k in sorted(per_k, key=int):
            res = {a: b for a, b in per_k[k].items()
                   if allow_order_dependent or a not in ORDER_DEPENDENT}
            best = min(res, key=res.get)
            if prev in res and res[prev] <= (1 + tol) * res[best]:
                best = prev
            table.append((name, dt, int(k), best, cls))
            prev = best
    return table


# the single fixed plain form each plan choice is compared with
PLAIN = {"REDUCE": "R1_two_pass", "MAPREDUCE": "MR0_unfused", "SCAN": "S1_reduce_then_scan",
         "MAP": "M0_scalar", "MAPOVERLAP1D": "O1a_direct", "MAPOVERLAP2D": "O2a_direct"}


def write_summary(report, table, path, header):
    """Markdown: for every skeleton and size, every variant's time, the
    plan's choice and its speedup over the fixed plain form."""
    choice = {(name, k): v for name, _dt, k, v, _c in table}
    with open(path, "w") as f:
        f.write("# Off-line tuning sweep: every variant at every size (us per call)\n\n")
        for line in header:
            f.write(f"{line}\n\n")
        f.write("Command: `python -m paper_1405_2915_amd.autotune --report FILE.json "
                "--summary FILE.md` (writes the plan to plans/gfx950.plan).\n\n")
        for name, per_k in report["results"].items():
            variants = sorted({v for r in per_k.values() for v in r})
            plain = PLAIN.get(name)
            f.write(f"## {name} ({report['dtypes'].get(name, 'f32')})\n\n")
            f.write("| log2 n | " + " | ".join(variants) + " | plan | speedup vs "
                    f"{plain} |\n")
            f.write("|---:|" + "---:|" * len(variants) + "---|---:|\n")
            for k in sorted(per_k, key=int):
                r = per_k[k]
                pick = choice.get((name, int(k)))
                cells = [f"{r[v]:.2f}" if v in r else "-" for v in variants]
                sp = (f"{r[plain] / r[pick]:.2f}" if plain in r and pick in r and r[pick] > 0
                      else "-")
                f.write(f"| {k} | " + " | ".join(cells) + f" | {pick} | {sp} |\n")
            f.write("\n")


def write_plan(table, path, header):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("# execution plan: fastest variant per (skeleton, dtype, log2 n[, stencil "
                "class])\n")
        for line in header:
            f.write(f"# {line}\n")
        # keep only the sizes where the choice changes (nearest lower key rules)
        last = {}
        for name, dt, k, v, cls in table:
            if last.get((name, dt, cls)) != v:
                f.write(f"{name} {dt} {k} {v}" + ("" if cls is None else f" {cls}") + "\n")
                last[(name, dt, cls)] = v


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PLAN)
    ap.add_argument("--report", default=None)
    ap.add_argument("--summary", default=None,
                    help="also write a markdown table of every timing and the speedup over "
                         "the fixed plain form")
    ap.add_argument("--min", type=int, default=10)
    ap.add_argument("--max", type=int, default=28)
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--allow-order-dependent", action="store_true",
                    help="let the plan pick the atomic-finish Reduce")
    ap.add_argument("--from-report", default=None,
                    help="write the plan from a saved JSON report, without timing")
    ap.add_argument("--adaptive", action="store_true",
                    help="sample sizes adaptively (bisect only where the choice changes)")
    ap.add_argument("--compare", default=None,
                    help="a full sweep's JSON report: state how far the written plan's "
                         "choices are from that sweep's fastest variants")
    args = ap.parse_args()
    if args.from_report:
        with open(args.from_report) as f:
            report = json.load(f)
        table = plan_from_report(report, allow_order_dependent=args.allow_order_dependent)
        write_plan(table, args.out, report.get("header", []))
        if args.summary:
            write_summary(report, table, args.summary, report.get("header", []))
        res = {"plan": args.out, "entries": len(table)}
        if args.compare:
            with open(args.compare) as f:
                full = json.load(f)
            res["against_full_sweep"], _ = compare_with_full(table, full,
                                                             args.allow_order_dependent)
        print(json.dumps(res))
        return
    log = lambda m: print(f"[autotune] {m}", file=sys.stderr, flush=True)
    table, report = tune(args.min, args.max, args.reps, log, args.allow_order_dependent,
                         adaptive=args.adaptive)
    import torch
    dev = torch.cuda.get_device_properties(0)
    report["header"] = [f"device: {dev.name} ({dev.gcnArchName}), "
                        f"{dev.multi_processor_count} CUs",
                        f"sizes 2^{args.min}..2^{args.max}"
                        + (" sampled adaptively" if args.adaptive else "")
                        + f", median of {args.reps}, Infinity Cache evicted (plain-load read "
                        "of 1 GiB) before each timed call; a choice is kept while within 5% "
                        "of the fastest"]
    report["header"].append(f"sizes up to 2^{BURST_MAX_LOG2}: bursts of {BURST} back-to-back "
                            "calls per event pair, enqueued behind a spin kernel (device "
                            "time)")
    write_plan(table, args.out, report["header"])
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    if args.summary:
        write_summary(report, table, args.summary, report["header"])
    res = {"plan": args.out, "entries": len(table)}
    if args.adaptive:
        res["samples"] = {name: len(ks) for name, ks in report["sampled"].items()}
        res["rounds"] = report["rounds"]
    if args.compare:
        with open(args.compare) as f:
            full = json.load(f)
        res["against_full_sweep"], _ = compare_with_full(table, full,
                                                         args.allow_order_dependent)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
