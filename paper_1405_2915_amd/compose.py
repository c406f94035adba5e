"""Bulk selection of skeleton variants over a chain of calls.

Section V of the paper: run-time selection that is greedy and local to each
call can be suboptimal for chains and loops of dependent calls, because a
call's choice changes the costs its successors meet; a global composition
step instead selects for several calls at once (bulk selection).  Here the
execution plan (Section III) picks each call's variant from that call's
context alone -- which the off-line tuner measures with the Infinity Cache
in a fixed state -- while inside a chain a call runs after its predecessor,
e.g. after a large write that left the cache full of dirty lines.

    assignment, report = bulk_select(time_chain, sites, start)

`time_chain(assignment)` runs the chain with the given forced variants and
returns its time; `sites` maps each call of the chain to the variants that
may serve it; `start` is the per-call plan's assignment.  The search is a
coordinate descent over whole-chain times: each call in turn tries its other
variants with the rest fixed, and a change is kept only when it shortens the
chain by more than `min_gain` (relative; timing noise stays out of the
choice).  The result feeds forced variants into the same C entry points.
"""
from __future__ import annotations


def bulk_select(time_chain, sites, start, min_gain=0.003, passes=2):
    """Return (assignment, report).  report: {"start_ms", "final_ms",
    "trials": [(call, variant, ms), ...]}; variants for which time_chain
    raises (not selectable for that call) are skipped."""
    current = dict(start)
    best_ms = time_chain(current)
    report = {"start_ms": best_ms, "trials": []}
    for _ in range(passes):
        changed = False
        for call, candidates in sites.items():
            for v in candidates:
                if v == current[call]:
                    continue
                trial = dict(current)
                trial[call] = v
                try:
                    ms = time_chain(trial)
                except Exception:  # not selectable for this call: skip it
                    continue
                report["trials"].append((call, v, ms))
                if ms < best_ms * (1.0 - min_gain):
                    current, best_ms, changed = trial, ms, True
        if not changed:
            break
    # the kept assignment, timed once more so that the figure is not the
    # minimum of many noisy trials
    report["final_ms"] = time_chain(current)
    return current, report
