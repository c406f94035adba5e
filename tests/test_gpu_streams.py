"""Cross-stream ordering on the device (Section V: the containers find each
call's dependences from its operands).  A seeded random sequence of skeleton
calls over four shared containers -- Map saxpy (in place or not), 5-point
MapOverlap 1D, inclusive Scan (in place or not; the flat look-back S5, whose
binary32 combination order is fixed, where S2/S3 combine in timing-dependent
order), sum Reduce, dot MapReduce, host reads and host rewrites -- runs once
with every call on one stream and once with each call on one of three streams, a
spin kernel delaying some calls' streams so that later calls on other streams
would overtake them unless ordered.  Both runs launch the same kernels on the
same data in the same program order, so any missed dependence (a read before
another stream's write has finished, a write over data another stream is
still reading) shows as a difference: every container, every Reduce and
MapReduce result and every host read must be bitwise equal."""
import random

import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

N = (1 << 18) + 5
NCONT = 4


def make_ops(seed, count=60):
    rnd = random.Random(seed)
    ops = []
    for i in range(count):
        kind = rnd.choices(("axpy", "stencil", "scan", "reduce", "dot", "read", "write"),
                           weights=(25, 20, 15, 15, 10, 8, 7))[0]
        a, b, c = (rnd.randrange(NCONT) for _ in range(3))
        if kind == "stencil" and c == a:
            c = (a + 1) % NCONT
        ops.append({"kind": kind, "a": a, "b": b, "c": c, "stream": rnd.randrange(3),
                    "delay": rnd.random() < 0.3, "alpha": rnd.choice((0.5, -1.25, 2.0)),
                    "index": i})
    return ops


def run_trace(skel, torch, ops, streams):
    cs = [skel.Container.from_numpy(si.uniform_f32(N, -1.0, 1.0, 12, k)) for k in range(NCONT)]
    w5 = si.binomial5_weights()
    sums, seen = [], []
    for op in ops:
        s = streams[op["stream"] % len(streams)]
        a, b, c = cs[op["a"]], cs[op["b"]], cs[op["c"]]
        if op["delay"]:
            with torch.cuda.stream(s):
                torch.cuda._sleep(40000)  # some tens of microseconds
        if op["kind"] == "axpy":
            skel.skel_map(skel.MAP_AXPY, [op["alpha"]], [a, b], c, stream=s)
        elif op["kind"] == "stencil":
            skel.skel_mapoverlap1d(a, c, w5, 2, skel.EDGE_CLAMP, stream=s)
        elif op["kind"] == "scan":
            skel.skel_scan(a, c, skel.INCLUSIVE, skel.SUM,
                           variant=skel.variant_index(skel.SK_SCAN, "S5_flat_lookback"), stream=s)
        elif op["kind"] == "reduce":
            r = skel.Container.empty(skel.F32, 1)
            skel.skel_reduce(skel.SUM, a, r, stream=s)
            sums.append(r)
        elif op["kind"] == "dot":
            r = skel.Container.empty(skel.F32, 1)
            skel.skel_mapreduce(skel.MAP_MUL, None, [a, b], skel.SUM, r, stream=s)
            sums.append(r)
        elif op["kind"] == "read":
            seen.append(a.to_numpy().copy())
        else:
            a.write_numpy(si.uniform_f32(N, -1.0, 1.0, 13, op["index"]))
    final = [x.to_numpy().copy() for x in cs]
    sums = [float(r.to_numpy()[0]) for r in sums]
    torch.cuda.synchronize()
    for x in cs:
        x.destroy()
    return final, sums, seen


@pytest.mark.parametrize("seed", range(4))
def test_random_calls_on_three_streams_match_one_stream(skel, seed):
    import torch
    ops = make_ops(seed)
    one = [torch.cuda.Stream()]
    three = [torch.cuda.Stream() for _ in range(3)]
    print(f"stream trace seed={seed}: {len(ops)} calls", flush=True)
    ref = run_trace(skel, torch, ops, one)
    got = run_trace(skel, torch, ops, three)
    for k, (x, y) in enumerate(zip(ref[0], got[0])):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (seed, "container", k)
    assert ref[1] == got[1], (seed, "Reduce and MapReduce results")
    assert len(ref[2]) == len(got[2])
    for k, (x, y) in enumerate(zip(ref[2], got[2])):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (seed, "host read", k)
    skel.skel_sync()
