"""The allocation-free Scan entry point (skel_scan_noalloc) through the C ABI:
its results equal those of skel_scan (the entry point it is a variant of,
forced to the same reduce-then-scan variant, so bit-identical for every type)
and the oracle's, on two calls in a row with the second smaller, with no
device memory taken from the allocator; the size limit and the unsupported
kinds are refused before anything is enqueued; and the call replays correctly
from a captured graph, which is what callers that cannot allocate need."""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

TILE4 = 16 * 2048        # scan tile of 4-byte inputs
MAX4 = 32768 * TILE4     # the array's limit for 4-byte inputs (2^30)


def _tensor(torch, arr):
    return torch.from_numpy(np.ascontiguousarray(arr)).cuda()


def _via_skel_scan(skel, x, out_dtype, kind, op):
    """The existing entry point on containers, forced to S1 (the variant the
    allocation-free call runs)."""
    s1 = skel.variant_index(skel.SK_SCAN, "S1_reduce_then_scan")
    cx = skel.Container.from_numpy(x)
    cy = skel.Container.empty({np.dtype(np.int32): skel.I32, np.dtype(np.int64): skel.I64,
                               np.dtype(np.float32): skel.F32}[np.dtype(out_dtype)], x.size)
    skel.skel_scan(cx, cy, kind, op, variant=s1)
    return cy.to_numpy()


CASES = [
    # (input dtype, output dtype, kind, op, first n, second n)
    (np.int32, np.int64, "exclusive", "sum", 3 * TILE4 + 517, TILE4 + 5),
    (np.int32, np.int32, "inclusive", "sum", 2 * TILE4 + 1, 1000),
    (np.int64, np.int64, "inclusive", "max", 5 * 8192 + 3, 77),
    (np.float32, np.float32, "inclusive", "sum", 2 * TILE4 + 99, 3 * 64 + 1),
]


@pytest.mark.parametrize("din,dout,kind,op,n1,n2", CASES)
def test_noalloc_matches_skel_scan_two_calls(skel, oracle_mod, din, dout, kind, op, n1, n2):
    import torch
    code = {np.int32: skel.I32, np.int64: skel.I64, np.float32: skel.F32}
    kinds = {"inclusive": skel.INCLUSIVE, "exclusive": skel.EXCLUSIVE}
    ops = {"sum": skel.SUM, "min": skel.MIN, "max": skel.MAX}
    for call, n in enumerate((n1, n2)):  # the second call is smaller
        print(f"noalloc {np.dtype(din).name}->{np.dtype(dout).name} {kind} {op} n={n}",
              flush=True)
        if din == np.float32:
            x = si.uniform_f32(n, -1.0, 1.0, 3, 40 + call)
        elif din == np.int64:
            x = si.int_uniform_i64(n, -2**40, 2**40, 3, 40 + call)
        else:
            x = si.int_uniform_i32(n, 1000, 3, 40 + call)
        xt = _tensor(torch, x)
        yt = torch.full((n,), -7, dtype={np.int32: torch.int32, np.int64: torch.int64,
                                          np.float32: torch.float32}[dout], device="cuda")
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        skel.skel_scan_noalloc(xt.data_ptr(), code[din], yt.data_ptr(), code[dout], n,
                               kinds[kind], ops[op])
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        got = yt.cpu().numpy()
        want = _via_skel_scan(skel, x, dout, kinds[kind], ops[op])
        assert np.array_equal(got, want), "differs from skel_scan (S1) on the same input"
        if din == np.float32:
            ref, mag = oracle_mod.scan(x, kind, op)
            assert np.all(np.abs(got - ref) <= 1e-5 * mag + 1e-30)
        else:
            assert np.array_equal(got, oracle_mod.scan(x, kind, op, dout))


def test_noalloc_in_place(skel, oracle_mod):
    import torch
    n = TILE4 + 333
    x = si.int_uniform_i32(n, 100, 3, 50)
    t = _tensor(torch, x)
    skel.skel_scan_noalloc(t.data_ptr(), skel.I32, t.data_ptr(), skel.I32, n, skel.INCLUSIVE,
                           skel.SUM)
    assert np.array_equal(t.cpu().numpy(), oracle_mod.scan(x, "inclusive", "sum"))


def test_noalloc_refusals(skel):
    import torch
    x = torch.zeros(64, dtype=torch.int32, device="cuda")
    y = torch.zeros(64, dtype=torch.int64, device="cuda")

    def status(*a):
        try:
            skel.skel_scan_noalloc(*a)
        except skel.SkelError as e:
            return e.status
        return skel.OK
    p, q = x.data_ptr(), y.data_ptr()
    # beyond the array's limit: refused on the host, nothing launched
    assert status(p, skel.I32, q, skel.I64, MAX4 + 1, skel.INCLUSIVE, skel.SUM) == skel.E_SHAPE
    assert status(p, skel.I64, q, skel.I64, MAX4 // 2 + 1, skel.INCLUSIVE, skel.SUM) \
        == skel.E_SHAPE
    assert status(p, skel.I32, q, skel.I64, 64, skel.REVERSE_INCLUSIVE, skel.SUM) \
        == skel.E_UNSUPPORTED
    assert status(p, skel.I32, q, skel.F32, 64, skel.INCLUSIVE, skel.SUM) == skel.E_DTYPE
    assert status(p + 4, skel.I32, q, skel.I64, 60, skel.INCLUSIVE, skel.SUM) == skel.E_INVAL
    assert status(p, skel.I32, p + 64, skel.I32, 64, skel.INCLUSIVE, skel.SUM) == skel.E_INVAL
    assert status(0, skel.I32, q, skel.I64, 64, skel.INCLUSIVE, skel.SUM) == skel.E_INVAL
    assert status(p, skel.I32, q, skel.I64, 0, skel.INCLUSIVE, skel.SUM) == skel.OK


def test_noalloc_graph_replay(skel, oracle_mod):
    """Captured once, replayed three times with new inputs written between the
    replays (eager work and synchronisations in between); every replay equals
    the oracle."""
    import torch
    n = 2 * TILE4 + 1234
    xt = torch.zeros(n, dtype=torch.int32, device="cuda")
    yt = torch.zeros(n, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # once outside the capture on the capture stream
        skel.skel_scan_noalloc(xt.data_ptr(), skel.I32, yt.data_ptr(), skel.I64, n,
                               skel.EXCLUSIVE, skel.SUM)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        skel.skel_scan_noalloc(xt.data_ptr(), skel.I32, yt.data_ptr(), skel.I64, n,
                               skel.EXCLUSIVE, skel.SUM)
    for rep in range(3):
        x = si.int_uniform_i32(n, 1000, 3, 60 + rep)
        xt.copy_(torch.from_numpy(x))
        yt.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(yt.cpu().numpy(), oracle_mod.scan(x, "exclusive", "sum", np.int64))
