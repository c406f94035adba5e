"""Repeated runs of the kernels whose workgroups hand values to each other
(look-back scan, ticket reductions, the persistent batched Reduce): every run
must give the bit-identical result.  A race in the hand-off (a descriptor read
before it is valid, a stale epoch, a lost ticket) would show as a differing
run.  The launches have far more tiles or work items than the device holds
workgroups at once (S2 starts one workgroup per tile; the persistent forms
loop each resident workgroup over many).  The
comparison runs on the device (torch), against the oracle's result uploaded
once."""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", [2, 3, 4])
def test_lookback_scan_repeated(skel, oracle_mod, variant):
    import torch
    n = 1 << 27
    xh = si.int_uniform_i32(n, 1000, 1, 2)
    ref = torch.from_numpy(oracle_mod.scan(xh, "exclusive", "sum", np.int64)).cuda()
    x = torch.from_numpy(xh).cuda()
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    cx, co = skel.wrap_tensor(x), skel.wrap_tensor(out)
    for rep in range(40):
        out.fill_(-1)
        skel.skel_scan(cx, co, skel.EXCLUSIVE, skel.SUM, variant=variant)
        assert torch.equal(out, ref), rep
    # the reverse form walks the tiles in the other order
    rref = torch.from_numpy(oracle_mod.scan(xh, "reverse_inclusive", "sum", np.int64)).cuda()
    for rep in range(10):
        out.fill_(-1)
        skel.skel_scan(cx, co, skel.REVERSE_INCLUSIVE, skel.SUM, variant=variant)
        assert torch.equal(out, rref), rep
    skel.skel_sync()
    cx.destroy()
    co.destroy()


def test_ticket_reductions_repeated(skel, oracle_mod):
    import torch
    n = (1 << 24) + 7
    xh = si.normal_f32(n, 12, 0)
    x = torch.from_numpy(xh).cuda()
    cx = skel.wrap_tensor(x)
    r = torch.empty(1, dtype=torch.float32, device="cuda")
    cr = skel.wrap_tensor(r)
    for v in (2, 4):  # R2 ticket, R4 compensated
        vals = set()
        for _ in range(100):
            skel.skel_reduce(skel.SUM, cx, cr, variant=v)
            vals.add(float(r.item()))
        assert len(vals) == 1, (v, vals)
        assert abs(vals.pop() - oracle_mod.reduce("sum", xh)) <= 1e-5 * oracle_mod.abs_sum(xh)
    xi = torch.from_numpy(si.int_uniform_i64(n, -2 ** 40, 2 ** 40, 12, 1)).cuda()
    ri = torch.empty(1, dtype=torch.int64, device="cuda")
    cxi, cri = skel.wrap_tensor(xi), skel.wrap_tensor(ri)
    want = oracle_mod.reduce("sum", xi.cpu().numpy(), np.int64)
    for _ in range(100):
        skel.skel_reduce(skel.SUM, cxi, cri, variant=2)
        assert int(ri.item()) == want
    skel.skel_sync()
    for c in (cx, cr, cxi, cri):
        c.destroy()


def test_persistent_segments_repeated(skel, oracle_mod):
    import torch
    lens = si.log_uniform_lengths(1024, 32, 1 << 20, config=3, index=11)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    xh = si.normal_f32(int(off[-1]), 3, 5)
    ref = np.array([oracle_mod.reduce("sum", xh[off[s]:off[s + 1]]) for s in range(len(lens))])
    mag = np.array([oracle_mod.abs_sum(xh[off[s]:off[s + 1]]) for s in range(len(lens))])
    x, o = torch.from_numpy(xh).cuda(), torch.from_numpy(off).cuda()
    out = torch.empty(len(lens), dtype=torch.float32, device="cuda")
    cx, co, cout = skel.wrap_tensor(x), skel.wrap_tensor(o), skel.wrap_tensor(out)
    b1 = skel.variant_index(skel.SK_REDUCE_SEGMENTS, "B1_persistent")
    skel.skel_reduce_segments(skel.SUM, cx, co, cout, variant=b1)
    first = out.clone()
    got = first.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= 1e-5 * mag + 1e-30)
    for rep in range(40):
        out.fill_(np.nan)
        skel.skel_reduce_segments(skel.SUM, cx, co, cout, variant=b1)
        assert torch.equal(out, first), rep
    skel.skel_sync()
    for c in (cx, co, cout):
        c.destroy()


def test_shrunk_tile_lookback_stress(skel):
    """The look-back with tiles shrunk to two wavefronts (the library built
    with SKEL_SCAN_WAVES=2: 32768 tiles for 2^27 elements instead of 4096, so
    each tile looks back over many more unfinished predecessors), in a child
    process that loads that build: 20 repeats of each single-pass variant,
    bit-identical to the oracle."""
    import os
    import subprocess
    import sys
    from paper_1405_2915_amd import build_lib
    if not os.path.exists(build_lib.SCAN_STRESS_LIB):
        pytest.fail("libskel_scan_w2.so not built (paper_1405_2915_amd/build_lib.py)")
    child = os.path.join(os.path.dirname(os.path.abspath(__file__)), "scan_stress_child.py")
    env = dict(os.environ, SKEL_LIBRARY=build_lib.SCAN_STRESS_LIB)
    res = subprocess.run([sys.executable, "-u", child], env=env, capture_output=True,
                         text=True, timeout=240)
    print(res.stdout[-2000:], res.stderr[-2000:])
    assert res.returncode == 0 and res.stdout.strip().endswith("ok")
