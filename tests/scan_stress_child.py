"""Child process of the shrunk-tile look-back stress test (run with
SKEL_LIBRARY naming the library built with two-wavefront scan tiles): the
2^27 int32 -> int64 exclusive scan, 20 times with each single-pass variant,
against the oracle, stopping at the first mismatch."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle  # noqa: E402
import paper_1405_2915_amd as skel  # noqa: E402
import synth_inputs as si  # noqa: E402


def main():
    assert skel.LIB_PATH == os.environ.get("SKEL_LIBRARY"), "not the stress build"
    skel.skel_init(0, "torch")
    n = 1 << 27
    xh = si.int_uniform_i32(n, 1000, 1, 2)
    ref = torch.from_numpy(oracle.scan(xh, "exclusive", "sum", np.int64)).cuda()
    x = torch.from_numpy(xh).cuda()
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    cx, co = skel.wrap_tensor(x), skel.wrap_tensor(out)
    for variant in (2, 3):
        for rep in range(20):
            out.fill_(-1)
            skel.skel_scan(cx, co, skel.EXCLUSIVE, skel.SUM, variant=variant)
            if not torch.equal(out, ref):
                print(f"mismatch: variant {variant}, repeat {rep}", flush=True)
                return 1
        print(f"variant {variant}: 20 repeats bit-identical", flush=True)
    skel.skel_sync()
    cx.destroy()
    co.destroy()
    print("ok", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
