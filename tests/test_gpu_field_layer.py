"""The batched field layer at its full size (64 fields of 2048 x 2048 f32): a
5-point stencil on every field, then prefix sums along every field row, and the
backward pass (reverse row-wise scan of the upstream gradient, then the
stencil's transpose on every field), run through the C ABI exactly as the
benchmark runs it (one batched-field stencil call per pass).  Two whole fields
(the first and the last: 8.4 million outputs per pass) are checked against the
oracle element by element, and sampled rows of other fields: a row of the
stencil (or of its transpose) depends only on the three field rows around it,
so the oracle runs on those three rows and the scan on the whole row.

Bars: forward |z - z*| <= 1e-5 * (prefix sums of the stencil's term
magnitudes); backward |dx - dx*| <= 1e-5 * (the transpose's term magnitudes
over the reverse prefix sums of |g|)."""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

F, H, W = 64, 2048, 2048
FULL_FIELDS = (0, F - 1)
SAMPLES = [(1, 0), (5, 1), (9, 1000), (62, 2047), (31, 2046), (17, 555)]


def block(a, r):
    """The three field rows around row r (clamped at the field's ends) and the
    index of row r in them."""
    lo = min(max(r - 1, 0), H - 3)
    return a[lo:lo + 3], r - lo


def test_field_layer_full_size(skel, oracle_mod):
    import torch
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(si.BASE_SEED + 1000 * 4)
    x = torch.randn((F, H, W), generator=gen, device=dev)
    gz = torch.randn((F, H, W), generator=gen, device=dev)
    y, z, gy, gx = (torch.empty_like(x) for _ in range(4))
    w5 = si.five_point_weights(0.5, 0.1, 0.2, 0.05, 0.15)  # asymmetric: catches flips
    made = []

    def wrap(t):
        made.append(skel.wrap_tensor(t))
        return made[-1]
    cx, cy, cz, cgz, cgy, cgx = (wrap(t.view(-1, W)) for t in (x, y, z, gz, gy, gx))
    skel.skel_mapoverlap2d_fields(cx, cy, F, w2d=w5, edge=skel.EDGE_CLAMP)
    skel.skel_scan_rows(cy, cz, skel.INCLUSIVE, skel.SUM)
    skel.skel_scan_rows(cgz, cgy, skel.REVERSE_INCLUSIVE, skel.SUM)
    skel.skel_mapoverlap2d_fields_backward(cgy, cgx, F, w2d=w5, edge=skel.EDGE_CLAMP)
    skel.skel_sync()
    for f in FULL_FIELDS:
        xf, gzf = x[f].cpu().numpy(), gz[f].cpu().numpy()
        yref, mag = oracle_mod.mapoverlap2d(xf, 1, 1, w2d=w5, edge="clamp")
        zref, _ = oracle_mod.scan_rows(yref.astype(np.float32), "inclusive")
        bound = 1e-5 * oracle_mod.scan_rows(mag.astype(np.float32), "inclusive")[0] + 1e-30
        err = np.abs(z[f].cpu().numpy().astype(np.float64) - zref)
        assert np.all(err <= bound), ("forward", f, np.unravel_index(np.argmax(err - bound),
                                                                     err.shape))
        gyf, gmag = oracle_mod.scan_rows(gzf, "reverse_inclusive")
        assert np.all(np.abs(gy[f].cpu().numpy() - gyf) <= 1e-5 * gmag + 1e-30), ("rev", f)
        dref, _ = oracle_mod.mapoverlap2d_adjoint(gyf.astype(np.float32), 1, 1, w2d=w5,
                                                  edge="clamp")
        _, dmag = oracle_mod.mapoverlap2d_adjoint(gmag.astype(np.float32), 1, 1,
                                                  w2d=np.abs(w5), edge="clamp")
        err = np.abs(gx[f].cpu().numpy().astype(np.float64) - dref)
        assert np.all(err <= 1e-5 * dmag + 1e-30), ("backward", f)
    for f, r in SAMPLES:
        xb, k = block(x[f].cpu().numpy(), r)
        yb, mag = oracle_mod.mapoverlap2d(xb, 1, 1, w2d=w5, edge="clamp")
        # the oracle's scan of the stencil row (rounded once to binary32: at
        # most 2^-24 of each |term| sum, far inside the bar), and the prefix
        # sums of the term magnitudes as the bound
        zref, _ = oracle_mod.scan(yb[k].astype(np.float32), "inclusive", "sum")
        bound = 1e-5 * oracle_mod.scan(mag[k].astype(np.float32), "inclusive", "sum")[0] + 1e-30
        got = z[f, r].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - zref) <= bound), ("forward", f, r)
        gb, k = block(gz[f].cpu().numpy(), r)
        gyb, gmag = oracle_mod.scan_rows(gb, "reverse_inclusive")
        assert np.all(np.abs(gy[f, r].cpu().numpy() - gyb[k]) <= 1e-5 * gmag[k] + 1e-30)
        # the transpose of the exact reverse sums, bounded by their magnitudes
        dref, _ = oracle_mod.mapoverlap2d_adjoint(gyb.astype(np.float32), 1, 1, w2d=w5,
                                                  edge="clamp")
        _, dmag = oracle_mod.mapoverlap2d_adjoint(gmag.astype(np.float32), 1, 1,
                                                  w2d=np.abs(w5), edge="clamp")
        got = gx[f, r].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - dref[k]) <= 1e-5 * dmag[k] + 1e-30), ("backward", f, r)
    for c in made:
        c.destroy()
