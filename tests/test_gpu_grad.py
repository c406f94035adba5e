"""GPU parity of the reverse-mode kernels (adjoints) against the oracle's
adjoints, through the C ABI, and of the torch.autograd functions built on them.

Bars: reverse scans as the forward scans (integers bit-exact, floating point
|y_i - y*_i| <= 1e-5 * sum of |terms|); Map backward elementwise
|dx - dx*| <= 1e-6 * |g| * (magnitude of the derivative's factors), parameter
gradients |dp - dp*| <= 1e-5 * sum |g df/dp|; MapOverlap adjoints
|dx - dx*| <= 1e-6 * sum of |w g| over the terms of each element.
"""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

MAP_OPS = {"identity": 0, "axpy": 1, "affine": 2, "tanh": 3, "affine_tanh": 4, "mul": 5,
           "square": 6}
PARAMS = {"axpy": [2.5], "affine": [0.75, -0.5], "affine_tanh": [1.5, 0.25]}
EDGES = {"clamp": 0, "const": 1, "cyclic": 2}
RED_OPS = {"sum": 0, "min": 1, "max": 2}
SCAN_SIZES = [1, 2, 3, 5, 64, 1000, 4097, 16383, 16384, 16385, 32767, 32768, 32769,
              (1 << 20) + 3]


def cont(skel, a, dtype=None):
    return skel.Container.from_numpy(a, dtype)


# ------------------------------------------------------------ reverse scans
SINGLE_PASS = (2, 3, 4, 5)  # S2 decoupled look-back, S3 its persistent form, S4 small
# tiles, S5 flat look-back


@pytest.mark.parametrize("pair", ["i32_i32", "i32_i64", "i64_i64"])
@pytest.mark.parametrize("op", list(RED_OPS))
def test_reverse_scan_int_bit_exact(skel, oracle_mod, pair, op):
    din, dout, npd = {"i32_i32": (skel.I32, skel.I32, np.int32),
                      "i32_i64": (skel.I32, skel.I64, np.int64),
                      "i64_i64": (skel.I64, skel.I64, np.int64)}[pair]
    for n in SCAN_SIZES:
        g = si.rng(8, n)
        if din == skel.I32:
            x = g.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
        else:
            x = g.integers(-2 ** 62, 2 ** 62, n, dtype=np.int64)
        for kind, code in (("reverse_inclusive", skel.REVERSE_INCLUSIVE),
                           ("reverse_exclusive", skel.REVERSE_EXCLUSIVE)):
            ref = oracle_mod.scan(x, kind, op, npd)
            for v in SINGLE_PASS:
                out = skel.Container.empty(dout, n)
                skel.skel_scan(cont(skel, x), out, code, RED_OPS[op], variant=v)
                got = out.to_numpy()
                assert np.array_equal(got, ref), (pair, op, n, kind, v,
                                                  np.flatnonzero(got != ref)[:5])


def test_reverse_scan_f32(skel, oracle_mod):
    for n in SCAN_SIZES:
        x = si.normal_f32(n, 8, 1)
        for kind, code in (("reverse_inclusive", skel.REVERSE_INCLUSIVE),
                           ("reverse_exclusive", skel.REVERSE_EXCLUSIVE)):
            ref, mag = oracle_mod.scan(x, kind)
            for v in SINGLE_PASS:
                out = skel.Container.empty(skel.F32, n)
                skel.skel_scan(cont(skel, x), out, code, skel.SUM, variant=v)
                bad = np.abs(out.to_numpy().astype(np.float64) - ref) > 1e-5 * mag + 1e-30
                assert not bad.any(), (n, kind, v, np.flatnonzero(bad)[:5])


def test_reverse_scan_variants_and_full_size(skel, oracle_mod):
    x = si.int_uniform_i32(4097, 1000, 8, 2)
    for v, ok in ((0, False), (1, False), (2, True), (3, True)):
        out = skel.Container.empty(skel.I64, x.size)
        if ok:
            skel.skel_scan(cont(skel, x), out, skel.REVERSE_EXCLUSIVE, skel.SUM, variant=v)
            assert np.array_equal(out.to_numpy(),
                                  oracle_mod.scan(x, "reverse_exclusive", "sum", np.int64))
        else:
            with pytest.raises(skel.SkelError) as e:
                skel.skel_scan(cont(skel, x), out, skel.REVERSE_EXCLUSIVE, skel.SUM, variant=v)
            assert e.value.status == skel.E_UNSUPPORTED
    # full size of the large scan workload: the first and last tiles and
    # sampled positions against the exact suffix sums
    n = 1 << 27
    xs = si.int_uniform_i32(n, 1000, 1, 2)
    out = skel.Container.empty(skel.I64, n)
    skel.skel_scan(cont(skel, xs), out, skel.REVERSE_EXCLUSIVE, skel.SUM)
    got = out.to_numpy()
    suffix = oracle_mod.scan(xs, "reverse_inclusive", "sum", out_dtype=np.int64)
    assert got[-1] == 0
    idx = np.concatenate([np.arange(40000), np.arange(n - 40000, n - 1),
                          si.rng(8, 3).integers(0, n - 1, 4000)])
    assert np.array_equal(got[idx], suffix[idx + 1])


# -------------------------------------------------------------- Map backward
def grad_scale(op, p, x, y):
    """magnitude of the derivative's factors (dx, dy) for the elementwise bar"""
    ax, ay = np.abs(x.astype(np.float64)), np.abs(y.astype(np.float64))
    one = np.ones_like(ax)
    if op in ("identity", "tanh"):
        return one, None
    if op == "axpy":
        return abs(p[0]) * one, one
    if op == "affine":
        return abs(p[0]) * one, None
    if op == "affine_tanh":
        return max(1.0, abs(p[0])) * one, None
    if op == "mul":
        return ay, ax
    return 2 * ax, None


@pytest.mark.parametrize("op", list(MAP_OPS))
@pytest.mark.parametrize("bcast", [False, True])
def test_map_backward(skel, oracle_mod, op, bcast):
    p = PARAMS.get(op, [])
    two = op in oracle_mod.TWO_INPUT_MAP_OPS
    for n in (0, 1, 3, 4, 5, 1000, 4097, (1 << 20) + 3):
        x = si.normal_f32(n, 9, 0)
        y = si.normal_f32(n, 9, 1)
        gfull = si.normal_f32(n, 9, 2)
        g1 = np.float32(0.8125)
        gv = np.full(n, g1, np.float32) if bcast else gfull
        dx_ref, dy_ref, dp_ref, dp_mag = oracle_mod.map_grad(op, p, x, gv, y if two else None)
        cx, cy = cont(skel, x), cont(skel, y)
        cg = cont(skel, np.array([g1], np.float32)) if bcast else cont(skel, gfull)
        gx, gy = skel.Container.empty(skel.F32, n), skel.Container.empty(skel.F32, n)
        gp = skel.Container.empty(skel.F32, len(p)) if p else None
        skel.skel_map_backward(MAP_OPS[op], p, [cx, cy] if two else [cx], cg,
                               [gx, gy] if two else [gx], gp)
        sx, sy = grad_scale(op, p, x, y)
        ag = np.abs(gv.astype(np.float64))
        bad = np.abs(gx.to_numpy() - dx_ref) > 1e-6 * ag * sx + 1e-30
        assert not bad.any(), (op, n, bcast, np.flatnonzero(bad)[:5])
        if two:
            bad = np.abs(gy.to_numpy() - dy_ref) > 1e-6 * ag * sy + 1e-30
            assert not bad.any(), (op, n, bcast, "dy", np.flatnonzero(bad)[:5])
        if p:
            got = gp.to_numpy().astype(np.float64)
            assert np.all(np.abs(got - dp_ref) <= 1e-5 * dp_mag + 1e-30), (op, n, got, dp_ref)


def test_map_backward_rejects_bad_calls(skel):
    x = cont(skel, np.ones(8, np.float32))
    g = cont(skel, np.ones(8, np.float32))
    d = skel.Container.empty(skel.F32, 8)

    def status(*a, **k):
        with pytest.raises(skel.SkelError) as e:
            skel.skel_map_backward(*a, **k)
        return e.value.status

    assert status(skel.MAP_TANH, None, [x], g, [x]) == skel.E_INVAL       # aliases input
    assert status(skel.MAP_TANH, None, [x], g, [g]) == skel.E_INVAL       # aliases g
    assert status(skel.MAP_TANH, None, [x], cont(skel, np.ones(3, np.float32)), [d]) \
        == skel.E_SHAPE
    assert status(skel.MAP_AFFINE, [1.0, 2.0], [x], g, [d],
                  skel.Container.empty(skel.F32, 3)) == skel.E_SHAPE
    assert status(skel.MAP_AFFINE, [1.0], [x], g, [d]) == skel.E_INVAL   # needs 2 params


# -------------------------------------------------------- MapOverlap adjoints
@pytest.mark.parametrize("edge", list(EDGES))
@pytest.mark.parametrize("r", [0, 1, 2, 4, 7])
def test_mapoverlap1d_backward(skel, oracle_mod, edge, r):
    w = si.uniform_f32(2 * r + 1, -1.0, 1.0, 9, 10 + r)
    for n in (1, 2, 5, 17, 1000, 1025, 4099, (1 << 20) + 2):
        g = si.uniform_f32(n, -1.0, 1.0, 9, 3)
        ref, mag = oracle_mod.mapoverlap1d_adjoint(g, w, r, edge)
        for v in range(skel.skel_variant_count(skel.SK_MAPOVERLAP1D_BACKWARD)):
            out = skel.Container.empty(skel.F32, n)
            skel.skel_mapoverlap1d_backward(cont(skel, g), out, w, r, EDGES[edge], variant=v)
            bad = np.abs(out.to_numpy().astype(np.float64) - ref) > 1e-6 * mag + 1e-30
            assert not bad.any(), (edge, r, n, v, np.flatnonzero(bad)[:5])


SHAPES_2D = [(1, 1), (1, 17), (13, 1), (3, 5), (64, 64), (65, 63), (257, 300)]


@pytest.mark.parametrize("edge", list(EDGES))
@pytest.mark.parametrize("ry,rx", [(4, 4), (1, 1), (3, 1), (0, 2), (8, 8)])
def test_mapoverlap2d_backward(skel, oracle_mod, edge, ry, rx):
    w2d = si.uniform_f32((2 * ry + 1) * (2 * rx + 1), -1.0, 1.0, 9, 20).reshape(
        2 * ry + 1, 2 * rx + 1)
    wy = si.uniform_f32(2 * ry + 1, 0.0, 1.0, 9, 21)
    wx = si.uniform_f32(2 * rx + 1, -1.0, 1.0, 9, 22)
    for rows, cols in SHAPES_2D:
        g = si.uniform_f32(rows * cols, -1.0, 1.0, 9, 23).reshape(rows, cols)
        for kw in ({"w2d": w2d}, {"wy": wy, "wx": wx}):
            ref, mag = oracle_mod.mapoverlap2d_adjoint(g, ry, rx, edge=edge, **kw)
            for v in range(skel.skel_variant_count(skel.SK_MAPOVERLAP2D_BACKWARD)):
                out = skel.Container.empty(skel.F32, rows, cols)
                skel.skel_mapoverlap2d_backward(cont(skel, g), out, ry=ry, rx=rx,
                                                edge=EDGES[edge], variant=v, **kw)
                bad = np.abs(out.to_numpy().reshape(rows, cols).astype(np.float64) - ref) \
                    > 1e-6 * mag + 1e-30
                assert not bad.any(), (edge, ry, rx, rows, cols, v, list(kw),
                                       np.argwhere(bad)[:5])


@pytest.mark.parametrize("edge", list(EDGES))
@pytest.mark.parametrize("ry,rx", [(1, 1), (2, 2), (0, 2)])
def test_mapoverlap2d_backward_large(skel, oracle_mod, edge, ry, rx):
    # 2^20 elements and more: the flipped transpose runs the marching-window
    # forward kernel (radius <= 2) for either weight form
    w2d = si.uniform_f32((2 * ry + 1) * (2 * rx + 1), -1.0, 1.0, 19, 20).reshape(
        2 * ry + 1, 2 * rx + 1)
    wy = si.uniform_f32(2 * ry + 1, 0.0, 1.0, 19, 21)
    wx = si.uniform_f32(2 * rx + 1, -1.0, 1.0, 19, 22)
    for rows, cols in [(1024, 1024), (1040, 1032)]:
        g = si.uniform_f32(rows * cols, -1.0, 1.0, 19, cols).reshape(rows, cols)
        for kw in ({"w2d": w2d}, {"wy": wy, "wx": wx}):
            ref, mag = oracle_mod.mapoverlap2d_adjoint(g, ry, rx, edge=edge, **kw)
            out = skel.Container.empty(skel.F32, rows, cols)
            skel.skel_mapoverlap2d_backward(cont(skel, g), out, ry=ry, rx=rx, edge=EDGES[edge],
                                            **kw)
            bad = np.abs(out.to_numpy().reshape(rows, cols).astype(np.float64) - ref) \
                > 1e-6 * mag + 1e-30
            assert not bad.any(), (edge, ry, rx, rows, cols, list(kw), np.argwhere(bad)[:5])


# ----------------------------------------------------------- autograd layer
def test_autograd_functions(skel, oracle_mod):
    import torch

    from paper_1405_2915_amd import autograd as ag
    dev = torch.device("cuda", 0)
    n = 4099
    xh, yh, gh = si.normal_f32(n, 10, 0), si.normal_f32(n, 10, 1), si.normal_f32(n, 10, 2)
    t = lambda a: torch.from_numpy(a).to(dev)

    # Map with a differentiable parameter tensor
    x, y = t(xh).requires_grad_(), t(yh).requires_grad_()
    p = torch.tensor([1.5, 0.25], dtype=torch.float32, requires_grad=True)
    out = ag.map_fn(skel.MAP_AFFINE_TANH, x, params=p)
    (out * t(gh)).sum().backward()
    dx, _, dp, dpm = oracle_mod.map_grad("affine_tanh", [1.5, 0.25], xh, gh)
    assert np.all(np.abs(x.grad.cpu().numpy() - dx) <= 1e-6 * np.abs(gh) * 1.5 + 1e-30)
    assert np.all(np.abs(p.grad.numpy() - dp) <= 1e-5 * dpm + 1e-30)

    # two-input Map
    x.grad = None
    out = ag.map_fn(skel.MAP_MUL, x, y)
    (out * t(gh)).sum().backward()
    dx, dy, _, _ = oracle_mod.map_grad("mul", [], xh, gh, yh)
    assert np.all(np.abs(x.grad.cpu().numpy() - dx) <= 1e-6 * np.abs(gh * yh) + 1e-30)
    assert np.all(np.abs(y.grad.cpu().numpy() - dy) <= 1e-6 * np.abs(gh * xh) + 1e-30)

    # sum, dot: the upstream scalar broadcast through the chain rule
    x.grad = y.grad = None
    s = ag.reduce_sum_fn(x)
    assert abs(s.item() - oracle_mod.reduce("sum", xh)) <= 1e-5 * oracle_mod.abs_sum(xh)
    (3.0 * s).backward()
    assert torch.all(x.grad == 3.0)
    x.grad = None
    d = ag.mapreduce_sum_fn(skel.MAP_MUL, x, y)
    d.backward()
    assert torch.equal(x.grad, t(yh)) and torch.equal(y.grad, t(xh))

    # stencils
    w5 = si.binomial5_weights()
    x.grad = None
    o1 = ag.mapoverlap1d_fn(x, w5, 2, skel.EDGE_CLAMP)
    (o1 * t(gh)).sum().backward()
    ref, mag = oracle_mod.mapoverlap1d_adjoint(gh, w5, 2, "clamp")
    assert np.all(np.abs(x.grad.cpu().numpy() - ref) <= 1e-6 * mag + 1e-30)
    img = t(si.uniform_f32(65 * 63, 0.0, 1.0, 10, 3).reshape(65, 63)).requires_grad_()
    gimg = si.normal_f32(65 * 63, 10, 4).reshape(65, 63)
    g9 = si.gaussian_weights(4, 2.0)
    o2 = ag.mapoverlap2d_fn(img, wy=g9, wx=g9, edge=skel.EDGE_CLAMP)
    (o2 * t(gimg)).sum().backward()
    ref, mag = oracle_mod.mapoverlap2d_adjoint(gimg, 4, 4, wy=g9, wx=g9, edge="clamp")
    assert np.all(np.abs(img.grad.cpu().numpy() - ref) <= 1e-6 * mag + 1e-30)

    # scan: the gradient of prefix sums is the suffix sum of the upstream gradient
    x.grad = None
    sc = ag.scan_sum_fn(x, skel.EXCLUSIVE)
    ref, mag = oracle_mod.scan(xh, "exclusive")
    assert np.all(np.abs(sc.detach().cpu().numpy() - ref) <= 1e-5 * mag + 1e-30)
    (sc * t(gh)).sum().backward()
    ref, mag = oracle_mod.scan(gh, "reverse_exclusive")
    assert np.all(np.abs(x.grad.cpu().numpy() - ref) <= 1e-5 * mag + 1e-30)

    # the layer of the batched fields: stencil on every field, then prefix sums
    # along the rows; the gradient is the stencil's transpose of the rows'
    # suffix sums of the upstream gradient
    F_, H_, W_ = 3, 33, 70
    w5 = si.five_point_weights(0.5, 0.1, 0.2, 0.05, 0.15)
    xf = si.normal_f32(F_ * H_ * W_, 10, 8).reshape(F_, H_, W_)
    gf = si.normal_f32(F_ * H_ * W_, 10, 9).reshape(F_, H_, W_)
    xt = t(xf).requires_grad_()
    zt = ag.scan_rows_sum_fn(ag.mapoverlap2d_fields_fn(xt, w2d=w5))
    (zt * t(gf)).sum().backward()
    for k in range(F_):
        yref, ymag = oracle_mod.mapoverlap2d(xf[k], 1, 1, w2d=w5, edge="clamp")
        got = zt.detach()[k].cpu().numpy()
        # the oracle's row scans of the stencil output (rounded once to
        # binary32, 2^-24 of each magnitude) and of the term magnitudes
        zref, _ = oracle_mod.scan_rows(yref.astype(np.float32), "inclusive")
        zmag, _ = oracle_mod.scan_rows(ymag.astype(np.float32), "inclusive")
        assert np.all(np.abs(got - zref) <= 1e-5 * zmag + 1e-30), k
        gy, gmag = oracle_mod.scan_rows(gf[k], "reverse_inclusive")
        dref, _ = oracle_mod.mapoverlap2d_adjoint(gy.astype(np.float32), 1, 1, w2d=w5,
                                                  edge="clamp")
        _, dmag = oracle_mod.mapoverlap2d_adjoint(gmag.astype(np.float32), 1, 1,
                                                  w2d=np.abs(w5), edge="clamp")
        assert np.all(np.abs(xt.grad[k].cpu().numpy() - dref) <= 1e-5 * dmag + 1e-30), k

    # scan along the last axis of a batch of fields (3 x 40 x 2048, and an odd
    # width): each row's gradient is its own suffix sum
    for shape in [(3, 40, 2048), (5, 37)]:
        nel = int(np.prod(shape))
        fh = si.normal_f32(nel, 10, 6).reshape(shape)
        gf = si.normal_f32(nel, 10, 7).reshape(shape)
        f = t(fh).requires_grad_()
        sr = ag.scan_rows_sum_fn(f, skel.INCLUSIVE)
        ref, mag = oracle_mod.scan_rows(fh.reshape(-1, shape[-1]), "inclusive")
        got = sr.detach().cpu().numpy().reshape(ref.shape)
        assert np.all(np.abs(got - ref) <= 1e-5 * mag + 1e-30), shape
        (sr * t(gf)).sum().backward()
        ref, mag = oracle_mod.scan_rows(gf.reshape(-1, shape[-1]), "reverse_inclusive")
        got = f.grad.cpu().numpy().reshape(ref.shape)
        assert np.all(np.abs(got - ref) <= 1e-5 * mag + 1e-30), shape


def test_wrap_tensor_round_trip(skel, oracle_mod):
    import torch
    dev = torch.device("cuda", 0)
    xh = si.normal_f32(1000, 10, 5)
    x = torch.from_numpy(xh).to(dev)
    y = torch.empty_like(x)
    cx, cy = skel.wrap_tensor(x), skel.wrap_tensor(y)
    skel.skel_map(skel.MAP_AFFINE, [2.0, 1.0], [cx], cy)
    assert cy.stats()["h2d"] == 0 and cx.stats()["h2d"] == 0
    got = cy.to_numpy()  # host read of the wrapped device copy: one copy
    assert cy.stats()["d2h"] == 1
    ref = oracle_mod.map_f32("affine", [2.0, 1.0], xh)
    assert np.all(np.abs(got - ref) <= 1e-6 * (2 * np.abs(xh) + 1))
    assert torch.equal(y.cpu(), torch.from_numpy(got))
    cx.destroy()
    cy.destroy()
    assert torch.isfinite(x).all()  # the caller's memory is untouched and alive
    with pytest.raises(skel.SkelError) as e:  # a view at a 4-byte offset
        skel.wrap_tensor(x[1:5])
    assert e.value.status == skel.E_INVAL
    # an empty tensor of any shape is an empty container (Reduce: the identity)
    ce = skel.wrap_tensor(torch.empty((0, 5), device=dev))
    assert ce.shape == (1, 0)
    out = skel.Container.empty(skel.F32, 1)
    skel.skel_reduce(skel.SUM, ce, out)
    assert out.to_numpy()[0] == 0.0
    ce.destroy()
