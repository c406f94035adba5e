"""The call chain Map -> MapOverlap 2D -> Reduce SUM through the C ABI (both
variants: composed and fused) and through its autograd function, against the
oracle's binary64 composition of the same three skeleton definitions and its
reverse mode.

Bars: the loss |L - L*| <= 1e-5 * (sum of |W[a][b] * read value| over every
term), the Reduce bound; the gradient elementwise |dx - dx*| <= 1e-6 * g1 *
(sum of |W| over the taps that read the element) * max(1, |p0|) (the
magnitudes of the derivative's factors, as for the Map adjoint: 1 - tanh^2 is
at most 1); parameter gradients |dp - dp*| <= 1e-5 * sum |terms|."""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

OPS = {"identity": (0, []), "affine": (2, [0.75, -0.5]), "tanh": (3, []),
       "affine_tanh": (4, [0.75, -0.25]), "square": (6, [])}
EDGES = {"clamp": 0, "const": 1, "cyclic": 2}


def _asym5():
    return si.five_point_weights(0.5, 0.1, 0.2, 0.05, 0.15)


def _weights(kind, seed):
    """(w2d, wy, wx, ry, rx) of a weight form"""
    if kind == "5pt":
        return _asym5(), None, None, 1, 1
    if kind == "dense5x3":
        return si.uniform_f32(5 * 3, -1.0, 1.0, 9, seed).reshape(5, 3), None, None, 2, 1
    if kind == "sep9":
        g = si.gaussian_weights(4, 2.0)
        return None, g, si.binomial5_weights(), 4, 2
    if kind == "dense17x3":
        return si.uniform_f32(17 * 3, -1.0, 1.0, 9, seed).reshape(17, 3), None, None, 8, 1
    raise KeyError(kind)


def _factor_mag(skel_mod, oracle_mod, x, w2d, wy, wx, ry, rx, edge, g1, p0):
    """sum of |W g1| over the taps that read each element, times max(1, |p0|)"""
    wa = None if w2d is None else np.abs(w2d)
    ya = None if wy is None else np.abs(wy)
    xa = None if wx is None else np.abs(wx)
    _, mag, _, _ = oracle_mod.chain_grad("identity", [], np.zeros_like(x), ry, rx, abs(g1),
                                         w2d=wa, wy=ya, wx=xa, edge=edge)
    return mag * max(1.0, abs(p0))


def _run(skel, x3, op, params, w2d, wy, wx, ry, rx, edge, pad, variant, g1):
    f, h, w = x3.shape
    cx = skel.Container.from_numpy(x3.reshape(f * h, w))
    out = skel.Container.empty(skel.F32, 1)
    skel.skel_map_overlap2d_reduce(OPS[op][0], params, cx, f, out, w2d=w2d, wy=wy, wx=wx, ry=ry,
                                   rx=rx, edge=EDGES[edge], pad=pad, variant=variant)
    g = skel.Container.from_numpy(np.array([g1], np.float32))
    dx = skel.Container.empty(skel.F32, f * h, w)
    npar = len(params)
    dp = skel.Container.empty(skel.F32, npar) if npar else None
    skel.skel_map_overlap2d_reduce_backward(OPS[op][0], params, cx, f, g, dx, dp, w2d=w2d,
                                            wy=wy, wx=wx, ry=ry, rx=rx, edge=EDGES[edge],
                                            variant=variant)
    return (float(out.to_numpy()[0]), dx.to_numpy().reshape(f, h, w),
            dp.to_numpy() if npar else np.zeros(0))


def _check(skel, oracle_mod, x3, op, wkind, edge, variant, pad=0.375, g1=1.25):
    params = OPS[op][1]
    w2d, wy, wx, ry, rx = _weights(wkind, 90)
    loss, dx, dp = _run(skel, x3, op, params, w2d, wy, wx, ry, rx, edge, pad, variant, g1)
    ref, mag = oracle_mod.chain(op, params, x3, ry, rx, w2d=w2d, wy=wy, wx=wx, edge=edge,
                                pad=pad)
    assert abs(loss - ref) <= 1e-5 * mag + 1e-30, ("loss", loss, ref, mag)
    dref, _, dpref, dpmag = oracle_mod.chain_grad(op, params, x3, ry, rx, g1, w2d=w2d, wy=wy,
                                                  wx=wx, edge=edge)
    bar = 1e-6 * _factor_mag(skel, oracle_mod, x3, w2d, wy, wx, ry, rx, edge, g1,
                             params[0] if params else 1.0)
    err = np.abs(dx.astype(np.float64) - dref)
    assert np.all(err <= bar + 1e-30), ("dx", float(err.max()), np.unravel_index(err.argmax(),
                                                                                 err.shape))
    assert np.all(np.abs(dp - dpref) <= 1e-5 * dpmag + 1e-30), ("dp", dp, dpref)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("edge", ["clamp", "const", "cyclic"])
@pytest.mark.parametrize("op", list(OPS))
def test_chain_16x16(skel, oracle_mod, variant, edge, op):
    """The differentiation workload's check size: two 16 x 16 fields."""
    x = si.normal_f32(2 * 16 * 16, 9, 1).reshape(2, 16, 16)
    _check(skel, oracle_mod, x, op, "5pt", edge, variant)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("shape,wkind", [((1, 1, 1), "5pt"), ((3, 2, 3), "5pt"),
                                         ((2, 37, 41), "dense5x3"), ((1, 5, 1030), "sep9"),
                                         ((4, 3, 7), "sep9"), ((2, 300, 257), "5pt"),
                                         ((5, 20, 6), "dense17x3"), ((7, 64, 64), "dense5x3")])
@pytest.mark.parametrize("edge", ["clamp", "const", "cyclic"])
def test_chain_shapes(skel, oracle_mod, variant, shape, wkind, edge):
    """Fields smaller than the stencil, rows that are not whole vectors (so a
    vector straddles rows and fields), several fields per launch chunk."""
    x = si.normal_f32(int(np.prod(shape)), 9, 2).reshape(shape)
    _check(skel, oracle_mod, x, "affine_tanh", wkind, edge, variant)


def test_chain_variants_agree_and_are_deterministic(skel):
    x = si.normal_f32(3 * 130 * 128, 9, 3).reshape(3, 130, 128)
    w2d, _, _, _, _ = _weights("5pt", 0)
    got = []
    for variant in (1, 1, 0, 0):
        loss, dx, dp = _run(skel, x, "affine_tanh", [0.75, -0.25], w2d, None, None, 1, 1, "clamp",
                            0.0, variant, 1.0)
        got.append((loss, dx, dp))
    # each variant repeats bit for bit (fixed combination order)
    assert got[0][0] == got[1][0] and np.array_equal(got[0][1], got[1][1])
    assert got[2][0] == got[3][0] and np.array_equal(got[2][1], got[3][1])


def test_chain_empty_and_validation(skel):
    import paper_1405_2915_amd as sk
    out = skel.Container.empty(skel.F32, 1)
    e = skel.Container.empty(skel.F32, 4, 0)
    skel.skel_map_overlap2d_reduce(4, [0.75, -0.25], e, 2, out, w2d=_asym5())
    assert out.to_numpy()[0] == 0.0
    x = skel.Container.from_numpy(np.ones((6, 8), np.float32))

    def status(*a, **k):
        try:
            skel.skel_map_overlap2d_reduce(*a, **k)
        except sk.SkelError as err:
            return err.status
        return sk.OK
    assert status(1, [2.5], x, 1, out, w2d=_asym5()) == sk.E_INVAL       # AXPY: two inputs
    assert status(4, [0.75], x, 1, out, w2d=_asym5()) == sk.E_INVAL      # one parameter short
    assert status(4, [0.75, 0.1], x, 4, out, w2d=_asym5()) == sk.E_SHAPE  # 6 rows, 4 fields
    two = skel.Container.empty(skel.F32, 2)
    assert status(4, [0.75, 0.1], x, 1, two, w2d=_asym5()) == sk.E_SHAPE  # output not 1 elt
    assert status(4, [0.75, 0.1], x, 1, x, w2d=_asym5()) == sk.E_INVAL   # output aliases input
    assert status(4, [0.75, 0.1], x, 1, out, w2d=_asym5(), variant=7) == sk.E_UNSUPPORTED


def test_chain_autograd(skel, oracle_mod):
    import torch
    from paper_1405_2915_amd import autograd as ag
    x = si.normal_f32(3 * 16 * 16, 9, 4).reshape(3, 16, 16)
    w5 = _asym5()
    xt = torch.from_numpy(x).cuda().requires_grad_()
    p = torch.tensor([0.75, -0.25], dtype=torch.float32, requires_grad=True)
    loss = ag.map_overlap2d_reduce_fn(4, xt, p, w2d=w5)
    (2.0 * loss).backward()
    ref, mag = oracle_mod.chain("affine_tanh", [0.75, -0.25], x, 1, 1, w2d=w5)
    assert abs(loss.item() - ref) <= 1e-5 * mag
    dref, _, dpref, dpmag = oracle_mod.chain_grad("affine_tanh", [0.75, -0.25], x, 1, 1, 2.0,
                                                  w2d=w5)
    bar = 1e-6 * _factor_mag(skel, oracle_mod, x, w5, None, None, 1, 1, "clamp", 2.0, 0.75)
    assert np.all(np.abs(xt.grad.cpu().numpy() - dref) <= bar)
    assert np.all(np.abs(p.grad.numpy() - dpref) <= 1e-5 * dpmag)


def test_chain_full_size(skel, oracle_mod):
    """The differentiation workload at its size: 64 fields of 2048 x 2048
    N(0, 1), loss = Reduce(5-point MapOverlap2D(tanh(w x + b))), fused, as
    the benchmark runs it: the loss against the oracle over all 64 fields, the
    gradient element by element on three whole fields (a field's gradient
    depends on that field alone) and the parameter gradients over all."""
    import torch
    F, H, W = 64, 2048, 2048
    x = si.normal_f32(F * H * W, 4, 0).reshape(F, H, W)
    w5 = si.five_point_weights()
    params = [0.75, -0.25]
    xt = torch.from_numpy(x).cuda()
    cx = skel.wrap_tensor(xt.view(F * H, W))
    out = skel.Container.empty(skel.F32, 1)
    skel.skel_map_overlap2d_reduce(4, params, cx, F, out, w2d=w5)
    g = skel.Container.from_numpy(np.array([1.0], np.float32))
    dxt = torch.empty_like(xt)
    cdx = skel.wrap_tensor(dxt.view(F * H, W))
    dp = skel.Container.empty(skel.F32, 2)
    skel.skel_map_overlap2d_reduce_backward(4, params, cx, F, g, cdx, dp, w2d=w5)
    skel.skel_sync()
    ref, mag = oracle_mod.chain("affine_tanh", params, x, 1, 1, w2d=w5)
    loss = float(out.to_numpy()[0])
    assert abs(loss - ref) <= 1e-5 * mag, (loss, ref, mag)
    for f in (0, 31, 63):
        dref, _, _, _ = oracle_mod.chain_grad("affine_tanh", params, x[f], 1, 1, 1.0, w2d=w5)
        bar = 1e-6 * _factor_mag(skel, oracle_mod, x[f:f + 1], w5, None, None, 1, 1, "clamp", 1.0,
                                 0.75)[0]
        got = dxt[f].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - dref) <= bar), f
    _, _, dpref, dpmag = oracle_mod.chain_grad("affine_tanh", params, x, 1, 1, 1.0, w2d=w5)
    assert np.all(np.abs(dp.to_numpy() - dpref) <= 1e-5 * dpmag), (dp.to_numpy(), dpref)
    cx.destroy()
    cdx.destroy()
