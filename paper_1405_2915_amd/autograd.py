"""torch.autograd functions over the skeletons.

Forward and backward both run in libskel's HIP kernels; torch only holds the
tensors (wrapped as containers over their device memory, so nothing is
copied) and orders the calls on its current stream.  The backward kernels are
the reverse-mode adjoints declared in include/skel.h:

    map_fn             chain rule of the element function (parameter
                       gradients summed over the elements)
    reduce_sum_fn      gradient broadcast (Map backward of the identity)
    mapreduce_sum_fn   Map backward with the broadcast upstream gradient
    mapoverlap1d_fn    transposed neighbourhood map (clamped reads
    mapoverlap2d_fn    accumulate onto the edge elements)
    mapoverlap2d_fields_fn  the same over a batch of fields, one launch
    map_overlap2d_reduce_fn  the call chain Map -> MapOverlap 2D -> Reduce SUM
                       as one call (fused: reads x once), and its adjoint in
                       one pass (dx and the parameter gradients)
    scan_sum_fn        reverse scan of the upstream gradient
    scan_rows_sum_fn   reverse scan of each row of the upstream gradient

All tensors are float32 CUDA tensors.  Stencil weights are constants (no
gradient); Map parameters get a gradient when given as a tensor that
requires one.
"""
from __future__ import annotations

import contextlib

import numpy as np
import torch

from . import (EDGE_CLAMP, EXCLUSIVE, INCLUSIVE, MAP_AFFINE, MAP_AFFINE_TANH, MAP_AXPY,
               MAP_IDENTITY, MAP_MUL, REVERSE_EXCLUSIVE, REVERSE_INCLUSIVE, SUM, skel_map,
               skel_map_backward, skel_mapoverlap1d, skel_mapoverlap1d_backward,
               skel_mapoverlap2d, skel_mapoverlap2d_backward, skel_mapoverlap2d_fields,
               skel_mapoverlap2d_fields_backward, skel_mapreduce, skel_reduce, skel_scan,
               skel_scan_rows, wrap_tensor, skel_map_overlap2d_reduce,
               skel_map_overlap2d_reduce_backward, VARIANT_AUTO)

_TWO_INPUTS = {MAP_AXPY, MAP_MUL}
_NPARAMS = {MAP_AXPY: 1, MAP_AFFINE: 2, MAP_AFFINE_TANH: 2}


@contextlib.contextmanager
def _wrapped(*tensors):
    """Containers over the tensors' memory for the duration of one call."""
    cs = []
    try:
        for t in tensors:
            cs.append(None if t is None else wrap_tensor(t))
        yield cs
    finally:
        for c in cs:
            if c is not None:
                c.destroy()


def _f32(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError(f"{name} must be a float32 CUDA tensor")
    t = t.contiguous()
    # the kernels read 16-byte vectors: a view at an unaligned offset is
    # copied into a fresh (aligned) allocation first
    return t if t.data_ptr() % 16 == 0 else t.clone()


def _param_values(params):
    if params is None:
        return [], None
    if isinstance(params, torch.Tensor):
        return [float(v) for v in params.detach().reshape(-1).cpu().tolist()], params
    return [float(v) for v in params], None


class _MapFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, pvals, ptensor, x, y):
        out = torch.empty_like(x)
        with _wrapped(x, y, out) as (cx, cy, co):
            skel_map(op, pvals, [cx, cy] if y is not None else [cx], co)
        ctx.op, ctx.pvals = op, pvals
        ctx.has_pt = ptensor is not None
        ctx.save_for_backward(x, y, ptensor)
        return out

    @staticmethod
    def backward(ctx, g):
        x, y, ptensor = ctx.saved_tensors
        g = _f32(g, "grad")
        dx = torch.empty_like(x)
        dy = torch.empty_like(y) if y is not None else None
        np_ = _NPARAMS.get(ctx.op, 0)
        want_p = ctx.has_pt and ctx.needs_input_grad[2] and np_ > 0
        dp = torch.empty(np_, dtype=torch.float32, device=x.device) if want_p else None
        with _wrapped(x, y, g, dx, dy, dp) as (cx, cy, cg, cdx, cdy, cdp):
            ins = [cx, cy] if y is not None else [cx]
            grads = [cdx, cdy] if y is not None else [cdx]
            skel_map_backward(ctx.op, ctx.pvals, ins, cg, grads, cdp)
        gp = dp.reshape(ptensor.shape).to(ptensor.device) if want_p else None
        return None, None, gp, dx, dy


def map_fn(op: int, x, y=None, params=None):
    """out = f(x, y; params) elementwise, differentiable in x, y and params."""
    x = _f32(x, "x")
    if op in _TWO_INPUTS:
        y = _f32(y, "y")
        if y.shape != x.shape:
            raise ValueError("x and y shapes differ")
    else:
        y = None
    pvals, pt = _param_values(params)
    return _MapFn.apply(op, pvals, pt, x, y)


class _ReduceSumFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        out = torch.empty(1, dtype=torch.float32, device=x.device)
        with _wrapped(x, out) as (cx, co):
            skel_reduce(SUM, cx, co)
        ctx.save_for_backward(x)
        return out.reshape(())

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        g1 = _f32(g.reshape(1), "grad")
        dx = torch.empty_like(x)
        with _wrapped(x, g1, dx) as (cx, cg, cdx):
            skel_map_backward(MAP_IDENTITY, None, [cx], cg, [cdx])
        return dx


def reduce_sum_fn(x):
    """sum of all elements (binary32 accumulation), differentiable."""
    return _ReduceSumFn.apply(_f32(x, "x"))


class _MapReduceSumFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, pvals, ptensor, x, y):
        out = torch.empty(1, dtype=torch.float32, device=x.device)
        with _wrapped(x, y, out) as (cx, cy, co):
            skel_mapreduce(op, pvals, [cx, cy] if y is not None else [cx], SUM, co)
        ctx.op, ctx.pvals = op, pvals
        ctx.has_pt = ptensor is not None
        ctx.save_for_backward(x, y, ptensor)
        return out.reshape(())

    @staticmethod
    def backward(ctx, g):
        x, y, ptensor = ctx.saved_tensors
        g1 = _f32(g.reshape(1), "grad")
        dx = torch.empty_like(x)
        dy = torch.empty_like(y) if y is not None else None
        np_ = _NPARAMS.get(ctx.op, 0)
        want_p = ctx.has_pt and ctx.needs_input_grad[2] and np_ > 0
        dp = torch.empty(np_, dtype=torch.float32, device=x.device) if want_p else None
        with _wrapped(x, y, g1, dx, dy, dp) as (cx, cy, cg, cdx, cdy, cdp):
            ins = [cx, cy] if y is not None else [cx]
            grads = [cdx, cdy] if y is not None else [cdx]
            skel_map_backward(ctx.op, ctx.pvals, ins, cg, grads, cdp)
        gp = dp.reshape(ptensor.shape).to(ptensor.device) if want_p else None
        return None, None, gp, dx, dy


def mapreduce_sum_fn(op: int, x, y=None, params=None):
    """sum_i f(x_i, y_i; params) without a stored intermediate, differentiable."""
    x = _f32(x, "x")
    if op in _TWO_INPUTS:
        y = _f32(y, "y")
    else:
        y = None
    pvals, pt = _param_values(params)
    return _MapReduceSumFn.apply(op, pvals, pt, x, y)


class _Overlap1DFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, w, radius, edge, pad):
        out = torch.empty_like(x)
        with _wrapped(x, out) as (cx, co):
            skel_mapoverlap1d(cx, co, w, radius, edge, pad)
        ctx.w, ctx.radius, ctx.edge = w, radius, edge
        return out

    @staticmethod
    def backward(ctx, g):
        g = _f32(g, "grad")
        dx = torch.empty_like(g)
        with _wrapped(g, dx) as (cg, cdx):
            skel_mapoverlap1d_backward(cg, cdx, ctx.w, ctx.radius, ctx.edge)
        return dx, None, None, None, None


def mapoverlap1d_fn(x, w, radius: int, edge: int = EDGE_CLAMP, pad: float = 0.0):
    """1D neighbourhood map over a flat tensor, differentiable in x."""
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
    return _Overlap1DFn.apply(_f32(x, "x").reshape(-1), w, int(radius), int(edge), float(pad))


class _Overlap2DFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, w2d, wy, wx, edge, pad):
        out = torch.empty_like(x)
        with _wrapped(x, out) as (cx, co):
            skel_mapoverlap2d(cx, co, w2d=w2d, wy=wy, wx=wx, edge=edge, pad=pad)
        ctx.w2d, ctx.wy, ctx.wx, ctx.edge = w2d, wy, wx, edge
        return out

    @staticmethod
    def backward(ctx, g):
        g = _f32(g, "grad")
        dx = torch.empty_like(g)
        with _wrapped(g, dx) as (cg, cdx):
            skel_mapoverlap2d_backward(cg, cdx, w2d=ctx.w2d, wy=ctx.wy, wx=ctx.wx,
                                       edge=ctx.edge)
        return dx, None, None, None, None, None


def mapoverlap2d_fn(x, w2d=None, wy=None, wx=None, edge: int = EDGE_CLAMP, pad: float = 0.0):
    """2D neighbourhood map over a (rows, cols) tensor, differentiable in x."""
    x = _f32(x, "x")
    if x.dim() != 2:
        raise ValueError("x must be 2D")
    cv = lambda a: None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return _Overlap2DFn.apply(x, cv(w2d), cv(wy), cv(wx), int(edge), float(pad))


class _Overlap2DFieldsFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, fields, w2d, wy, wx, edge, pad):
        out = torch.empty_like(x)
        with _wrapped(x, out) as (cx, co):
            skel_mapoverlap2d_fields(cx, co, fields, w2d=w2d, wy=wy, wx=wx, edge=edge, pad=pad)
        ctx.fields, ctx.w2d, ctx.wy, ctx.wx, ctx.edge = fields, w2d, wy, wx, edge
        return out

    @staticmethod
    def backward(ctx, g):
        g = _f32(g, "grad")
        dx = torch.empty_like(g)
        with _wrapped(g, dx) as (cg, cdx):
            skel_mapoverlap2d_fields_backward(cg, cdx, ctx.fields, w2d=ctx.w2d, wy=ctx.wy,
                                              wx=ctx.wx, edge=ctx.edge)
        return dx, None, None, None, None, None, None


def mapoverlap2d_fields_fn(x, w2d=None, wy=None, wx=None, edge: int = EDGE_CLAMP,
                           pad: float = 0.0):
    """2D neighbourhood map over every (H, W) field of a (fields, H, W) tensor
    (each with its own borders), in one launch; differentiable in x."""
    x = _f32(x, "x")
    if x.dim() != 3:
        raise ValueError("x must be (fields, H, W)")
    f, h, w = x.shape
    cv = lambda a: None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    out = _Overlap2DFieldsFn.apply(x.reshape(f * h, w), int(f), cv(w2d), cv(wy), cv(wx),
                                   int(edge), float(pad))
    return out.reshape(f, h, w)


class _MapOverlapReduceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, op, pvals, ptensor, x, fields, w2d, wy, wx, edge, pad, variant):
        out = torch.empty(1, dtype=torch.float32, device=x.device)
        with _wrapped(x, out) as (cx, co):
            skel_map_overlap2d_reduce(op, pvals, cx, fields, co, w2d=w2d, wy=wy, wx=wx,
                                      edge=edge, pad=pad, variant=variant)
        ctx.op, ctx.pvals, ctx.fields = op, pvals, fields
        ctx.w2d, ctx.wy, ctx.wx, ctx.edge, ctx.variant = w2d, wy, wx, edge, variant
        ctx.has_pt = ptensor is not None
        ctx.save_for_backward(x, ptensor)
        return out.reshape(())

    @staticmethod
    def backward(ctx, g):
        x, ptensor = ctx.saved_tensors
        g1 = _f32(g.reshape(1), "grad")
        dx = torch.empty_like(x)
        np_ = _NPARAMS.get(ctx.op, 0)
        want_p = ctx.has_pt and ctx.needs_input_grad[2] and np_ > 0
        dp = torch.empty(np_, dtype=torch.float32, device=x.device) if want_p else None
        with _wrapped(x, g1, dx, dp) as (cx, cg, cdx, cdp):
            skel_map_overlap2d_reduce_backward(ctx.op, ctx.pvals, cx, ctx.fields, cg, cdx, cdp,
                                               w2d=ctx.w2d, wy=ctx.wy, wx=ctx.wx, edge=ctx.edge,
                                               variant=ctx.variant)
        gp = dp.reshape(ptensor.shape).to(ptensor.device) if want_p else None
        return None, None, gp, dx, None, None, None, None, None, None, None


def map_overlap2d_reduce_fn(op: int, x, params=None, w2d=None, wy=None, wx=None,
                            edge: int = EDGE_CLAMP, pad: float = 0.0,
                            variant: int = VARIANT_AUTO):
    """sum over every field of the 2D neighbourhood map of f(x; params), for x
    of shape (fields, H, W) or (H, W): the chain Map -> MapOverlap 2D ->
    Reduce SUM in one call, differentiable in x and in params (a tensor)."""
    x = _f32(x, "x")
    if x.dim() == 2:
        x = x.unsqueeze(0)
    if x.dim() != 3:
        raise ValueError("x must be (fields, H, W) or (H, W)")
    f, h, w = x.shape
    pvals, pt = _param_values(params)
    cv = lambda a: None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return _MapOverlapReduceFn.apply(op, pvals, pt, x.reshape(f * h, w), int(f), cv(w2d),
                                     cv(wy), cv(wx), int(edge), float(pad), int(variant))


class _ScanSumFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, kind):
        out = torch.empty_like(x)
        with _wrapped(x, out) as (cx, co):
            skel_scan(cx, co, kind, SUM)
        ctx.kind = kind
        return out

    @staticmethod
    def backward(ctx, g):
        g = _f32(g, "grad")
        dx = torch.empty_like(g)
        rev = {INCLUSIVE: REVERSE_INCLUSIVE, EXCLUSIVE: REVERSE_EXCLUSIVE,
               REVERSE_INCLUSIVE: INCLUSIVE, REVERSE_EXCLUSIVE: EXCLUSIVE}[ctx.kind]
        with _wrapped(g, dx) as (cg, cdx):
            skel_scan(cg, cdx, rev, SUM)
        return dx, None


def scan_sum_fn(x, kind: int = INCLUSIVE):
    """Prefix (or suffix) sums of a flat float32 tensor, differentiable."""
    return _ScanSumFn.apply(_f32(x, "x").reshape(-1), int(kind))


_REVERSE = {INCLUSIVE: REVERSE_INCLUSIVE, EXCLUSIVE: REVERSE_EXCLUSIVE,
            REVERSE_INCLUSIVE: INCLUSIVE, REVERSE_EXCLUSIVE: EXCLUSIVE}


class _ScanRowsSumFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, kind):
        out = torch.empty_like(x)
        with _wrapped(x, out) as (cx, co):
            skel_scan_rows(cx, co, kind, SUM)
        ctx.kind = kind
        return out

    @staticmethod
    def backward(ctx, g):
        g = _f32(g, "grad")
        dx = torch.empty_like(g)
        with _wrapped(g, dx) as (cg, cdx):
            skel_scan_rows(cg, cdx, _REVERSE[ctx.kind], SUM)
        return dx, None


def scan_rows_sum_fn(x, kind: int = INCLUSIVE):
    """Prefix (or suffix) sums along the last axis of a float32 tensor,
    differentiable; leading axes are rows."""
    x = _f32(x, "x")
    if x.dim() < 2:
        raise ValueError("x needs at least 2 dimensions")
    shape = x.shape
    return _ScanRowsSumFn.apply(x.reshape(-1, shape[-1]), int(kind)).reshape(shape)


__all__ = ["map_fn", "reduce_sum_fn", "mapreduce_sum_fn", "mapoverlap1d_fn",
           "mapoverlap2d_fn", "mapoverlap2d_fields_fn", "map_overlap2d_reduce_fn", "scan_sum_fn",
           "scan_rows_sum_fn"]
