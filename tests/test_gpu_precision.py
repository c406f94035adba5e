"""Accuracy of the compensated Reduce / MapReduce variants (R4, MR4) against
exactly rounded sums from the oracle.

The plain variants keep one binary32 accumulator per lane; their error grows
with the conditioning sum|x| / |sum x|.  The compensated variants carry every
addition's rounding error exactly (TwoSum) and every product's (TwoProduct)
in a second binary32 word, so their error is that of a sum kept to about twice
the working precision:  |r - s| <= u |s| + O(depth^2 u^2) sum|x|, with u = 2^-24
and depth the longest chain of dependent additions (a few hundred at the
launch shapes used here).  The bar written below, u*2|s| + 2^-36 sum|x|, sits
between that worst case and the typical error; the plain variants are held to
the general floating-point reduction bar 1e-5 sum|x|.

The pairwise variants (R5, MR5) add every value along a balanced tree: each
lane's chunk as a tree, the chunk sums by a binary counter of partial sums,
then the cross-lane and cross-workgroup trees, at most 64 additions deep at
these sizes (about 54 at 2^28), so |r - s| <= 64 u sum|x| (recursive summation
bound of depth 64; one more u per product for the dot).  The sizes run up to
2^28, the precision workload itself.
"""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
R2, R4, R5 = 2, 4, 5
MR2, MR4, MR5 = 2, 4, 5
PAIR_DEPTH = 64


def comp_bar(exact, mag):
    return 2 * U * abs(exact) + 2.0 ** -36 * mag


def run_reduce(skel, arr, dtype, v):
    out = skel.Container.empty(skel.F32, 1)
    skel.skel_reduce(skel.SUM, skel.Container.from_numpy(arr, dtype), out, variant=v)
    return float(out.to_numpy()[0])


def run_dot(skel, a, b, dtype, v, mop=None):
    out = skel.Container.empty(skel.F32, 1)
    ins = [skel.Container.from_numpy(a, dtype)]
    if b is not None:
        ins.append(skel.Container.from_numpy(b, dtype))
    skel.skel_mapreduce(skel.MAP_MUL if mop is None else mop, None, ins, skel.SUM, out,
                        variant=v)
    return float(out.to_numpy()[0])


@pytest.mark.parametrize("n", [0, 1, 7, 4097, (1 << 20) + 3, 1 << 24, 1 << 26, 1 << 28])
def test_compensated_bf16_sum(skel, oracle_mod, n):
    print(f"bf16 sum n={n}", flush=True)
    xb = si.log_uniform_signed_bf16(n, config=4, index=11)
    xf = si.bf16_bits_to_f32(xb)
    exact = oracle_mod.sum_bf16_exact(xb)
    mag = oracle_mod.abs_sum(xf)
    del xf
    plain = run_reduce(skel, xb, skel.BF16, R2)
    comp = run_reduce(skel, xb, skel.BF16, R4)
    pair = run_reduce(skel, xb, skel.BF16, R5)
    ep, ec, ew = abs(plain - exact), abs(comp - exact), abs(pair - exact)
    print(f"bf16 sum n={n}: exact={exact:.9g} plain_err={ep:.3g} comp_err={ec:.3g} "
          f"pair_err={ew:.3g} sum|x|={mag:.3g}")
    assert ep <= 1e-5 * mag + 1e-30
    assert ec <= comp_bar(exact, mag) + 1e-30, (ec, exact, mag)
    assert ew <= PAIR_DEPTH * U * mag + 1e-30, (ew, exact, mag)


@pytest.mark.parametrize("n", [4097, (1 << 22) + 1, 1 << 26, 1 << 28])
def test_compensated_bf16_dot(skel, oracle_mod, n):
    print(f"bf16 dot n={n}", flush=True)
    xb = si.log_uniform_signed_bf16(n, config=4, index=12)
    yb = si.log_uniform_signed_bf16(n, config=4, index=13)
    exact = oracle_mod.dot_bf16_exact(xb, yb)
    xf, yf = si.bf16_bits_to_f32(xb), si.bf16_bits_to_f32(yb)
    # bf16 x bf16 products are exact in binary32 (8 + 8 significand bits), so
    # the binary64 sum of their absolute values in index order is sum|x y|
    # to within 2^-53 n
    mag = oracle_mod.abs_sum(xf * yf)
    del xf, yf
    plain = run_dot(skel, xb, yb, skel.BF16, MR2)
    comp = run_dot(skel, xb, yb, skel.BF16, MR4)
    pair = run_dot(skel, xb, yb, skel.BF16, MR5)
    ep, ec, ew = abs(plain - exact), abs(comp - exact), abs(pair - exact)
    print(f"bf16 dot n={n}: exact={exact:.9g} plain_err={ep:.3g} comp_err={ec:.3g} "
          f"pair_err={ew:.3g} sum|xy|={mag:.3g}")
    assert ep <= 1e-5 * mag + 1e-30
    assert ec <= comp_bar(exact, mag) + 1e-30, (ec, exact, mag)
    assert ew <= (PAIR_DEPTH + 1) * U * mag + 1e-30, (ew, exact, mag)


def test_compensated_f32_products(skel, oracle_mod):
    # binary32 products are exact in binary64 (24 + 24 <= 53 significand
    # bits), so fsum of the binary64 products is the exactly rounded dot
    n = (1 << 21) + 5
    x = si.normal_f32(n, 1, 21)
    y = si.normal_f32(n, 1, 22)
    prod = x.astype(np.float64) * y.astype(np.float64)
    exact, mag = oracle_mod.fsum(prod), oracle_mod.fsum(np.abs(prod))
    ec = abs(run_dot(skel, x, y, skel.F32, MR4) - exact)
    assert ec <= comp_bar(exact, mag), (ec, exact)
    sq = x.astype(np.float64) ** 2
    exact2 = oracle_mod.fsum(sq)
    ec2 = abs(run_dot(skel, x, None, skel.F32, MR4, skel.MAP_SQUARE) - exact2)
    assert ec2 <= comp_bar(exact2, exact2), (ec2, exact2)


def test_compensated_cancellation(skel, oracle_mod):
    # large terms that cancel in pairs around small ones: the exact sum is the
    # sum of the small terms, far below the rounding unit of the large ones
    n_big, n_small = 1 << 20, 1 << 16
    g = si.rng(5, 0)
    big = (g.standard_normal(n_big) * 1e6).astype(np.float32)
    small = (g.standard_normal(n_small) * 1e-3).astype(np.float32)
    x = np.concatenate([big, -big, small])
    x = x[g.permutation(x.size)]
    exact = oracle_mod.fsum(x.astype(np.float64))
    mag = oracle_mod.abs_sum(x)
    ep = abs(run_reduce(skel, x, skel.F32, R2) - exact)
    ec = abs(run_reduce(skel, x, skel.F32, R4) - exact)
    print(f"cancellation: exact={exact:.9g} plain_err={ep:.3g} comp_err={ec:.3g}")
    assert ec <= comp_bar(exact, mag)
    assert ec <= ep


def test_compensated_deterministic(skel):
    xb = si.log_uniform_signed_bf16((1 << 22) + 9, config=4, index=14)
    vals = {run_reduce(skel, xb, skel.BF16, R4) for _ in range(3)}
    assert len(vals) == 1
