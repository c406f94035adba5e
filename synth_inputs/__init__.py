"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module draws random numbers and builds fixed weight vectors; it holds
none of the skeleton arithmetic.  Every array is reproducible from
(config, index): the generator is numpy's PCG64 seeded with
``BASE_SEED + 1000 * config + index``.

Workload shapes follow the skeleton workloads the build is measured on:
  * small plain skeletons on 2^20 elements (Map saxpy, Reduce, inclusive Scan,
    5-point MapOverlap 1D),
  * a 9x9 Gaussian MapOverlap 2D on a 4096x4096 image, a dot-product
    MapReduce over 2^26 elements and an exclusive widening Scan over 2^27.
The paper measures on no public dataset; these synthetic inputs stand in for
"problem sizes" in general.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 14052915


def rng(config: int, index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + 1000 * config + index))


def uniform_f32(n, a: float, b: float, config: int = 0, index: int = 0):
    """binary32 U[a, b): a + (b - a) * r with r on numpy's 2^-24 grid.
    For U[-1, 1) every value is 2r - 1, which is exact in binary32."""
    r = rng(config, index).random(n, dtype=np.float32)
    if a == -1.0 and b == 1.0:
        return (np.float32(2.0) * r - np.float32(1.0)).astype(np.float32)
    return (np.float32(a) + np.float32(b - a) * r).astype(np.float32)


def normal_f32(n, config: int = 0, index: int = 0):
    return rng(config, index).standard_normal(n, dtype=np.float32)


def int_uniform_i32(n, k: int, config: int = 0, index: int = 0):
    """int32 U{0..k}."""
    return rng(config, index).integers(0, k + 1, n, dtype=np.int32)


def int_uniform_i64(n, lo: int, hi: int, config: int = 0, index: int = 0):
    return rng(config, index).integers(lo, hi + 1, n, dtype=np.int64)


def binomial5_weights() -> np.ndarray:
    """[1, 4, 6, 4, 1] / 16: exact in binary32."""
    return (np.array([1, 4, 6, 4, 1], dtype=np.float64) / 16.0).astype(np.float32)


def gaussian_weights(radius: int = 4, sigma: float = 2.0) -> np.ndarray:
    """Point-sampled Gaussian exp(-k^2 / (2 sigma^2)), k = -radius..radius,
    normalised in binary64 and then rounded to binary32."""
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return (g / g.sum()).astype(np.float32)


def five_point_weights(center=0.5, north=0.125, south=0.125, west=0.125,
                       east=0.125) -> np.ndarray:
    """3x3 weight matrix of a 5-point stencil (row index = y offset -1..1)."""
    w = np.zeros((3, 3), dtype=np.float32)
    w[1, 1] = center
    w[0, 1] = north
    w[2, 1] = south
    w[1, 0] = west
    w[1, 2] = east
    return w


def log_uniform_lengths(count: int, lo: int, hi: int, config: int = 2,
                        index: int = 10) -> np.ndarray:
    """floor(exp(U[ln lo, ln hi])) as int64, used for batches of uneven
    vectors."""
    u = rng(config, index).random(count)
    return np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))
                    ).astype(np.int64)


def bf16_bits_from_f32(x: np.ndarray) -> np.ndarray:
    """Round binary32 to bfloat16 (nearest-even) and return the uint16 bit
    patterns.  Inputs are finite."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (b >> np.uint32(16)) & np.uint32(1)
    r = (b + np.uint32(0x7FFF) + lsb) >> np.uint32(16)
    return r.astype(np.uint16)


def bf16_bits_to_f32(h: np.ndarray) -> np.ndarray:
    return (np.ascontiguousarray(h, dtype=np.uint16).astype(np.uint32)
            << np.uint32(16)).view(np.float32)


def log_uniform_signed_bf16(n, lo: float = 1e-3, hi: float = 1e3,
                            config: int = 4, index: int = 0) -> np.ndarray:
    """|x| log-uniform in [lo, hi] with random signs, drawn in binary64,
    rounded to binary32 then to bfloat16.  Returns the bf16 bit patterns."""
    g = rng(config, index)
    mag = np.exp(math.log(lo) + g.random(n) * (math.log(hi) - math.log(lo)))
    sign = np.where(g.random(n) < 0.5, -1.0, 1.0)
    return bf16_bits_from_f32((sign * mag).astype(np.float32))
