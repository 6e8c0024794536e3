"""Seeded synthetic inputs and the named workload parameters.

This module holds no arithmetic of the method: it only names the parameters of
each workload (grid sizes, kernel, length scale, spacing, batch) and draws seeded
random arrays of a size the caller passes in. Both the library's tests/bench and
the FP64 oracle take their inputs from here, so the two sides see the same values.

Spacing convention: a workload's "length as a fraction of the domain" is taken
against the extent of the final grid, i.e. delta_L = 1 / n_L and
delta_0 = 2^L / n_L per axis.
"""

from __future__ import annotations

import math

import numpy as np

# Each entry: ndim, shape0, depth, delta0 (per axis), kernel, scale, length, batch,
# chart and its parameters. Level sizes follow from shape0 and depth.
WORKLOADS = {
    # 1-D Matern-3/2, length 0.2, level-0 12 px, 5 levels (final 260 px), FP64
    "icr1d_m32_12to260": dict(ndim=1, shape0=(12,), depth=5, delta0=(32.0 / 260.0,),
                              kernel="matern32", scale=1.0, length=0.2, batch=1,
                              chart="regular", precision="f64"),
    # 2-D squared exponential, length 0.05, 16^2 -> 1540^2 over 7 levels, batch 16
    "icr2d_se_16to1540_b16": dict(ndim=2, shape0=(16, 16), depth=7,
                                  delta0=(128.0 / 1540.0,) * 2, kernel="sqexp", scale=1.0,
                                  length=0.05, batch=16, chart="regular", precision="f32"),
    # 3-D Matern-5/2, length 0.1, 10^3 -> 388^3 over 6 levels, one sample
    "icr3d_m52_10to388": dict(ndim=3, shape0=(10, 10, 10), depth=6,
                              delta0=(64.0 / 388.0,) * 3, kernel="matern52", scale=1.0,
                              length=0.1, batch=1, chart="regular", precision="f32"),
    # 2-D log-radial chart, Matern-3/2 length 0.05 (physical units), 24^2 -> 1284^2
    "icr2d_chart_24to1284": dict(ndim=2, shape0=(24, 24), depth=6, delta0=(1.0 / 24.0,) * 2,
                                 kernel="matern32", scale=1.0, length=0.05, batch=1,
                                 chart="logradial2d",
                                 chart_params=(0.1, math.log(10.0), 0.5 * math.pi),
                                 precision="f32"),
    # 3-D log-radial cylinder chart (radius 0.1 -> 1 over the level-0 box, a quarter
    # turn, height 1), Matern-3/2 length 0.05 (physical units), 10^3 -> 388^3
    "icr3d_chart_10to388": dict(ndim=3, shape0=(10, 10, 10), depth=6, delta0=(0.1,) * 3,
                                kernel="matern32", scale=1.0, length=0.05, batch=1,
                                chart="logradial_cyl3d",
                                chart_params=(0.1, math.log(10.0), 0.5 * math.pi, 1.0),
                                precision="f32"),
}


def standard_normal(n: int, seed: int, batch: int | None = None) -> np.ndarray:
    """FP64 N(0, 1) draws, shape (n,) or (batch, n), from numpy's PCG64 stream."""
    rng = np.random.default_rng(seed)
    shape = (n,) if batch is None else (batch, n)
    return rng.standard_normal(shape)


def standard_normal_f32(n: int, seed: int, batch: int | None = None) -> np.ndarray:
    """FP32 N(0, 1) draws for sizes where an FP64 intermediate would be wasteful."""
    rng = np.random.default_rng(seed)
    shape = (n,) if batch is None else (batch, n)
    return rng.standard_normal(shape, dtype=np.float32)


def bernoulli_mask(n: int, p_observed: float, seed: int) -> np.ndarray:
    """FP64 0/1 mask with P(1) = p_observed."""
    rng = np.random.default_rng(seed)
    return (rng.random(n) < p_observed).astype(np.float64)


def uniform(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, n)


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32/FP64 values to the nearest bfloat16 (ties to even), returned as FP32.

    Storage-format conversion only: used to hand both sides the same bf16 inputs.
    """
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)
