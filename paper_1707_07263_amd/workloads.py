"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no Fourier arithmetic: it only draws random numbers, so both
the GPU path's tests and the FP64 oracle can be fed the same inputs.  Every
generator uses ``numpy.random.Generator(PCG64(seed))``, draws in FP64 in the
order documented on each function, and returns complex128 (callers cast with
round-to-nearest-even to the storage type they test).

The paper measures 1-D transforms of 16..65536 points and motivates the work
with remote-sensing (SAR) images (abstract; Sec. 3).  It ships no data, so:

* ``uniform_1d``   - the small 1-D case (1024 points, re/im ~ U[-1, 1]).
* ``normal_batch`` - batched 1-D signals, re/im ~ N(0, 1).
* ``speckle_image``- a 2-D image with SAR-like statistics: a smooth amplitude
                     field (a sum of Gaussian blobs) times unit-mean
                     exponential speckle, with uniform random phase.
* ``uneven_sizes`` / ``uneven_batch`` - many transforms with power-of-two
                     lengths whose exponents are uniform over a range (the
                     "few thousand to tens of thousands" SAR range of Sec. 3
                     falls inside 2^8..2^16).
* ``autograd_case``- signals plus a fixed real weight and sampled coordinates
                     for the differentiable transform.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_1d(n: int = 1024, batch: int = 1, seed: int = 0) -> np.ndarray:
    """re ~ U[-1, 1] of shape [batch, n], then im ~ U[-1, 1]."""
    g = rng(seed)
    re = g.uniform(-1.0, 1.0, size=(batch, n))
    im = g.uniform(-1.0, 1.0, size=(batch, n))
    return re + 1j * im


def normal_batch(n: int, batch: int, seed: int) -> np.ndarray:
    """re ~ N(0, 1) of shape [batch, n], then im ~ N(0, 1)."""
    g = rng(seed)
    re = g.standard_normal(size=(batch, n))
    im = g.standard_normal(size=(batch, n))
    return re + 1j * im


def speckle_image(rows: int = 4096, cols: int = 4096, seed: int = 2,
                  blobs: int = 8, sigma_min: float = 64.0,
                  sigma_max: float = 512.0) -> np.ndarray:
    """Complex image z = S * E * exp(i*phi).

    Draw order: ``blobs`` centres (cy, cx) ~ U[0, rows) x U[0, cols) (cy for
    all blobs, then cx); sigma = sigma_min * (sigma_max/sigma_min)^U[0,1]
    (log-uniform, isotropic); weights a ~ U[0.5, 1.5]; then speckle
    E ~ Exp(1) per pixel; then phase phi ~ U[0, 2*pi) per pixel.
    S = sum_g a_g exp(-r_g^2 / (2 sigma_g^2)) is non-periodic and normalised
    to mean 1.
    """
    g = rng(seed)
    cy = g.uniform(0.0, rows, size=blobs)
    cx = g.uniform(0.0, cols, size=blobs)
    sigma = sigma_min * (sigma_max / sigma_min) ** g.uniform(0.0, 1.0, size=blobs)
    weight = g.uniform(0.5, 1.5, size=blobs)
    yy = np.arange(rows, dtype=np.float64)[:, None]
    xx = np.arange(cols, dtype=np.float64)[None, :]
    field = np.zeros((rows, cols), dtype=np.float64)
    for b in range(blobs):
        # separable Gaussian: exp(-(dy^2 + dx^2)/(2 s^2)) = gy * gx
        gy = np.exp(-((yy - cy[b]) ** 2) / (2.0 * sigma[b] ** 2))
        gx = np.exp(-((xx - cx[b]) ** 2) / (2.0 * sigma[b] ** 2))
        field += weight[b] * (gy * gx)
    field /= field.mean()
    speckle = g.exponential(1.0, size=(rows, cols))
    phase = g.uniform(0.0, 2.0 * np.pi, size=(rows, cols))
    amp = field * speckle
    return amp * np.cos(phase) + 1j * (amp * np.sin(phase))


def uneven_sizes(count: int = 512, lo_exp: int = 8, hi_exp: int = 16,
                 seed: int = 3) -> np.ndarray:
    """Lengths 2^e with e uniform over {lo_exp..hi_exp} (both inclusive)."""
    g = rng(seed)
    exps = g.integers(lo_exp, hi_exp + 1, size=count)
    return (np.int64(1) << exps.astype(np.int64)).astype(np.int64)


def uneven_batch(count: int = 512, lo_exp: int = 8, hi_exp: int = 16,
                 seed: int = 3):
    """(sizes, packed): sizes as ``uneven_sizes``; then, for each transform in
    draw order, re ~ N(0,1) of its length followed by im ~ N(0,1); the
    transforms are packed back to back, unsorted."""
    g = rng(seed)
    exps = g.integers(lo_exp, hi_exp + 1, size=count)
    sizes = (np.int64(1) << exps.astype(np.int64)).astype(np.int64)
    parts = []
    for n in sizes:
        re = g.standard_normal(int(n))
        im = g.standard_normal(int(n))
        parts.append(re + 1j * im)
    return sizes, np.concatenate(parts)


def autograd_case(batch: int = 64, n: int = 65536, seed: int = 4,
                  probes: int = 32):
    """(x, weight, coords): x re then im ~ N(0,1) [batch, n]; weight ~ U[0,1]
    [batch, n] (real); ``probes`` distinct flat indices into x."""
    g = rng(seed)
    re = g.standard_normal(size=(batch, n))
    im = g.standard_normal(size=(batch, n))
    weight = g.uniform(0.0, 1.0, size=(batch, n))
    coords = g.choice(batch * n, size=probes, replace=False)
    return re + 1j * im, weight, np.sort(coords)
