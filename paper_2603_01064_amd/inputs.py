"""Seeded synthetic inputs shared by the GPU path and the tests.

This module only draws random numbers and paints images; it holds none of the
solver's arithmetic (no operator, transfer or smoother).  Right-hand sides
``b = A u*`` are formed by whichever side consumes ``u*``.

All generators use ``numpy.random.default_rng(seed)`` (PCG64) and return
float64 NumPy arrays so both sides receive identical bits.
"""
from __future__ import annotations

import math

import numpy as np

ALPHA_CHOICES_2D = (1e-2, 1e-3, 1e-4)


def grid_nodes(n: int) -> np.ndarray:
    """Interior node coordinates ``(i+1)/(n+1)`` of a zero-boundary grid."""
    return (np.arange(n, dtype=np.float64) + 1.0) / (n + 1)


def sinusoids_and_steps_1d(n: int, seed: int, n_sin: int = 8, max_freq: int = 128,
                           n_steps: int = 3) -> np.ndarray:
    """1D true solution: sinusoids with N(0,1) amplitudes and integer
    frequencies uniform in 1..max_freq, plus a piecewise-constant term made of
    ``n_steps`` unit steps with N(0,1) heights at sorted U(0,1) positions."""
    rng = np.random.default_rng(seed)
    x = grid_nodes(n)
    a = rng.standard_normal(n_sin)
    f = rng.integers(1, max_freq + 1, size=n_sin)
    u = np.zeros(n)
    for aj, fj in zip(a, f):
        u += aj * np.sin(2.0 * math.pi * fj * x)
    c = rng.standard_normal(n_steps)
    t = np.sort(rng.uniform(0.0, 1.0, size=n_steps))
    for cm, tm in zip(c, t):
        u += cm * (x >= tm)
    return u


def boxes_image(n: int, seed: int, n_boxes: int = 20, noise_std: float = 0.1) -> np.ndarray:
    """2D true solution: ``n_boxes`` axis-aligned boxes painted in order (each
    overwrites what is under it) with values U(0,1), plus i.i.d. Gaussian noise
    of standard deviation ``noise_std`` (variance 0.01 by default)."""
    rng = np.random.default_rng(seed)
    u = np.zeros((n, n))
    for _ in range(n_boxes):
        r = np.sort(rng.integers(0, n, size=2))
        c = np.sort(rng.integers(0, n, size=2))
        v = rng.uniform(0.0, 1.0)
        u[r[0]:r[1] + 1, c[0]:c[1] + 1] = v
    return u + noise_std * rng.standard_normal((n, n))


def blobs_image(n: int, seed: int, n_blobs: int = 500, wmin: float = 2.0, wmax: float = 20.0) -> np.ndarray:
    """2D sum of Gaussian blobs ``a exp(-|p-c|^2/(2 w^2))`` with widths U(wmin,
    wmax) pixels, amplitudes N(0,1) and centres uniform over the image."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(wmin, wmax, size=n_blobs)
    a = rng.standard_normal(n_blobs)
    cy = rng.uniform(0.0, n - 1.0, size=n_blobs)
    cx = rng.uniform(0.0, n - 1.0, size=n_blobs)
    yy = np.arange(n, dtype=np.float64)
    out = np.zeros((n, n))
    for k in range(n_blobs):
        rad = int(math.ceil(6.0 * w[k]))
        y0, y1 = max(0, int(cy[k]) - rad), min(n, int(cy[k]) + rad + 2)
        x0, x1 = max(0, int(cx[k]) - rad), min(n, int(cx[k]) + rad + 2)
        gy = np.exp(-((yy[y0:y1] - cy[k]) ** 2) / (2.0 * w[k] ** 2))
        gx = np.exp(-((yy[x0:x1] - cx[k]) ** 2) / (2.0 * w[k] ** 2))
        out[y0:y1, x0:x1] += a[k] * gy[:, None] * gx[None, :]
    return out


def iid_normal(shape, seed: int) -> np.ndarray:
    """I.i.d. N(0,1) entries (training error vectors)."""
    return np.random.default_rng(seed).standard_normal(shape)


def alpha_mix(batch: int, seed: int, choices=ALPHA_CHOICES_2D) -> np.ndarray:
    """Per right-hand-side regularisation weights drawn uniformly from ``choices``."""
    rng = np.random.default_rng(seed)
    return np.asarray(choices, dtype=np.float64)[rng.integers(0, len(choices), size=batch)]


def he_normal_weights(channels, ksize: int, dim: int, seed: int):
    """Bias-free CNN weights, layer i of shape ``[C_{i+1}, C_i, k]`` (1D) or
    ``[C_{i+1}, C_i, k, k]`` (2D), He-normal with std ``sqrt(2/(C_i k^dim))``.
    Layer i of a level uses its own stream ``seed + i``."""
    out = []
    for i, (cin, cout) in enumerate(zip(channels[:-1], channels[1:])):
        rng = np.random.default_rng(seed + i)
        shape = (cout, cin) + (ksize,) * dim
        std = math.sqrt(2.0 / (cin * ksize ** dim))
        out.append(std * rng.standard_normal(shape))
    return out


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def log_uniform(lo: float, hi: float, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))


def fno_params(dim: int, width: int, layers: int, modes: int, ksize: int, seed: int) -> dict:
    """Seeded FNO parameters (float32-representable float64 arrays): lift and
    projection ~ N(0, 1) and N(0, 1/C), biases ~ N(0, 0.1^2), spectral
    weights (re, im) ~ N(0, 1/C^2), convolutions He-normal.  Shapes: R_re /
    R_im [2][C][C][k][k] (2D) or [C][C][k] (1D), W [C][C][ks](x[ks])."""
    rng = np.random.default_rng(seed)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    C = width
    rshape = (2, C, C, modes, modes) if dim == 2 else (C, C, modes)
    out = {"lift_w": f32(rng.standard_normal(C)), "lift_b": f32(0.1 * rng.standard_normal(C)), "layers": []}
    for _ in range(layers):
        out["layers"].append({
            "R_re": f32(rng.standard_normal(rshape) / C), "R_im": f32(rng.standard_normal(rshape) / C),
            "W": f32(math.sqrt(2.0 / (C * ksize ** dim)) * rng.standard_normal((C, C) + (ksize,) * dim)),
            "B": f32(0.1 * rng.standard_normal(C))})
    out["proj_w"] = f32(rng.standard_normal(C) / math.sqrt(C))
    out["proj_b"] = f32(0.1 * rng.standard_normal(()))
    return out
