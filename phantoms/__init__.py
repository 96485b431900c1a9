"""Seeded synthetic inputs: ellipse phantoms degraded by Gaussian then salt & pepper noise.

This module is shared by the tests, the benchmark and the oracle's callers. It holds
none of the de-noising arithmetic (no window statistics, no Wiener step); it only
draws images. The paper's own pipeline starts from a radiograph passed through an
undefined ``degradImage`` (Alg. 1, steps 1-3); the recipe here stands in for it:

* phantom: constant background (30), ten ellipses painted in order, later ones
  overwrite earlier ones; centre uniform in the image, semi-axes uniform in
  [0.05, 0.30] of (H, W), angle uniform in [0, pi), integer intensity uniform in
  ``intensity`` (inclusive).
* Gaussian noise first: ``g = clip(rint(x + N(0, sigma^2)), 0, M)`` (rint = round
  half to even), then salt & pepper: each pixel independently with probability
  ``d`` becomes 0 or M with probability 1/2 each.
* every slice draws from ``numpy.random.default_rng(SeedSequence(key))`` (PCG64),
  with ``key = [config_index, role, slice_index]`` so no two slices share a stream.

The five named workloads (``CONFIGS``) fix shapes, dtypes and noise levels for the
single-image, batched, surrogate and stress cases.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

ROLE_EVAL = 0
ROLE_TRAIN = 1


def _rng(key: Sequence[int]) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(list(int(k) for k in key)))


def ellipse_phantom(h: int, w: int, rng: np.random.Generator, intensity=(40, 220),
                    background: int = 30, n_ellipses: int = 10) -> np.ndarray:
    """Clean phantom as int32 (H, W): background plus ``n_ellipses`` filled ellipses."""
    img = np.full((h, w), background, dtype=np.int32)
    lo, hi = intensity
    for _ in range(n_ellipses):
        cy = rng.uniform(0, h)
        cx = rng.uniform(0, w)
        ay = rng.uniform(0.05, 0.30) * h
        ax = rng.uniform(0.05, 0.30) * w
        th = rng.uniform(0.0, np.pi)
        val = int(rng.integers(lo, hi + 1))
        # bounding box of the rotated ellipse
        ext = max(ay, ax)
        y0, y1 = max(0, int(np.floor(cy - ext))), min(h, int(np.ceil(cy + ext)) + 1)
        x0, x1 = max(0, int(np.floor(cx - ext))), min(w, int(np.ceil(cx + ext)) + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        dy = yy + 0.5 - cy
        dx = xx + 0.5 - cx
        c, s = np.cos(th), np.sin(th)
        u = dx * c + dy * s
        v = -dx * s + dy * c
        inside = (u / ax) ** 2 + (v / ay) ** 2 <= 1.0
        img[y0:y1, x0:x1][inside] = val
    return img


def degrade_image(clean: np.ndarray, sigma: float, density: float, max_value: int,
                  rng: np.random.Generator) -> np.ndarray:
    """Gaussian noise then salt & pepper, as int32 in [0, max_value]."""
    noisy = np.rint(clean.astype(np.float64) + rng.normal(0.0, sigma, clean.shape))
    noisy = np.clip(noisy, 0, max_value).astype(np.int32)
    if density > 0:
        hit = rng.random(clean.shape) < density
        salt = rng.random(clean.shape) < 0.5
        noisy[hit & salt] = max_value
        noisy[hit & ~salt] = 0
    return noisy


@dataclass
class Slice:
    clean: np.ndarray      # int32 (H, W)
    noisy: np.ndarray      # storage dtype (uint8 / uint16), (H, W)
    sigma: float
    density: float


@dataclass
class Workload:
    name: str
    dtype: str             # "u8" or "u16"
    max_value: int
    smax: int
    win: int
    shapes: List[Tuple[int, int]]
    sigma: Tuple[float, float]       # (lo, hi); equal for a fixed sigma
    density: Tuple[float, float]
    intensity: Tuple[int, int]
    config_index: int
    role: int = ROLE_EVAL
    note: str = ""

    @property
    def np_dtype(self):
        return np.uint8 if self.dtype == "u8" else np.uint16

    @property
    def n_pixels(self) -> int:
        return int(sum(h * w for h, w in self.shapes))

    def make_slice(self, i: int) -> Slice:
        h, w = self.shapes[i]
        rng = _rng([self.config_index, self.role, i])
        sigma = float(self.sigma[0]) if self.sigma[0] == self.sigma[1] else float(rng.uniform(*self.sigma))
        dens = float(self.density[0]) if self.density[0] == self.density[1] else float(rng.uniform(*self.density))
        clean = ellipse_phantom(h, w, rng, self.intensity)
        noisy = degrade_image(clean, sigma, dens, self.max_value, rng).astype(self.np_dtype)
        return Slice(clean=clean, noisy=noisy, sigma=sigma, density=dens)

    def slices(self, limit: Optional[int] = None) -> List[Slice]:
        n = len(self.shapes) if limit is None else min(limit, len(self.shapes))
        return [self.make_slice(i) for i in range(n)]


def _uneven_shapes() -> List[Tuple[int, int]]:
    return [(256, 256)] * 96 + [(512, 512)] * 112 + [(1024, 1024)] * 48


CONFIGS = {
    # single 512x512 u8 phantom, sigma 10, s&p 0.10, Smax 7, Wiener 3x3
    "c1": Workload("c1_512_u8_smax7_w3", "u8", 255, 7, 3, [(512, 512)], (10, 10), (0.10, 0.10),
                   (40, 220), 0),
    # single 1600x1600 u8 phantom (the paper's 2.5 MB image size), sigma 15, s&p 0.20, Smax 9, W 5x5
    "c2": Workload("c2_1600_u8_smax9_w5", "u8", 255, 9, 5, [(1600, 1600)], (15, 15), (0.20, 0.20),
                   (40, 220), 1),
    # 256 uneven 12-bit slices, sigma 40, s&p U[0.05, 0.30] per slice, Smax 11, W 5x5
    "c3": Workload("c3_256x_uneven_u16_smax11_w5", "u16", 4095, 11, 5, _uneven_shapes(), (40, 40),
                   (0.05, 0.30), (0, 4095), 2),
    # surrogate inference set: 64 x 1024^2 u8, sigma U[5,25], s&p U[0.05,0.30]; plain targets Smax 9, W 5
    "c4": Workload("c4_64x1024_u8_surrogate", "u8", 255, 9, 5, [(1024, 1024)] * 64, (5, 25),
                   (0.05, 0.30), (40, 220), 3),
    # stress: 16 x 4096^2 12-bit, sigma 60, s&p 0.50, Smax 15, W 7x7
    "c5": Workload("c5_16x4096_u16_smax15_w7", "u16", 4095, 15, 7, [(4096, 4096)] * 16, (60, 60),
                   (0.50, 0.50), (0, 4095), 4),
}


def training_set_like(wl: Workload, n: int, size: int) -> Workload:
    """Surrogate training images for workload `wl`: n x size^2 slices with its dtype, max
    value, noise ranges and intensities, drawn from the training role's seeds."""
    return Workload(f"{wl.name}_train_{n}x{size}", wl.dtype, wl.max_value, wl.smax, wl.win, [(size, size)] * n,
                    wl.sigma, wl.density, wl.intensity, wl.config_index, role=ROLE_TRAIN)


def surrogate_train_set(n: int = 2000, size: int = 256) -> Workload:
    """Training pairs for the surrogate: n x size^2 u8, sigma U[5,25], s&p U[0.05,0.30]."""
    return Workload(f"c4_train_{n}x{size}_u8", "u8", 255, 9, 5, [(size, size)] * n, (5, 25),
                    (0.05, 0.30), (40, 220), 3, role=ROLE_TRAIN)


def random_image(shape, max_value: int, seed: int, values: Optional[Sequence[int]] = None,
                 dtype=np.int32) -> np.ndarray:
    """Uniform random test image (values in [0, max_value] or drawn from ``values``)."""
    rng = _rng([1000, seed])
    if values is not None:
        v = np.asarray(values)
        return v[rng.integers(0, len(v), shape)].astype(dtype)
    return rng.integers(0, max_value + 1, shape).astype(dtype)


def noisy_phantom(h: int, w: int, max_value: int, sigma: float, density: float, seed: int,
                  dtype=np.int32) -> np.ndarray:
    """One degraded phantom of any size (test helper around the same recipe)."""
    rng = _rng([2000, seed])
    inten = (40, 220) if max_value <= 255 else (0, max_value)
    clean = ellipse_phantom(h, w, rng, inten)
    return degrade_image(clean, sigma, density, max_value, rng).astype(dtype)


def psnr(x: np.ndarray, ref: np.ndarray) -> float:
    """10*log10(1/MSE) for images already divided by their max value."""
    mse = float(np.mean((np.asarray(x, np.float64) - np.asarray(ref, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


# ---- surrogate network parameters ------------------------------------------------------
SURROGATE_CH = 32
SURROGATE_N_PARAMS = 2 * (9 * SURROGATE_CH + SURROGATE_CH) + 4 * (9 * SURROGATE_CH * SURROGATE_CH
                                                                    + SURROGATE_CH) - SURROGATE_CH + 1


def surrogate_params(seed: int, scale_last: float = 0.1) -> np.ndarray:
    """Seeded initial parameters of the 6-layer 3x3 conv surrogate, flat float32 in the
    order W1 (9,32), b1, W2..W5 (9,32,32) [tap, out, in] with their biases, W6 (9,32), b6:
    He-normal weights (fan-in 9 * C_in), zero biases, the last layer scaled by
    `scale_last` so that the untrained network starts near y = x."""
    rng = _rng([5000, seed])
    c = SURROGATE_CH
    parts = [rng.normal(0, np.sqrt(2.0 / 9), 9 * c), np.zeros(c)]
    for _ in range(4):
        parts += [rng.normal(0, np.sqrt(2.0 / (9 * c)), 9 * c * c), np.zeros(c)]
    parts += [rng.normal(0, scale_last * np.sqrt(1.0 / (9 * c)), 9 * c), np.zeros(1)]
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == SURROGATE_N_PARAMS
    return flat
