"""Seeded synthetic RGB images and the paper's noise models.

This module holds no filter arithmetic: it only draws inputs. Both the GPU path
and the CPU oracle read the arrays it produces.

Clean image (a stand-in for the natural photographs of the paper's image set,
Section 4): a sum of 8 random linear colour gradients and 16 random Gaussian
colour blobs, mapped per channel onto [0.02, 0.98] of the channel range and
rounded, so that exact 0 and the channel maximum come only from the noise.

Noise models (Section 4, noise-model equation):
  * uncorrelated impulsive: each channel independently replaced with
    probability phi by r_k (salt-and-pepper r_k in {0, MAX}, or uniform);
  * correlated impulsive: with probability phi the pixel is corrupted; the
    default replaces all three channels with uniform values, the "paper"
    variant splits as in the equation (one channel with probability
    phi_k * phi each, all three with (1 - sum phi_k) * phi, phi_k = 0.25);
  * mixed: additive Gaussian noise first, then correlated impulses.
"""
from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np


def _rng(config: int, image: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([config, image, stream])


def clean_image(height: int, width: int, dtype=np.uint8, config: int = 0, image: int = 0,
                sigma_scale: Optional[float] = None) -> np.ndarray:
    """Smooth synthetic RGB image (seeded by (config, image))."""
    rng = _rng(config, image, 0)
    maxv = float(np.iinfo(dtype).max)
    size = float(max(height, width))
    if sigma_scale is None:
        sigma_scale = size / 256.0
    ys = np.arange(height, dtype=np.float64)
    xs = np.arange(width, dtype=np.float64)
    # 8 linear ramps: their sum is one plane per channel, a_k x + b_k y
    a = np.zeros(3)
    b = np.zeros(3)
    for _ in range(8):
        c = rng.uniform(-1.0, 1.0, 3)
        th = rng.uniform(0.0, 2.0 * math.pi)
        a += c * math.cos(th) / size
        b += c * math.sin(th) / size
    # 16 separable Gaussian blobs: sum_b amp_b gy_b(y) gx_b(x) as a product
    gy = np.empty((height, 16))
    gx = np.empty((width, 16))
    amp = np.empty((16, 3))
    for i in range(16):
        amp[i] = rng.uniform(-1.0, 1.0, 3)
        my = rng.uniform(0.0, height)
        mx = rng.uniform(0.0, width)
        sig = math.exp(rng.uniform(math.log(5.0), math.log(40.0))) * sigma_scale
        gy[:, i] = np.exp(-((ys - my) ** 2) / (2.0 * sig * sig))
        gx[:, i] = np.exp(-((xs - mx) ** 2) / (2.0 * sig * sig))
    lo, hi = 0.02 * maxv, 0.98 * maxv
    out = np.empty((height, width, 3), dtype=dtype)
    for k in range(3):
        ch = (gy * amp[:, k]) @ gx.T
        ch += xs[None, :] * a[k]
        ch += ys[:, None] * b[k]
        mn, mx_ = ch.min(), ch.max()
        span = mx_ - mn if mx_ > mn else 1.0
        ch -= mn
        ch *= (hi - lo) / span
        ch += lo
        out[:, :, k] = np.rint(ch)
    return out


def impulse_uncorrelated(img: np.ndarray, phi: float, rng: np.random.Generator,
                         salt_pepper: bool = True) -> np.ndarray:
    maxv = np.iinfo(img.dtype).max
    out = img.copy()
    hit = rng.random(img.shape) < phi
    if salt_pepper:
        vals = np.where(rng.random(img.shape) < 0.5, 0, maxv)
    else:
        vals = rng.integers(0, int(maxv) + 1, size=img.shape)
    out[hit] = vals[hit].astype(img.dtype)
    return out


def impulse_correlated(img: np.ndarray, phi: float, rng: np.random.Generator,
                       paper_split: bool = False, channel_phi: float = 0.25) -> np.ndarray:
    maxv = np.iinfo(img.dtype).max
    H, W, _ = img.shape
    out = img.copy()
    hit = rng.random((H, W)) < phi
    if not paper_split:
        out[hit] = rng.integers(0, int(maxv) + 1, size=(int(hit.sum()), 3)).astype(img.dtype)
        return out
    vals = rng.integers(0, int(maxv) + 1, size=img.shape).astype(img.dtype)
    which = rng.random((H, W))
    # channel k alone with probability channel_phi each, all three otherwise
    for k in range(3):
        sel = hit & (which >= k * channel_phi) & (which < (k + 1) * channel_phi)
        out[sel, k] = vals[sel, k]
    allsel = hit & (which >= 3 * channel_phi)
    out[allsel] = vals[allsel]
    return out


def gaussian(img: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    maxv = float(np.iinfo(img.dtype).max)
    noisy = img.astype(np.float64) + rng.normal(0.0, sigma, img.shape)
    return np.clip(np.rint(noisy), 0, maxv).astype(img.dtype)


# Workload recipes: image shape, dtype, noise. Indices follow the configuration
# list of the benchmark: 0 small anchor, 1 headline 4096^2, 2 mixed-noise
# 4096^2, 3 uneven batch, 4 16-bit 8192^2.

def workload_image(config: int, image: int = 0, height: Optional[int] = None,
                   width: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """(clean, noisy) image of a workload configuration; sizes may be overridden
    (same recipe, smaller image) for tests."""
    if config == 0:
        H, W, dt = 256, 256, np.uint8
    elif config in (1, 2):
        H, W, dt = 4096, 4096, np.uint8
    elif config == 3:
        H, W, dt = batch_shapes()[image] + (np.uint8,)
    elif config == 4:
        H, W, dt = 8192, 8192, np.uint16
    else:
        raise ValueError(config)
    H = height or H
    W = width or W
    clean = clean_image(H, W, dt, config, image)
    rng = _rng(config, image, 1)
    if config == 0:
        noisy = impulse_uncorrelated(clean, 0.10, rng, salt_pepper=True)
    elif config == 1:
        noisy = impulse_correlated(clean, 0.20, rng)
    elif config == 2:
        noisy = impulse_correlated(gaussian(clean, 10.0, rng), 0.10, rng)
    elif config == 3:
        noisy = impulse_correlated(clean, 0.15, rng)
    else:
        noisy = impulse_correlated(gaussian(clean, 400.0, rng), 0.25, rng)
    return clean, noisy


def batch_shapes(count: int = 256, seed: int = 3):
    """Image sizes of the uneven batch: area log-uniform in [320*240, 4000*3000],
    aspect ratio log-uniform in [1/2, 2]."""
    rng = np.random.default_rng([seed, 0, 2])
    lo, hi = math.log(320 * 240), math.log(4000 * 3000)
    shapes = []
    for _ in range(count):
        area = math.exp(rng.uniform(lo, hi))
        aspect = math.exp(rng.uniform(math.log(0.5), math.log(2.0)))
        w = max(1, int(round(math.sqrt(area * aspect))))
        h = max(1, int(round(area / w)))
        shapes.append((h, w))
    return shapes


def batch_assignments(count: int = 256, seed: int = 3):
    """Per image: (filter, window) drawn uniformly from the four filters and {3,5,7}."""
    rng = np.random.default_rng([seed, 0, 3])
    filters = ("vdf", "ddf", "amnfe", "evmf")
    return [(filters[int(rng.integers(0, 4))], (3, 5, 7)[int(rng.integers(0, 3))])
            for _ in range(count)]


NOISE_MODELS = ("uncorrelated", "correlated", "mixed")


def quality_set(model: str, phi: float = 0.10, count: int = 8, height: int = 512, width: int = 512,
                sigma: float = 10.0, seed: int = 5):
    """(clean, noisy) pairs for the exact-versus-approximate tables (Section 4,
    its three noise models at corruption probability phi): uncorrelated
    impulses (each channel replaced by a random value with probability phi),
    correlated impulses (a pixel hit with probability phi; channels 1, 2, 3
    alone with probability 0.25 each, all three otherwise), and mixed
    (Gaussian noise of standard deviation sigma, then correlated impulses)."""
    if model not in NOISE_MODELS:
        raise ValueError(model)
    out = []
    for i in range(count):
        clean = clean_image(height, width, np.uint8, 5, 1000 * seed + i)
        rng = _rng(5, 1000 * seed + i, 1 + NOISE_MODELS.index(model))
        if model == "uncorrelated":
            noisy = impulse_uncorrelated(clean, phi, rng, salt_pepper=False)
        elif model == "correlated":
            noisy = impulse_correlated(clean, phi, rng, paper_split=True)
        else:
            noisy = impulse_correlated(gaussian(clean, sigma, rng), phi, rng, paper_split=True)
        out.append((clean, noisy))
    return out
