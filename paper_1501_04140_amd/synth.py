"""Seeded synthetic grey-level images for the encoder's workloads.

This module only draws pixels. It holds none of the encoder's arithmetic, so
both the GPU library's tests and the CPU oracle's tests can take their inputs
from it.

The paper measures on Lena, Baboon and F16 (Section 4, Tables 1-2), which are
not available here. Seeded images with comparable structure stand in for them:

* ``gradients_blobs``: smooth gradients, Gaussian blobs and small integer noise
  (the single-level 128x128 workload).
* ``power_law``: 1/f^beta noise with random phase, optionally with hard-edged
  rectangles. ``beta`` is the exponent of the *power* spectrum, so the
  amplitude falls as |f|^(-beta/2).

Every generator uses ``numpy.random.default_rng`` (PCG64) in float64 and ends
with ``clip(rint(x), 0, 255).astype(uint8)``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gradients_blobs",
    "power_law",
    "single_level_image",
    "quadtree_image",
    "precision_image",
    "batch_images",
    "BATCH_SIDES",
    "learned_train_image",
    "learned_eval_image",
    "MLP_SHAPES",
    "mlp_init",
    "unit_rows_f16",
    "grad_like",
]

BATCH_SIDES = (256, 384, 512, 768, 1024, 2048)


def _to_u8(x: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def gradients_blobs(n: int = 128, seed: int = 0, n_grad: int = 6, n_blobs: int = 10,
                    noise: int = 8) -> np.ndarray:
    """Base 128 + ``n_grad`` linear ramps + ``n_blobs`` Gaussian blobs + integer noise."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    img = np.full((n, n), 128.0)
    c = n / 2.0
    for _ in range(n_grad):
        theta = rng.uniform(0.0, 2.0 * np.pi)
        a = rng.uniform(-60.0, 60.0)
        img += a * ((xx - c) * np.cos(theta) + (yy - c) * np.sin(theta)) / n
    for _ in range(n_blobs):
        amp = rng.uniform(-80.0, 80.0)
        cy, cx = rng.uniform(0.0, n, size=2)
        sigma = rng.uniform(4.0, 20.0)
        img += amp * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2.0 * sigma * sigma))
    img += rng.integers(-noise, noise + 1, size=(n, n))
    return _to_u8(img)


def power_law(h: int, w: int | None = None, beta: float = 2.0, seed: int | np.random.Generator = 0,
              n_rect: int = 0) -> np.ndarray:
    """1/f^beta noise (power spectrum ~ f^-beta, DC removed, random phase), rescaled to 0..255,
    then ``n_rect`` constant-grey rectangles painted in order."""
    w = h if w is None else w
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.fftfreq(w)[None, :]
    f = np.sqrt(fy * fy + fx * fx)
    amp = np.zeros_like(f)
    nz = f > 0
    amp[nz] = f[nz] ** (-beta / 2.0)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(h, w))
    field = np.real(np.fft.ifft2(amp * np.exp(1j * phase)))
    lo, hi = field.min(), field.max()
    img = (field - lo) * (255.0 / (hi - lo)) if hi > lo else np.zeros_like(field)
    for _ in range(n_rect):
        rh = int(rng.integers(h // 16, h // 4 + 1))
        rw = int(rng.integers(w // 16, w // 4 + 1))
        y0 = int(rng.integers(0, h - rh + 1))
        x0 = int(rng.integers(0, w - rw + 1))
        img[y0:y0 + rh, x0:x0 + rw] = float(rng.integers(0, 256))
    return _to_u8(img)


def single_level_image(seed: int = 0, n: int = 128) -> np.ndarray:
    """The plain single-level workload: 128x128 gradients + blobs + noise."""
    return gradients_blobs(n, seed)


def quadtree_image(seed: int = 0, n: int = 512) -> np.ndarray:
    """The quadtree workload: 512x512 1/f^2 noise with 3 hard-edged rectangles."""
    return power_law(n, n, beta=2.0, seed=seed, n_rect=3)


def precision_image(seed: int = 0, n: int = 1024) -> np.ndarray:
    """The precision workload: 1024x1024 1/f^1.8 noise."""
    return power_law(n, n, beta=1.8, seed=seed)


def batch_images(count: int = 64, master_seed: int = 0, sides=BATCH_SIDES):
    """``count`` images; image i draws its side from ``sides`` and beta from U[1.5, 2.5]
    with ``default_rng([master_seed, i])``."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([master_seed, i])
        side = int(sides[int(rng.integers(0, len(sides)))])
        beta = float(rng.uniform(1.5, 2.5))
        out.append(power_law(side, side, beta=beta, seed=rng))
    return out


def _beta_image(seed: int, n: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    beta = float(rng.uniform(1.5, 2.5))
    return power_law(n, n, beta=beta, seed=rng)


def learned_train_image(i: int, n: int = 512) -> np.ndarray:
    """Training image i (seed 1000 + i), beta ~ U[1.5, 2.5]."""
    return _beta_image(1000 + i, n)


def learned_eval_image(i: int, n: int = 2048) -> np.ndarray:
    """Evaluation image i (seed 2000 + i), beta ~ U[1.5, 2.5]."""
    return _beta_image(2000 + i, n)


# Parameter layout of the proposal network (64 -> 256 -> 256 -> 64): W of shape
# (out, in) then b, layer by layer, concatenated.
MLP_SHAPES = ((256, 64), (256,), (256, 256), (256,), (64, 256), (64,))


def mlp_init(seed: int = 0) -> np.ndarray:
    """Initial parameters (float32): He-uniform weights U(-sqrt(6/fan_in), +), zero biases,
    rounded to the nearest float16 so that every consumer starts from the same values."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            bound = np.sqrt(6.0 / shape[1])
            parts.append(rng.uniform(-bound, bound, size=shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float16).astype(np.float32)


def unit_rows_f16(n: int, seed: int = 0, dim: int = 64, n_dup: int = 0) -> np.ndarray:
    """n random unit rows rounded to float16; the last n_dup rows repeat earlier rows
    (exact ties)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, dim))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    x = x.astype(np.float16)
    if n_dup:
        src = rng.integers(0, max(n - n_dup, 1), size=n_dup)
        x[n - n_dup:] = x[src]
    return x


def grad_like(n: int, seed: int = 0, scale: float = 1e-2) -> np.ndarray:
    """Synthetic float32 gradient: normal values with a spread of magnitudes and some zeros."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(n) * scale * np.exp(rng.uniform(-4, 2, size=n))
    g[rng.random(n) < 0.05] = 0.0
    return g.astype(np.float32)
