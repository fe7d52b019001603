"""Seeded synthetic natural-image-like inputs (no wavelet arithmetic here).

The paper measures on images it does not specify, so every workload here uses
one seeded generator: a flat 8-bit grey level of 128, plus 16 isotropic
Gaussian blobs (amplitude uniform in [-64, 64), standard deviation 5-20 % of
the image width, centres uniform over the image), plus white Gaussian noise of
standard deviation 8, rounded half-to-even and clamped to [0, 255].

Draw order (fixed, so that a seed names one image): for each of the 16 blobs
cx, cy, amp, u (sigma = u * width); then the noise in raster order.  The image
is built in blocks of rows; blocking changes neither the draw order nor any
element's arithmetic.

This module is shared by the tests, the benchmark and the examples; both the
GPU path and the CPU oracle consume its arrays, and it holds none of the
transform's arithmetic.
"""
from __future__ import annotations

import numpy as np

N_BLOBS = 16
NOISE_SIGMA = 8.0
ROW_BLOCK = 1024


def image(w: int, h: int, seed: int, dtype=np.float32) -> np.ndarray:
    """An h x w image of the blob + noise family, as float32 or int32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    blobs = []
    for _ in range(N_BLOBS):
        cx = rng.uniform(0.0, w)
        cy = rng.uniform(0.0, h)
        amp = rng.uniform(-64.0, 64.0)
        u = rng.uniform(0.05, 0.20)
        blobs.append((cx, cy, amp, u * w))
    xs = np.arange(w, dtype=np.float64)
    gx = [np.exp(-((xs - cx) ** 2) / (2.0 * s * s)) for (cx, _, _, s) in blobs]
    out = np.empty((h, w), dtype=dtype)
    for r0 in range(0, h, ROW_BLOCK):
        r1 = min(h, r0 + ROW_BLOCK)
        ys = np.arange(r0, r1, dtype=np.float64)
        acc = np.full((r1 - r0, w), 128.0)
        for (cx, cy, amp, s), gxb in zip(blobs, gx):
            gy = amp * np.exp(-((ys - cy) ** 2) / (2.0 * s * s))
            acc += gy[:, None] * gxb[None, :]
        acc += rng.normal(0.0, NOISE_SIGMA, size=(r1 - r0, w))
        np.clip(np.rint(acc), 0.0, 255.0, out=acc)
        out[r0:r1] = acc.astype(dtype)
    return out


def ragged_sizes(n: int = 256, seed: int = 4, lo: int = 64, hi: int = 4096):
    """Widths then heights, each uniform on [lo, hi] (odd sizes included)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ws = rng.integers(lo, hi + 1, size=n)
    hs = rng.integers(lo, hi + 1, size=n)
    return [(int(a), int(b)) for a, b in zip(ws, hs)]


def ragged_images(n: int = 256, seed: int = 4, dtype=np.float32, lo: int = 64, hi: int = 4096):
    """The ragged batch: image i has the i-th size and seed 1000 * seed + i."""
    return [image(w, h, 1000 * seed + i, dtype) for i, (w, h) in
            enumerate(ragged_sizes(n, seed, lo, hi))]


def channel_batch(b: int, c: int, w: int, h: int, seed_base: int = 5000,
                  dtype=np.float32) -> np.ndarray:
    """A (b, c, h, w) batch; image (i, ch) has seed seed_base + c*i + ch."""
    out = np.empty((b, c, h, w), dtype=dtype)
    for i in range(b):
        for ch in range(c):
            out[i, ch] = image(w, h, seed_base + c * i + ch, dtype)
    return out


def image_device(w: int, h: int, seed: int, dtype=None, device="cuda"):
    """The same recipe built on the device (for large benchmark inputs): the
    blob parameters come from the same PCG64 draws as `image`, the noise from
    torch's device generator seeded with `seed`, so the pixels follow the same
    distribution but are not identical to `image(w, h, seed)`."""
    import torch

    dtype = torch.float32 if dtype is None else dtype
    rng = np.random.Generator(np.random.PCG64(seed))
    blobs = []
    for _ in range(N_BLOBS):
        cx = rng.uniform(0.0, w)
        cy = rng.uniform(0.0, h)
        amp = rng.uniform(-64.0, 64.0)
        u = rng.uniform(0.05, 0.20)
        blobs.append((cx, cy, amp, u * w))
    xs = torch.arange(w, dtype=torch.float64, device=device)
    ys = torch.arange(h, dtype=torch.float64, device=device)
    acc = torch.full((h, w), 128.0, dtype=torch.float64, device=device)
    for (cx, cy, amp, s) in blobs:
        gx = torch.exp(-((xs - cx) ** 2) / (2.0 * s * s))
        gy = amp * torch.exp(-((ys - cy) ** 2) / (2.0 * s * s))
        acc += gy[:, None] * gx[None, :]
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    acc += NOISE_SIGMA * torch.randn((h, w), generator=gen, dtype=torch.float64, device=device)
    return torch.clamp(torch.round(acc), 0.0, 255.0).to(dtype)
