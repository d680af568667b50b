"""Seeded synthetic RGB images that stand in for natural photographs.

This module holds input generation only - no superpixel arithmetic. Both the
HIP library's tests and the CPU oracle consume the bytes it produces.

Recipe (one image):
  * regions: ``R`` Voronoi sites drawn uniformly in [0,W) x [0,H); each pixel
    belongs to the site nearest (Euclidean) to its centre (x+0.5, y+0.5);
    each region gets a colour drawn uniformly from {0..255}^3;
  * gradient: a random direction theta and a linear ramp of 64 grey levels
    peak to peak (-32..+32 across the image along theta), added to all channels;
  * noise: i.i.d. N(0, sigma^2) per pixel and channel;
  * value = clip(rint(colour + ramp + noise), 0, 255) as uint8.
All draws come from numpy's PCG64 seeded with ``seed`` in a fixed order.
"""
from __future__ import annotations

import hashlib
import os

import numpy as np
from scipy.spatial import cKDTree


def _regions(H: int, W: int, sites: np.ndarray) -> np.ndarray:
    ys, xs = np.mgrid[0:H, 0:W]
    pts = np.stack([xs.ravel() + 0.5, ys.ravel() + 0.5], axis=1)
    # nearest-site queries are independent per point: threads change nothing
    _, idx = cKDTree(sites).query(pts, k=1, workers=min(8, os.cpu_count() or 1))
    return idx.reshape(H, W).astype(np.int32)


def _ramp(H: int, W: int, theta: float, x0: float = 0.0, Wfull: int | None = None) -> np.ndarray:
    Wfull = W if Wfull is None else Wfull
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    cx, cy = Wfull / 2.0, H / 2.0
    t = (xs + x0 + 0.5 - cx) * np.cos(theta) + (ys + 0.5 - cy) * np.sin(theta)
    corners = np.array([[0, 0], [Wfull, 0], [0, H], [Wfull, H]], np.float64)
    tmax = np.max(np.abs((corners[:, 0] - cx) * np.cos(theta) + (corners[:, 1] - cy) * np.sin(theta)))
    return 32.0 * t / max(tmax, 1e-9)


def voronoi_image(H: int, W: int, regions: int, sigma: float, seed: int,
                  return_regions: bool = False):
    """One H x W x 3 uint8 image (and optionally its H x W region map)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sites = rng.uniform(low=(0.0, 0.0), high=(float(W), float(H)), size=(regions, 2))
    colours = rng.integers(0, 256, size=(regions, 3)).astype(np.float64)
    theta = float(rng.uniform(0.0, 2.0 * np.pi))
    noise = rng.normal(0.0, sigma, size=(H, W, 3))
    reg = _regions(H, W, sites)
    img = colours[reg] + _ramp(H, W, theta)[:, :, None] + noise
    img = np.clip(np.rint(img), 0, 255).astype(np.uint8)
    return (img, reg) if return_regions else img


def sha256(img: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(img).tobytes()).hexdigest()


# Workloads ------------------------------------------------------------------

def single_481x321(seed: int = 1):
    """481 x 321 image, 30 regions, sigma 8 (the small single-image case)."""
    return voronoi_image(321, 481, 30, 8.0, seed)


def single_1080p(seed: int = 2):
    """1920 x 1080 image, 400 regions, sigma 8 (the large single-image case)."""
    return voronoi_image(1080, 1920, 400, 8.0, seed)


def batch_mixed(count: int = 64, seed: int = 3):
    """Mixed-size batch: W ~ U{320..1920}, H ~ U{240..1080}, R ~ U{50..600},
    sigma ~ U[4,16], K ~ U{200..2000} clamped to floor(N/256), L ~ U{3,4};
    image i is generated with seed 3000 + i. Returns a list of dicts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        W = int(rng.integers(320, 1921))
        H = int(rng.integers(240, 1081))
        R = int(rng.integers(50, 601))
        sigma = float(rng.uniform(4.0, 16.0))
        K = int(rng.integers(200, 2001))
        L = int(rng.integers(3, 5))
        K = max(1, min(K, (H * W) // 256))
        out.append(dict(H=H, W=W, regions=R, sigma=sigma, K=K, levels=L, seed=3000 + i))
    return out


class StreamScene:
    """Video stream: one Voronoi scene on a (W + 2*frames) x H canvas; frame f
    is the crop x in [2f, 2f + W) with fresh noise (seed noise_seed + f)."""

    def __init__(self, H: int = 2160, W: int = 3840, regions: int = 1500, frames: int = 300,
                 sigma: float = 8.0, seed: int = 4, noise_seed: int = 4000, shift: int = 2):
        self.H, self.W, self.frames, self.sigma = H, W, frames, sigma
        self.shift, self.noise_seed = shift, noise_seed
        Wc = W + shift * frames
        rng = np.random.Generator(np.random.PCG64(seed))
        sites = rng.uniform(low=(0.0, 0.0), high=(float(Wc), float(H)), size=(regions, 2))
        colours = rng.integers(0, 256, size=(regions, 3)).astype(np.float64)
        theta = float(rng.uniform(0.0, 2.0 * np.pi))
        self.regions = _regions(H, Wc, sites)
        self.base = colours[self.regions] + _ramp(H, Wc, theta)[:, :, None]

    def frame(self, f: int) -> np.ndarray:
        x0 = self.shift * f
        rng = np.random.Generator(np.random.PCG64(self.noise_seed + f))
        noise = rng.normal(0.0, self.sigma, size=(self.H, self.W, 3))
        img = self.base[:, x0:x0 + self.W] + noise
        return np.clip(np.rint(img), 0, 255).astype(np.uint8)
