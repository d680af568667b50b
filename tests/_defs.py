"""Test-side definitions, written from the paper independently of the oracle.

These are used to pin the oracle: energies straight from their definitions
(eqs. eqColorSum/eqColorMain/eqColorHistogram and boundaryterm/eqBoundaryMain,
in counts), a global flood-fill connectivity check (Sec. 3), and random
connected partitions for brute-force checks.
"""
from __future__ import annotations

from collections import deque
from fractions import Fraction

import numpy as np


def colour_histograms(labels: np.ndarray, bins: np.ndarray, K: int, nbins: int) -> np.ndarray:
    h = np.zeros((K, nbins), np.int64)
    np.add.at(h, (labels.ravel(), bins.ravel().astype(np.int64)), 1)
    return h


def energy_H(labels, bins, K, nbins) -> int:
    """H' = sum_k sum_j h_k(j)^2 (histograms in pixel counts)."""
    h = colour_histograms(labels, bins, K, nbins)
    return int((h * h).sum())


def energy_G(labels: np.ndarray) -> int:
    """G' = sum_i sum_k b_i(k)^2 with b_i the label counts of the 3x3 patch
    around i clipped to the image. sum_k b(k)^2 counts ordered pairs of
    patch pixels that share a label, which is what is summed here."""
    H, W = labels.shape
    pad = np.pad(labels.astype(np.int64), 1, constant_values=-1)
    patch = np.stack([pad[dy:dy + H, dx:dx + W] for dy in range(3) for dx in range(3)], -1)
    same = (patch[..., :, None] == patch[..., None, :]) & (patch[..., :, None] >= 0)
    return int(same.sum())


def energy(labels, bins, K, nbins, gamma) -> int:
    return energy_H(labels, bins, K, nbins) + gamma * energy_G(labels)


def components(labels: np.ndarray):
    """Number of 4-connected components of every label (dict label -> count)."""
    H, W = labels.shape
    seen = np.zeros((H, W), bool)
    comps = {}
    for y in range(H):
        for x in range(W):
            if seen[y, x]:
                continue
            l = int(labels[y, x])
            comps[l] = comps.get(l, 0) + 1
            q = deque([(y, x)])
            seen[y, x] = True
            while q:
                cy, cx = q.popleft()
                for ny, nx in ((cy - 1, cx), (cy + 1, cx), (cy, cx - 1), (cy, cx + 1)):
                    if 0 <= ny < H and 0 <= nx < W and not seen[ny, nx] and labels[ny, nx] == l:
                        seen[ny, nx] = True
                        q.append((ny, nx))
    return comps


def valid_partition(labels: np.ndarray, K: int) -> bool:
    c = components(labels)
    return len(c) == K and all(v == 1 for v in c.values())


def random_partition(H: int, W: int, K: int, rng: np.random.Generator) -> np.ndarray:
    """K connected regions grown from random seeds in random frontier order."""
    lab = -np.ones((H, W), np.int64)
    seeds = rng.choice(H * W, K, replace=False)
    frontier = []
    for k, s in enumerate(seeds):
        lab[s // W, s % W] = k
        frontier.append((s // W, s % W))
    while frontier:
        i = int(rng.integers(len(frontier)))
        y, x = frontier[i]
        frontier[i] = frontier[-1]
        frontier.pop()
        for ny, nx in ((y - 1, x), (y + 1, x), (y, x - 1), (y, x + 1)):
            if 0 <= ny < H and 0 <= nx < W and lab[ny, nx] < 0:
                lab[ny, nx] = lab[y, x]
                frontier.append((ny, nx))
    return lab.astype(np.int32)


def upsample(unit_labels: np.ndarray, side: int, H: int, W: int) -> np.ndarray:
    """Pixel labels of a unit grid of the given side."""
    return np.repeat(np.repeat(unit_labels, side, 0), side, 1)[:H, :W]


def intersection(h_a: np.ndarray, A: int, h_l: np.ndarray, m: int) -> Fraction:
    """Normalised histogram intersection sum_j min(h_a(j)/A, h_l(j)/m)."""
    return sum((min(Fraction(int(a), A), Fraction(int(b), m)) for a, b in zip(h_a, h_l)),
               Fraction(0))
