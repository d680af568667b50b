"""The window-weight form of the boundary term (Prop. 2) that the pixel phase
evaluates, checked against the oracle's explicit patch counts (CPU only).

The pixel decision sums, over the 5x5 window around p, the weight of each cell
holding a label: the number of in-image 3x3 patches centred on p's in-image
3x3 neighbours that contain the cell, which per axis is
|([p-1, p+1] clipped to the image) n [q-1, q+1]| for cell coordinate q (0 if q
is outside). For a pixel 2 or more cells inside the image this is 3 - |q - p|
per axis and |K_p| = 9: the constant form the kernel takes when every deciding
pixel of a wavefront is such a pixel. Both forms, with the Prop. 1 colour part
and ties to the smaller label, must reproduce the oracle's best candidate and
gain for every boundary pixel whose removal keeps its superpixel connected."""
import numpy as np
import pytest

import oracle
from _defs import colour_histograms, random_partition


def _axis_weight(p, q, n):
    if not 0 <= q < n:
        return 0
    lo = max(max(p - 1, 0), q - 1)
    hi = min(min(p + 1, n - 1), q + 1)
    return max(hi - lo + 1, 0)


def _window_gain(lab, x, y, k, n, constant):
    H, W = lab.shape
    wk = wn = 0
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            yy, xx = y + dy, x + dx
            if constant:
                c = (3 - abs(dx)) * (3 - abs(dy))
            else:
                c = _axis_weight(x, xx, W) * _axis_weight(y, yy, H)
            if c == 0:
                continue
            lv = lab[yy, xx]
            wk += c * (lv == k)
            wn += c * (lv == n)
    if constant:
        kp = 9
    else:
        kp = (min(x + 1, W - 1) - max(x - 1, 0) + 1) * (min(y + 1, H - 1) - max(y - 1, 0) + 1)
    return wn + kp - wk


def _candidates(lab, x, y):
    H, W = lab.shape
    k = lab[y, x]
    c = set()
    for ny, nx in ((y - 1, x), (y, x + 1), (y + 1, x), (y, x - 1)):
        if 0 <= ny < H and 0 <= nx < W and lab[ny, nx] != k:
            c.add(int(lab[ny, nx]))
    return sorted(c)


@pytest.mark.parametrize("seed", range(24))
def test_window_weights_reproduce_the_oracle_decisions(seed):
    rng = np.random.default_rng(7000 + seed)
    H, W = int(rng.integers(6, 16)), int(rng.integers(6, 16))
    B = int(rng.integers(1, 4))
    gamma = int(rng.choice([1, 2, 7]))
    rgb = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    K = int(rng.integers(2, 8))
    o = oracle.Oracle(rgb, K=K, levels=1, bins=B, gamma=gamma)
    lab = random_partition(H, W, o.K, rng)
    o.set_pixel_labels(lab)
    bins = o.bins()
    hist = colour_histograms(lab, bins, o.K, o.nbins)
    checked = {True: 0, False: 0}
    for cls in range(9):
        for d in o.decide(cls):
            if not d.boundary or not d.connect_ok:
                continue
            x, y, k, j = d.ux, d.uy, int(d.k), int(bins[d.uy, d.ux])
            interior = 2 <= x < W - 2 and 2 <= y < H - 2
            forms = [False, True] if interior else [False]
            for constant in forms:
                best, bn = None, None
                for n in _candidates(lab, x, y):
                    g = int(hist[n, j]) - int(hist[k, j]) + 1 + gamma * _window_gain(lab, x, y, k, n, constant)
                    if best is None or g > best:
                        best, bn = g, n
                assert (bn, best) == (d.n, d.gain), (x, y, constant)
                checked[constant] += 1
    assert checked[False] > 0
