"""Pins of the oracle's quality metrics (Sec. 6.1: UE, CUE, BR, ASA), as
integer numerators: a hand-checked example, identities that follow from the
definitions, and brute force from the definitions on tiny random cases."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

HAND_S = np.array([[0, 0, 0, 1, 1, 1], [0, 0, 0, 1, 1, 1], [2, 2, 2, 2, 2, 2]])
HAND_G = np.array([[0, 0, 1, 1, 1, 1], [0, 0, 1, 1, 1, 1], [0, 0, 0, 0, 2, 2]])


def test_hand_example():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "quality_hand_values.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for r in rows:
        eps, N, ue, asa, cue, hits, total = map(int, r)
        q = oracle.quality(HAND_S, HAND_G, 3, 3, eps)
        assert q == dict(N=N, ue=ue, asa=asa, cue=cue, br_hits=hits, br_total=total)


def _boundary(seg):
    H, W = seg.shape
    b = np.zeros((H, W), bool)
    b[:, :-1] |= seg[:, :-1] != seg[:, 1:]
    b[:, 1:] |= seg[:, 1:] != seg[:, :-1]
    b[:-1, :] |= seg[:-1, :] != seg[1:, :]
    b[1:, :] |= seg[1:, :] != seg[:-1, :]
    return b


def _brute(s, g, K, R, eps):
    """Straight from the definitions, with Python sets and all-pairs distances."""
    H, W = s.shape
    S = [set(zip(*np.nonzero(s == k))) for k in range(K)]
    G = [set(zip(*np.nonzero(g == i))) for i in range(R)]
    ue = sum(len(S[k] - G[i]) for i in range(R) for k in range(K) if S[k] & G[i])
    asa = sum(max(len(S[k] & G[i]) for i in range(R)) for k in range(K))
    cue = 0
    for k in range(K):
        ov = [len(S[k] & G[i]) for i in range(R)]
        cue += len(S[k] - G[int(np.argmax(ov))])
    bg = np.argwhere(_boundary(g))
    bs = np.argwhere(_boundary(s))
    hits = 0
    for p in bg:
        if len(bs) and np.min(np.hypot(*(bs - p).T)) < eps:
            hits += 1
    return dict(N=H * W, ue=ue, asa=asa, cue=cue, br_hits=hits, br_total=len(bg))


@pytest.mark.parametrize("seed", range(30))
def test_brute_force_on_tiny_random_segmentations(seed):
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(1, 9)), int(rng.integers(1, 9))
    K, R = int(rng.integers(1, 6)), int(rng.integers(1, 5))
    s = rng.integers(0, K, size=(H, W))
    g = rng.integers(0, R, size=(H, W))
    if seed % 3 == 0:          # blocky segmentations too, not only salt and pepper
        s = np.repeat(np.repeat(rng.integers(0, K, size=(3, 3)), 3, 0), 3, 1)[:H, :W]
        g = np.repeat(np.repeat(rng.integers(0, R, size=(2, 2)), 5, 0), 5, 1)[:H, :W]
    for eps in (1, 2, 3):
        assert oracle.quality(s, g, K, R, eps) == _brute(s, g, K, R, eps), (seed, eps)


def test_identities():
    rng = np.random.default_rng(5)
    g = np.repeat(np.repeat(rng.integers(0, 6, size=(6, 8)), 7, 0), 7, 1)
    N = g.size
    # the segmentation equal to the ground truth
    q = oracle.quality(g, g, 6, 6)
    assert q["ue"] == 0 and q["cue"] == 0 and q["asa"] == N and q["br_hits"] == q["br_total"]
    # a single superpixel over everything
    present = np.unique(g)
    q = oracle.quality(np.zeros_like(g), g, 1, 6)
    assert q["ue"] == (len(present) - 1) * N
    assert q["asa"] == np.bincount(g.ravel()).max()
    assert q["br_hits"] == 0
    # CUE = N - ASA for any segmentation
    for seed in range(5):
        s = np.random.default_rng(seed).integers(0, 9, size=g.shape)
        q = oracle.quality(s, g, 9, 6)
        assert q["cue"] == N - q["asa"]


def test_out_of_range_values_are_refused():
    s = np.zeros((4, 4), np.int32)
    with pytest.raises(ValueError):
        oracle.quality(s + 3, s, 3, 1)
    with pytest.raises(ValueError):
        oracle.quality(s, s - 1, 1, 1)
