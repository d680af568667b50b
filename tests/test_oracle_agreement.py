"""The Prop. 1 agreement measurement (oracle/agreement.py): its Prop. 1 test
must reproduce the oracle's own block decisions, and its exact energy tests
must match brute-force energies on small cases."""
import numpy as np
import pytest

from oracle import agreement as ag
from paper_1309_3848_amd import synth


def _H_norm(hists, sizes):
    from fractions import Fraction
    return sum(Fraction(int(np.dot(h, h)), int(a) ** 2) for h, a in zip(hists, sizes))


@pytest.mark.parametrize("seed", range(20))
def test_exact_tests_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    B3 = 8
    while True:   # redraw until k keeps pixels, the block has some and n exists
        hk = rng.integers(0, 6, B3)
        hn = rng.integers(0, 6, B3)
        hl = np.minimum(hk, rng.integers(0, 3, B3))
        if 0 < hl.sum() < hk.sum() and hn.sum() > 0:
            break
    ak, an, m = int(hk.sum()), int(hn.sum()), int(hl.sum())
    before = _H_norm([hk, hn], [ak, an])
    after = _H_norm([hk - hl, hn + hl], [ak - m, an + m])
    assert ag._exact_gain_positive(hk, hn, hl, ak, an, m) == (after > before)
    count_change = int(np.dot(hk - hl, hk - hl) + np.dot(hn + hl, hn + hl)
                       - np.dot(hk, hk) - np.dot(hn, hn))
    assert ag._count_gain_positive(hk, hn, hl) == (count_change > 0)


def _normalised_H_from_pixels(labels, bins):
    """H of eqs. eqColorSum, eqColorMain and eqColorHistogram written out over
    explicit pixel sets: for every superpixel, the set of its pixels, the
    share of them that falls in each colour bin, squared and summed."""
    from fractions import Fraction
    members = {}
    for y in range(labels.shape[0]):
        for x in range(labels.shape[1]):
            members.setdefault(int(labels[y, x]), []).append(int(bins[y, x]))
    total = Fraction(0)
    for pix in members.values():
        for j in set(pix):
            share = Fraction(pix.count(j), len(pix))
            total += share * share
    return total


@pytest.mark.parametrize("seed", range(30))
def test_exact_normalised_gain_against_pixel_sets(seed):
    """_exact_gain_positive against H recounted from the pixel sets of a small
    label map before and after moving one block (or pixel) from k to n.
    Every draw is used: the label map, the block and its target are chosen so
    that the block lies in k, k keeps pixels and n is another label."""
    rng = np.random.default_rng(100 + seed)
    Hh, Ww = int(rng.integers(4, 9)), int(rng.integers(4, 9))
    side = int(rng.choice([1, 2]))
    nb = int(rng.choice([2, 4, 8]))
    bins = rng.integers(0, nb, (Hh, Ww))
    labels = np.zeros((Hh, Ww), np.int64)
    labels[:, Ww // 2:] = 1                           # two superpixels side by side
    labels[: Hh // 2, Ww // 2:] = 2                   # and a third in one quadrant
    # the block: side x side at a random position inside label k's region
    while True:
        by = int(rng.integers(0, (Hh - side) // side + 1)) * side
        bx = int(rng.integers(0, (Ww - side) // side + 1)) * side
        blk = labels[by:by + side, bx:bx + side]
        k = int(blk[0, 0])
        if (blk == k).all() and (labels == k).sum() > blk.size:
            break
    n = int(rng.choice([l for l in (0, 1, 2) if l != k]))
    hist = lambda lab: np.array([np.bincount(bins[lab == l], minlength=nb) for l in (0, 1, 2)])
    h = hist(labels)
    sizes = [(labels == l).sum() for l in (0, 1, 2)]
    hl = np.bincount(bins[by:by + side, bx:bx + side].ravel(), minlength=nb)
    m = side * side
    moved = labels.copy()
    moved[by:by + side, bx:bx + side] = n
    # only k and n change; the other superpixel's share is the same on both sides
    want = _normalised_H_from_pixels(moved, bins) > _normalised_H_from_pixels(labels, bins)
    got = ag._exact_gain_positive(h[k], h[n], hl, int(sizes[k]), int(sizes[n]), m)
    assert got == want


def test_prop1_for_a_single_pixel_is_the_single_lookup():
    # one pixel of bin j: int(c_n, c_p) = h_n(j)/|A_n|, int(c_k\\p, c_p) = (h_k(j)-1)/(|A_k|-1)
    hk = np.array([5, 3, 2, 0], np.int64)
    hn = np.array([1, 4, 4, 1], np.int64)
    hl = np.array([0, 1, 0, 0], np.int64)
    # 4/10 vs 2/9: accept
    assert ag._prop1_accepts(hk, hn, hl, 10, 10, 1)
    hn2 = np.array([8, 1, 1, 0], np.int64)
    # 1/10 vs 2/9: reject
    assert not ag._prop1_accepts(hk, hn2, hl, 10, 10, 1)


def test_agreement_on_a_small_image_reproduces_the_oracle_decisions():
    img = synth.voronoi_image(97, 131, 12, 8.0, 3)
    r = ag.agreement(img, 40, 3, 5, 2, 1, 0)
    assert r["block_decisions_checked_against_oracle"] == r["block"]["total"] > 0
    assert r["pixel"]["total"] > 0
    for key in ("pixel", "block"):
        for rate in ("rate", "rate_count"):
            assert 0.0 < r[key][rate] <= 1.0
