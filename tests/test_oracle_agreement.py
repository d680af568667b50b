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
    hk = rng.integers(0, 6, B3)
    hn = rng.integers(0, 6, B3)
    hl = np.minimum(hk, rng.integers(0, 3, B3))
    if hl.sum() == 0 or hl.sum() == hk.sum() or hn.sum() == 0:
        pytest.skip("degenerate draw")
    ak, an, m = int(hk.sum()), int(hn.sum()), int(hl.sum())
    before = _H_norm([hk, hn], [ak, an])
    after = _H_norm([hk - hl, hn + hl], [ak - m, an + m])
    assert ag._exact_gain_positive(hk, hn, hl, ak, an, m) == (after > before)
    count_change = int(np.dot(hk - hl, hk - hl) + np.dot(hn + hl, hn + hl)
                       - np.dot(hk, hk) - np.dot(hn, hn))
    assert ag._count_gain_positive(hk, hn, hl) == (count_change > 0)


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
