"""The measurement hooks run and give plausible figures: the LDS-atomic rate
(the secondary roof), the latency floor of a phase launch (empty launches,
one round of window loads, two dependent rounds with atomics) and the traffic
probes (whose sums the library checks itself)."""
import sys

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1309_3848_amd import seeds
    seeds.lib()
    return seeds


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_lds_atomic_rate(S):
    _say("lds atomic rate")
    rate = S.seeds_lds_atomic_rate()
    # 256 CUs x 4 SIMDs at 2.4 GHz bound it far above this; a broken
    # measurement gives zero, NaN or absurd values
    assert 1.0 < rate < 10000.0


@pytest.mark.parametrize("groups,launches", [(900, 144), (81, 108), (1, 3)])
def test_launch_floor(S, groups, launches):
    _say(f"launch floor groups {groups} launches {launches}")
    empty, one, two = S.seeds_launch_floor(groups, launches)
    assert 0.0 < empty < 1000.0 and 0.0 < one < 1000.0 and 0.0 < two < 1000.0
    # over a long chain, two dependent rounds of loads cannot beat an empty
    # launch (over a few launches the graph's own start dominates)
    if launches >= 100:
        assert two > empty


@pytest.mark.parametrize("lines", [1 << 10, 1 << 19])
def test_traffic_probe(S, lines):
    _say(f"traffic probe lines {lines}")
    us = S.seeds_traffic_probe(lines)
    assert all(0.0 < t < 1e6 for t in us)
    if lines >= 1 << 19:
        # 64 MiB read at more than 8 TB/s would be faster than HBM allows
        # (the buffer was just written, but a 64 MiB read still cannot finish
        # in under 2 us)
        assert us[0] > 2.0
