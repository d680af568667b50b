"""Pins of the oracle's warm start for streams (keep the previous frame's
pixel labels, bin the new frame, recount, then I pixel sweeps; the paper
names video as an input the framework adapts to, Sec. 7, and its refinement
can stop and resume at any time, Sec. 5.4)."""
import numpy as np
import pytest

import oracle
from _defs import colour_histograms, energy, valid_partition
from paper_1309_3848_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore")


def _scene(H=96, W=128, frames=6):
    return synth.StreamScene(H=H, W=W, regions=20, frames=frames, seed=11, noise_seed=1100)


def test_warm_start_on_the_same_frame_equals_a_second_run():
    sc = _scene()
    f0 = sc.frame(0)
    a = oracle.Oracle(f0, 24, 3, 5, 3, 1, 0)
    b = oracle.Oracle(f0, 24, 3, 5, 3, 1, 0)
    a.run(-1)
    b.run(-1)
    a.warm_start(f0)
    assert a.run(-1) == 27
    assert b.run(-1) == 27
    assert np.array_equal(a.labels(), b.labels())
    assert np.array_equal(a.histograms()[0], b.histograms()[0])


def test_warm_start_keeps_labels_and_recounts_from_the_new_frame():
    sc = _scene()
    o = oracle.Oracle(sc.frame(0), 24, 3, 5, 3, 1, 0)
    o.run(-1)
    lab = o.labels()
    f1 = sc.frame(1)
    o.warm_start(f1)
    assert np.array_equal(o.labels(), lab)
    fresh = oracle.Oracle(f1, 24, 3, 5, 3, 1, 0)  # bins of the new frame
    assert np.array_equal(o.bins(), fresh.bins())
    hist, size = o.histograms()
    assert np.array_equal(hist, colour_histograms(lab, fresh.bins(), o.K, 125))
    assert np.array_equal(size, np.bincount(lab.ravel(), minlength=o.K))
    assert o.level == 0


def test_warm_start_needs_pixel_level():
    sc = _scene()
    o = oracle.Oracle(sc.frame(0), 24, 3, 5, 3, 1, 0)
    with pytest.raises(ValueError):
        o.warm_start(sc.frame(1))          # still at the top block level
    o.run(5)
    with pytest.raises(ValueError):
        o.warm_start(sc.frame(1))          # stopped inside the block levels


def test_stream_sweeps_never_lower_the_energy_and_keep_superpixels_connected():
    sc = _scene(frames=5)
    o = oracle.Oracle(sc.frame(0), 24, 3, 5, 2, 1, 0)
    o.run(-1)
    for f in range(1, 5):
        o.warm_start(sc.frame(f))
        bins = o.bins()
        prev = energy(o.labels(), bins, o.K, 125, 1)
        for _ in range(2 * 9):             # I = 2 pixel sweeps of nine phases
            assert o.run(1) == 1
            e = energy(o.labels(), bins, o.K, 125, 1)
            assert e >= prev, f"frame {f}: energy fell"
            prev = e
        lab = o.labels()
        assert valid_partition(lab, o.K)
        hist, size = o.histograms()
        assert np.array_equal(hist, colour_histograms(lab, bins, o.K, 125))


def test_a_stream_of_frames_reaches_a_fixed_number_of_phases():
    sc = _scene(frames=3)
    o = oracle.Oracle(sc.frame(0), 24, 3, 5, 2, 1, 0)
    assert o.run(-1) == 3 * 2 * 9
    for f in (1, 2):
        o.warm_start(sc.frame(f))
        assert o.run(-1) == 2 * 9
