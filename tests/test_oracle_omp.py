"""The all-core oracle build (OpenMP over the units of a phase) must give
exactly what the serial build gives: the decisions of a phase read only the
phase-start state, so deciding them in parallel changes nothing."""
import os

import numpy as np
import pytest

import oracle
from paper_1309_3848_amd import synth


@pytest.fixture(scope="module")
def omp():
    oracle.build(force=False)
    return oracle.lib_omp()


def test_omp_build_uses_several_threads(omp):
    assert oracle.lib().oracle_threads() == 1
    assert omp.oracle_threads() >= 1


@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("H,W,R,K,L,seed", [(161, 243, 20, 60, 3, 1), (97, 131, 12, 40, 4, 2),
                                             (60, 333, 9, 30, 2, 3)])
def test_all_core_build_equals_serial_build(omp, H, W, R, K, L, seed, rule):
    img = synth.voronoi_image(H, W, R, 8.0, seed)
    a = oracle.seeds(img, K, L, 5, 3, 1, rule)
    b = oracle.seeds(img, K, L, 5, 3, 1, rule, cdll=omp)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_decisions_of_every_phase_equal(omp):
    img = synth.voronoi_image(80, 100, 10, 8.0, 4)
    s = oracle.Oracle(img, 24, 3, 5, 2, 1, 1)
    p = oracle.Oracle(img, 24, 3, 5, 2, 1, 1, cdll=omp)
    while True:
        cs, cp = s.next_phase(), p.next_phase()
        assert cs == cp
        if cs < 0:
            break
        ds, dp = s.decide(cs), p.decide(cp)
        assert len(ds) == len(dp)
        for a, b in zip(ds, dp):
            assert bytes(a) == bytes(b)
        s.run(1)
        p.run(1)
    assert np.array_equal(s.labels(), p.labels())
