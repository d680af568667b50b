"""GPU energy hook (seeds_energy): H' = sum of squared histogram cells and
G' = sum over pixels of the squared label counts of their 3x3 patches (the
count forms of the colour and boundary terms of Sec. 4) must equal the
oracle's, exactly, at every level of the schedule (block levels read the
labels through the block grid), for both block rules and for an image of a
batch."""
import os
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1309_3848_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=True)
    from paper_1309_3848_amd import seeds
    seeds.lib()
    return seeds


@pytest.mark.parametrize("rule", [0, 1])
def test_energy_matches_oracle_along_the_schedule(S, rule):
    import torch
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(97, 131, 12, 8.0, seed=5)
    K, L, B, I, gamma = 40, 3, 5, 3, 1
    rgb = torch.from_numpy(img).cuda()
    for P in (0, 1, 9, 26, 27, 40, 54, 55, 70, 81):
        _say(f"energy rule={rule} after {P} phases")
        ctx = S.seeds_init(rgb, K, S.make_params(L, B, I, gamma, rule))
        try:
            S.seeds_refine_phases(ctx, P)
            got = S.seeds_energy(ctx)
        finally:
            S.seeds_destroy(ctx)
        o = oracle.Oracle(img, K, L, B, I, gamma, rule)
        assert o.run(P) == P
        assert got == o.energy(), f"after {P} phases"


def test_energy_equals_the_squared_histograms_and_rises(S):
    import torch
    from paper_1309_3848_amd import synth
    img = synth.single_481x321()
    rgb = torch.from_numpy(img).cuda()
    ctx = S.seeds_init(rgb, 200, S.make_params(3, 5, 4, 1, 1))
    try:
        h0, g0 = S.seeds_energy(ctx)
        S.seeds_refine_phases(ctx, 2 * 4 * 9)          # both block levels
        h1, g1 = S.seeds_energy(ctx)
        S.seeds_refine(ctx)                             # the pixel sweeps
        h2, g2 = S.seeds_energy(ctx)
        hist = torch.empty((S.seeds_num_superpixels(ctx), 125), dtype=torch.int32)
        S.seeds_histograms(ctx, hist, None)
    finally:
        S.seeds_destroy(ctx)
    assert h2 == int((hist.numpy().astype(np.int64) ** 2).sum())
    # hill climbing: under the exact rule block phases never lower H', and
    # pixel phases never lower H' + gamma G' (gamma = 1)
    assert h1 >= h0 and h2 + g2 >= h1 + g1
    assert (h1, g1) != (h0, g0) and (h2, g2) != (h1, g1)


def test_energy_of_batch_images(S):
    import torch
    from paper_1309_3848_amd import synth
    specs = [(97, 131, 12, 40, 3), (64, 333, 9, 30, 2), (33, 47, 4, 6, 1)]
    imgs = [synth.voronoi_image(H, W, R, 8.0, 300 + i) for i, (H, W, R, _, _) in enumerate(specs)]
    dev = [torch.from_numpy(im).cuda() for im in imgs]
    ctx = S.seeds_batch_init(dev, [s[3] for s in specs], S.make_params(3, 5, 2, 1, 0),
                             levels=[s[4] for s in specs])
    try:
        S.seeds_refine(ctx)
        got = [S.seeds_batch_energy(ctx, i) for i in range(len(specs))]
        with pytest.raises(S.SeedsError):
            S.seeds_batch_energy(ctx, len(specs))
    finally:
        S.seeds_destroy(ctx)
    for i, (im, s) in enumerate(zip(imgs, specs)):
        o = oracle.Oracle(im, s[3], s[4], 5, 2, 1, 0)
        o.run(-1)
        assert got[i] == o.energy(), f"image {i}"
