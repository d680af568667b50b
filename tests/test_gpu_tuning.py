"""Launch-mapping tuning never changes a result: every setting gives the
oracle's labels, and the autotuner leaves the context freshly initialised."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1309_3848_amd import synth

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


SETTINGS = [(1, 1), (0, 1), (1, 0), (0, 0)]


@pytest.mark.parametrize("setting", SETTINGS)
@pytest.mark.parametrize("rule", [0, 1])
def test_every_setting_matches_the_oracle(S, setting, rule):
    import torch
    _say(f"tuning {setting} rule {rule}")
    img = synth.single_481x321()
    ref, _, _ = oracle.seeds(img, 200, 3, 5, 4, 1, rule)
    ctx = S.seeds_init(torch.from_numpy(img).cuda(), 200, S.make_params(3, 5, 4, 1, rule))
    try:
        S.seeds_set_tuning(ctx, *setting)
        assert S.seeds_get_tuning(ctx) == {"pixel_compaction": setting[0], "xcd_remap": setting[1]}
        for mode in (0, 1):
            S.seeds_set_launch_mode(ctx, mode)
            S.seeds_reinit(ctx, torch.from_numpy(img).cuda())
            S.seeds_refine(ctx)
            lab = torch.empty(img.shape[:2], dtype=torch.int32)
            S.seeds_labels(ctx, lab)
            assert np.array_equal(lab.numpy(), ref), f"mode {mode}"
    finally:
        S.seeds_destroy(ctx)


def test_settings_on_a_batch(S):
    import torch
    _say("tuning batch")
    specs = [(97, 131, 12, 40, 3), (200, 160, 20, 60, 4), (33, 47, 4, 6, 1)]
    imgs = [synth.voronoi_image(H, W, R, 8.0, 40 + i) for i, (H, W, R, _, _) in enumerate(specs)]
    dev = [torch.from_numpy(im).cuda() for im in imgs]
    refs = [oracle.seeds(im, K, L, 5, 3, 1, 0)[0] for im, (_, _, _, K, L) in zip(imgs, specs)]
    ctx = S.seeds_batch_init(dev, [s[3] for s in specs], S.make_params(4, 5, 3, 1, 0),
                             levels=[s[4] for s in specs])
    try:
        for setting in SETTINGS:
            S.seeds_set_tuning(ctx, *setting)
            S.seeds_batch_reinit(ctx, dev)
            S.seeds_refine(ctx)
            for i, im in enumerate(imgs):
                lab = torch.empty(im.shape[:2], dtype=torch.int32)
                S.seeds_batch_labels(ctx, i, lab)
                assert np.array_equal(lab.numpy(), refs[i]), f"{setting} image {i}"
    finally:
        S.seeds_destroy(ctx)


def test_autotune_returns_a_fresh_context(S):
    import torch
    _say("autotune")
    img = synth.single_481x321()
    rgb = torch.from_numpy(img).cuda()
    ctx = S.seeds_init(rgb, 200, S.make_params(3, 5, 4, 1, 0))
    try:
        S.seeds_refine(ctx)                        # state that autotune must discard
        chosen, ms = S.seeds_autotune(ctx, reps=2)
        assert chosen in [{"pixel_compaction": a, "xcd_remap": b} for a, b in SETTINGS]
        assert all(m > 0 for m in ms)
        assert S.seeds_get_tuning(ctx) == chosen
        assert S.seeds_level(ctx) == 2             # back at the top level
        S.seeds_refine(ctx)
        lab = torch.empty(img.shape[:2], dtype=torch.int32)
        S.seeds_labels(ctx, lab)
        ref, _, _ = oracle.seeds(img, 200, 3, 5, 4, 1, 0)
        assert np.array_equal(lab.numpy(), ref)
        with pytest.raises(S.SeedsError):
            S.seeds_set_tuning(ctx, 2, 1)
        S.seeds_set_launch_mode(ctx, S.SEEDS_LAUNCH_PERSISTENT)
        with pytest.raises(S.SeedsError):
            S.seeds_autotune(ctx)
    finally:
        S.seeds_destroy(ctx)
