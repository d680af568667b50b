"""Launch-mapping tuning never changes a result: every setting gives the
oracle's labels, and the autotuner leaves the context freshly initialised."""
import functools
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


# (pixel_compaction, xcd_remap, items_per_group, init_rows, warm_rows,
# block_ppl): every mapping combination, each with one of the three tile
# heights, and every items_per_group with both block shapes
SETTINGS = [(c, r, it, (8, 16, 32)[(2 * c + r + it) % 3], (8, 16, 32)[(c + it) % 3],
             (1, 4)[(c + r) % 2])
            for c in (1, 0) for r in (1, 0) for it in (1, 2, 4)]
FIELDS = ("pixel_compaction", "xcd_remap", "items_per_group", "init_rows", "warm_rows",
          "block_ppl")


@functools.lru_cache(maxsize=None)
def _ref_481(rule):
    return oracle.seeds(synth.single_481x321(), 200, 3, 5, 4, 1, rule)[0]


@pytest.mark.parametrize("setting", SETTINGS)
@pytest.mark.parametrize("rule", [0, 1])
def test_every_setting_matches_the_oracle(S, setting, rule):
    import torch
    _say(f"tuning {setting} rule {rule}")
    img = synth.single_481x321()
    ref = _ref_481(rule)
    ctx = S.seeds_init(torch.from_numpy(img).cuda(), 200, S.make_params(3, 5, 4, 1, rule))
    try:
        S.seeds_set_tuning(ctx, *setting)
        assert S.seeds_get_tuning(ctx) == dict(zip(FIELDS, setting))
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
        assert chosen["pixel_compaction"] in (0, 1) and chosen["xcd_remap"] in (0, 1)
        assert chosen["items_per_group"] in (1, 2, 4) and chosen["init_rows"] in (8, 16, 32)
        assert chosen["warm_rows"] in (8, 16, 32) and chosen["block_ppl"] in (1, 4)
        assert len(ms) == S.SEEDS_TUNE_VARIANTS and all(m > 0 for m in ms)
        assert S.seeds_get_tuning(ctx) == chosen
        assert S.seeds_level(ctx) == 2             # back at the top level
        S.seeds_refine(ctx)
        lab = torch.empty(img.shape[:2], dtype=torch.int32)
        S.seeds_labels(ctx, lab)
        ref, _, _ = oracle.seeds(img, 200, 3, 5, 4, 1, 0)
        assert np.array_equal(lab.numpy(), ref)
        for bad in ((2, 1, 1, 16, 16, 1), (0, 1, 3, 16, 16, 1), (0, 1, 1, 12, 16, 1),
                    (0, 1, 1, 16, 7, 1), (0, 1, 1, 16, 16, 2)):
            with pytest.raises(S.SeedsError):
                S.seeds_set_tuning(ctx, *bad)
        S.seeds_set_launch_mode(ctx, S.SEEDS_LAUNCH_PERSISTENT)
        with pytest.raises(S.SeedsError):
            S.seeds_autotune(ctx)
    finally:
        S.seeds_destroy(ctx)


@pytest.mark.parametrize("rows", [8, 16, 32])
@pytest.mark.parametrize("items", [1, 4])
def test_warm_start_tiles(S, rows, items):
    """The warm start (re-bin and recount per frame) with every tile height,
    frame by frame against the oracle."""
    import torch
    _say(f"warm start rows {rows} items {items}")
    sc = synth.StreamScene(H=180, W=250, regions=40, frames=3)
    frames = [sc.frame(f) for f in range(3)]
    ctx = S.seeds_init(torch.from_numpy(frames[0]).cuda(), 120, S.make_params(3, 5, 2, 1, 0))
    o = oracle.Oracle(frames[0], 120, 3, 5, 2, 1, 0)
    try:
        S.seeds_set_tuning(ctx, 0, 1, items, 16, rows)
        S.seeds_reinit(ctx, torch.from_numpy(frames[0]).cuda())
        for f in range(3):
            if f:
                S.seeds_warm_start(ctx, torch.from_numpy(frames[f]).cuda())
                o.warm_start(frames[f])
            S.seeds_refine(ctx)
            o.run()
            lab = torch.empty((180, 250), dtype=torch.int32)
            S.seeds_labels(ctx, lab)
            assert np.array_equal(lab.numpy(), o.labels()), f"frame {f}"
            hist = torch.empty((S.seeds_num_superpixels(ctx), 125), dtype=torch.int32)
            S.seeds_histograms(ctx, hist, None)
            assert np.array_equal(hist.numpy(), o.histograms()[0]), f"frame {f}"
    finally:
        S.seeds_destroy(ctx)
