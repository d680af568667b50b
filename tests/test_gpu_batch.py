"""GPU parity of batch contexts: every image of a batch must get exactly the
labels, colour histograms and sizes that the CPU oracle computes for it on its
own (and that a single-image context computes), whatever the other images of
the batch are. Images differ in size, K and levels; the schedules are aligned
at their end."""
import os
import sys

import numpy as np
import pytest

import oracle
from _defs import valid_partition
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


# (H, W, regions, K, L) of a small mixed batch: several tiles, ragged edges,
# levels 1..4, one image much smaller than the rest
SMALL = [(97, 131, 12, 40, 3), (200, 160, 20, 60, 4), (64, 333, 9, 30, 2),
         (321, 481, 30, 200, 4), (33, 47, 4, 6, 1), (128, 128, 16, 64, 3)]


def _images(specs, seed0=100):
    return [synth.voronoi_image(H, W, R, 8.0, seed0 + i) for i, (H, W, R, _, _) in enumerate(specs)]


def _to_dev(imgs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(im)).cuda() for im in imgs]


def _read(S, ctx, i, H, W, B):
    import torch
    keff = S.seeds_batch_num_superpixels(ctx, i)
    lab = torch.empty((H, W), dtype=torch.int32, device="cuda")
    S.seeds_batch_labels(ctx, i, lab)
    hist = torch.empty((keff, B ** 3), dtype=torch.int32)
    size = torch.empty((keff,), dtype=torch.int32)
    S.seeds_batch_histograms(ctx, i, hist, size)
    return lab.cpu().numpy(), hist.numpy(), size.numpy()


def _batch_run(S, imgs, Ks, Ls, B, I, gamma, rule, mode=0, max_phases=-1, refines=1):
    dev = _to_dev(imgs)
    ctx = S.seeds_batch_init(dev, Ks, S.make_params(max(Ls), B, I, gamma, rule), levels=Ls)
    try:
        S.seeds_set_launch_mode(ctx, mode)
        assert S.seeds_batch_count(ctx) == len(imgs)
        for _ in range(refines):
            if max_phases < 0:
                S.seeds_refine(ctx)
            else:
                S.seeds_refine_phases(ctx, max_phases)
        out = [_read(S, ctx, i, im.shape[0], im.shape[1], B) for i, im in enumerate(imgs)]
        S.seeds_sync(ctx)
        return out
    finally:
        S.seeds_destroy(ctx)


def _own_phases(P, L, Lmax, I):
    """Phases image i has taken after P phases of the batch (schedules aligned
    at their end: the batch's levels above L-1 come first)."""
    if P < 0:
        return -1
    return max(0, P - (Lmax - L) * 9 * I)


def _check_image(got, img, K, L, B, I, gamma, rule, max_phases=-1, what=""):
    lab, hist, size = got
    ref_lab, ref_hist, ref_size = oracle.seeds(img, K, L, B, I, gamma, rule, max_phases)
    bad = np.argwhere(lab != ref_lab)
    assert bad.size == 0, f"{what}: {len(bad)} labels differ, first at {bad[:5].tolist()}"
    assert np.array_equal(size, ref_size), what
    assert np.array_equal(hist, ref_hist), what
    assert valid_partition(lab, len(ref_size)), what


@pytest.mark.parametrize("rule", [0, 1])
@pytest.mark.parametrize("mode", [0, 1])
def test_small_batch_matches_oracle(S, rule, mode):
    _say(f"small batch rule={rule} mode={mode}")
    imgs = _images(SMALL)
    Ks = [s[3] for s in SMALL]
    Ls = [s[4] for s in SMALL]
    got = _batch_run(S, imgs, Ks, Ls, 5, 3, 1, rule, mode)
    for i, im in enumerate(imgs):
        _check_image(got[i], im, Ks[i], Ls[i], 5, 3, 1, rule, what=f"image {i}")


@pytest.mark.parametrize("P", [0, 1, 9, 26, 27, 28, 40, 55, 80, 107, 200])
def test_partial_schedules_match_oracle(S, P):
    # Lmax = 4, I = 3: 27 phases per level; image i starts after (4 - L_i) levels
    _say(f"batch partial P={P}")
    imgs = _images(SMALL)
    Ks = [s[3] for s in SMALL]
    Ls = [s[4] for s in SMALL]
    got = _batch_run(S, imgs, Ks, Ls, 4, 3, 2, 0, 1, max_phases=P)
    for i, im in enumerate(imgs):
        own = _own_phases(P, Ls[i], max(Ls), 3)
        ref_lab, ref_hist, ref_size = oracle.seeds(im, Ks[i], Ls[i], 4, 3, 2, 0, own)
        assert np.array_equal(got[i][0], ref_lab), f"image {i} after {own} own phases"
        assert np.array_equal(got[i][1], ref_hist), f"image {i}"
        assert np.array_equal(got[i][2], ref_size), f"image {i}"


def test_second_refine_runs_more_pixel_sweeps(S):
    _say("batch second refine")
    imgs = _images(SMALL[:4])
    Ks = [s[3] for s in SMALL[:4]]
    Ls = [s[4] for s in SMALL[:4]]
    got = _batch_run(S, imgs, Ks, Ls, 5, 2, 1, 0, 0, refines=2)
    for i, im in enumerate(imgs):
        o = oracle.Oracle(im, Ks[i], Ls[i], 5, 2, 1, 0)
        o.run(-1)
        o.run(-1)
        assert np.array_equal(got[i][0], o.labels()), f"image {i}"
        assert np.array_equal(got[i][1], o.histograms()[0]), f"image {i}"


def test_reinit_with_new_images(S):
    import torch
    _say("batch reinit")
    specs = SMALL[:3]
    A, Bimgs = _images(specs, 200), _images(specs, 300)
    Ks = [s[3] for s in specs]
    Ls = [s[4] for s in specs]
    dA, dB = _to_dev(A), _to_dev(Bimgs)
    ctx = S.seeds_batch_init(dA, Ks, S.make_params(4, 5, 2, 1, 0), levels=Ls)
    try:
        for imgs, dev in ((A, dA), (Bimgs, dB), (A, dA), (A, dA)):
            S.seeds_batch_reinit(ctx, dev)
            S.seeds_refine(ctx)
            for i, im in enumerate(imgs):
                got = _read(S, ctx, i, im.shape[0], im.shape[1], 5)
                _check_image(got, im, Ks[i], Ls[i], 5, 2, 1, 0, what=f"image {i}")
        torch.cuda.synchronize()
    finally:
        S.seeds_destroy(ctx)


def test_tiny_images_with_empty_classes(S):
    # 8 x 8 at 4 levels has a single top block: eight of nine classes are
    # empty at the top level (in both images, so some phases launch nothing)
    _say("batch tiny")
    imgs = [synth.voronoi_image(8, 8, 2, 8.0, 7), synth.voronoi_image(9, 20, 3, 8.0, 8)]
    Ks, Ls = [1, 2], [4, 3]
    for mode in (0, 1):
        got = _batch_run(S, imgs, Ks, Ls, 3, 2, 1, 0, mode)
        for i, im in enumerate(imgs):
            _check_image(got[i], im, Ks[i], Ls[i], 3, 2, 1, 0, what=f"image {i} mode {mode}")


def test_single_image_with_empty_classes(S):
    import torch
    _say("single tiny")
    img = synth.voronoi_image(8, 8, 2, 8.0, 7)
    for mode in (0, 1, 2):
        rgb = torch.from_numpy(img).cuda()
        ctx = S.seeds_init(rgb, 1, S.make_params(4, 3, 2, 1, 0))
        try:
            S.seeds_set_launch_mode(ctx, mode)
            S.seeds_refine(ctx)
            lab = torch.empty((8, 8), dtype=torch.int32)
            S.seeds_labels(ctx, lab)
        finally:
            S.seeds_destroy(ctx)
        ref, _, _ = oracle.seeds(img, 1, 4, 3, 2, 1, 0)
        assert np.array_equal(lab.numpy(), ref), f"mode {mode}"


def test_batch_of_one_equals_single_context(S):
    import torch
    _say("batch of one")
    img = synth.single_481x321()
    rgb = torch.from_numpy(img).cuda()
    got = _batch_run(S, [img], [200], [4], 5, 4, 1, 0)[0]
    ctx = S.seeds_init(rgb, 200, S.make_params(4, 5, 4, 1, 0))
    try:
        S.seeds_refine(ctx)
        lab = torch.empty(img.shape[:2], dtype=torch.int32)
        S.seeds_labels(ctx, lab)
    finally:
        S.seeds_destroy(ctx)
    assert np.array_equal(got[0], lab.numpy())


def test_persistent_mode_is_refused_on_a_batch(S):
    import torch
    _say("batch persistent refused")
    dev = _to_dev(_images(SMALL[:2]))
    ctx = S.seeds_batch_init(dev, [40, 60], S.make_params(4), levels=[3, 4])
    try:
        with pytest.raises(S.SeedsError) as e:
            S.seeds_set_launch_mode(ctx, S.SEEDS_LAUNCH_PERSISTENT)
        assert e.value.status == S.SEEDS_E_INVAL
        with pytest.raises(S.SeedsError):
            S.seeds_reinit(ctx, dev[0])
        with pytest.raises(S.SeedsError):
            S.seeds_batch_labels(ctx, 2, torch.empty((1,), dtype=torch.int32))
        # the context is still usable after argument errors
        S.seeds_refine(ctx)
        S.seeds_sync(ctx)
    finally:
        S.seeds_destroy(ctx)


def test_mixed_batch_of_64_equals_solo_runs_and_oracle_samples(S):
    """The mixed batch at its full sizes: every image equals its own
    single-image context bit for bit; three images (the smallest, the largest,
    one in between) are also checked against the oracle."""
    import torch
    specs = synth.batch_mixed(64)
    _say("mixed batch of 64")
    imgs = [synth.voronoi_image(s["H"], s["W"], s["regions"], s["sigma"], s["seed"]) for s in specs]
    Ks = [s["K"] for s in specs]
    Ls = [s["levels"] for s in specs]
    got = _batch_run(S, imgs, Ks, Ls, 5, 4, 1, 0, 0)
    for i, im in enumerate(imgs):
        rgb = torch.from_numpy(im).cuda()
        ctx = S.seeds_init(rgb, Ks[i], S.make_params(Ls[i], 5, 4, 1, 0))
        try:
            S.seeds_refine(ctx)
            lab = torch.empty(im.shape[:2], dtype=torch.int32, device="cuda")
            S.seeds_labels(ctx, lab)
            solo = lab.cpu().numpy()
        finally:
            S.seeds_destroy(ctx)
        assert np.array_equal(got[i][0], solo), f"image {i} ({specs[i]})"
    npx = [s["H"] * s["W"] for s in specs]
    order = np.argsort(npx)
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        _say(f"oracle sample image {i} {specs[i]}")
        _check_image(got[i], imgs[i], Ks[i], Ls[i], 5, 4, 1, 0, what=f"image {i}")


@pytest.mark.parametrize("P", [-1, 0, 40])
def test_labels_of_every_image_at_once(S, P):
    """seeds_batch_labels_all writes what seeds_batch_labels writes image by
    image, for images at pixel level (one widening launch) and at block levels
    (their own expansion), into outputs prefilled with a guard value."""
    import torch
    _say(f"batch labels of every image P={P}")
    imgs = _images(SMALL)
    Ks = [s[3] for s in SMALL]
    Ls = [s[4] for s in SMALL]
    ctx = S.seeds_batch_init(_to_dev(imgs), Ks, S.make_params(max(Ls), 5, 3, 1, 0), levels=Ls)
    try:
        if P < 0:
            S.seeds_refine(ctx)
        else:
            S.seeds_refine_phases(ctx, P)
        outs = [torch.full(im.shape[:2], -7, dtype=torch.int32, device="cuda") for im in imgs]
        S.seeds_batch_labels_all(ctx, outs)
        for i, im in enumerate(imgs):
            one = torch.empty(im.shape[:2], dtype=torch.int32, device="cuda")
            S.seeds_batch_labels(ctx, i, one)
            assert torch.equal(outs[i], one), f"image {i}"
        S.seeds_sync(ctx)
    finally:
        S.seeds_destroy(ctx)


def test_labels_of_more_images_than_one_launch_takes(S):
    """70 images: the 16-bit planes are widened 64 per launch, then 6."""
    import torch
    _say("batch labels of 70 images")
    specs = [(24 + (i % 7) * 5, 30 + (i % 5) * 9, 3, 4 + i % 3, 1 + i % 2) for i in range(70)]
    imgs = _images(specs, seed0=700)
    ctx = S.seeds_batch_init(_to_dev(imgs), [s[3] for s in specs],
                             S.make_params(2, 4, 2, 1, 0), levels=[s[4] for s in specs])
    try:
        S.seeds_refine(ctx)
        outs = [torch.full(im.shape[:2], -7, dtype=torch.int32, device="cuda") for im in imgs]
        S.seeds_batch_labels_all(ctx, outs)
        for i, im in enumerate(imgs):
            one = torch.empty(im.shape[:2], dtype=torch.int32, device="cuda")
            S.seeds_batch_labels(ctx, i, one)
            assert torch.equal(outs[i], one), f"image {i}"
            ref_lab, _, _ = oracle.seeds(im, specs[i][3], specs[i][4], 4, 2, 1, 0)
            assert np.array_equal(one.cpu().numpy(), ref_lab), f"image {i}"
        S.seeds_sync(ctx)
    finally:
        S.seeds_destroy(ctx)
