"""Snapshots (seeds_snapshot / seeds_restore, Sec. 5.4: the refinement stops
and resumes at any phase) and the boundary-unit hook, through the C ABI.

A run stopped after n phases, saved to host memory and restored into a fresh
context must finish exactly as an uninterrupted run and as the CPU oracle:
labels, histograms and sizes bit for bit, for both block rules, batches and
second refinements. Boundary-unit counts must equal a count from the
definition on the labels the context returns."""
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


def _img(H, W, R, seed):
    from paper_1309_3848_amd import synth
    return synth.voronoi_image(H, W, R, 8.0, seed)


def _state(S, ctx, H, W, B, image=0):
    import torch
    keff = S.seeds_batch_num_superpixels(ctx, image)
    lab = torch.empty((H, W), dtype=torch.int32)
    S.seeds_batch_labels(ctx, image, lab)
    hist = torch.empty((keff, B ** 3), dtype=torch.int32)
    size = torch.empty((keff,), dtype=torch.int32)
    S.seeds_batch_histograms(ctx, image, hist, size)
    return lab.numpy(), hist.numpy(), size.numpy()


@pytest.mark.parametrize("rule", [0, 1], ids=["intersect", "exact"])
@pytest.mark.parametrize("stop", [0, 1, 10, 44, 80, 107])
def test_resumed_run_equals_uninterrupted_run_and_oracle(S, rule, stop):
    import torch
    H, W, K, L, B, I = 161, 243, 60, 3, 5, 4   # 108 phases
    img = _img(H, W, 20, 101)
    rgb = torch.from_numpy(img).cuda()
    params = S.make_params(L, B, I, 1, rule)
    _say("snapshot stop", stop, "rule", rule)
    a = S.seeds_init(rgb, K, params)
    S.seeds_refine_phases(a, stop)
    snap = S.seeds_snapshot(a)
    level_a = S.seeds_level(a)
    S.seeds_destroy(a)
    # restored into a context initialised from other pixels of the same size:
    # the snapshot brings the bins along
    other = torch.from_numpy(_img(H, W, 9, 202)).cuda()
    b = S.seeds_init(other, K, params)
    try:
        S.seeds_restore(b, snap)
        assert S.seeds_level(b) == level_a
        S.seeds_refine(b)
        got = _state(S, b, H, W, B)
    finally:
        S.seeds_destroy(b)
    c = S.seeds_init(rgb, K, params)
    try:
        S.seeds_refine(c)
        want = _state(S, c, H, W, B)
    finally:
        S.seeds_destroy(c)
    ref = oracle.seeds(img, K, L, B, I, 1, rule)
    for g, w, r in zip(got, want, ref):
        assert np.array_equal(g, w)
        assert np.array_equal(g, r)


def test_snapshot_of_a_stopped_state_matches_the_oracle_there(S):
    import torch
    H, W, K, L, B, I = 97, 131, 40, 3, 5, 2
    img = _img(H, W, 12, 7)
    rgb = torch.from_numpy(img).cuda()
    params = S.make_params(L, B, I, 1, 0)
    for stop in (5, 20, 33):
        _say("snapshot mid-state", stop)
        a = S.seeds_init(rgb, K, params)
        S.seeds_refine_phases(a, stop)
        b = S.seeds_init(rgb, K, params)
        S.seeds_restore(b, S.seeds_snapshot(a))
        got = _state(S, b, H, W, B)
        S.seeds_destroy(a)
        S.seeds_destroy(b)
        o = oracle.Oracle(img, K, L, B, I, 1, 0)
        o.run(stop)
        hist, size = o.histograms()
        assert np.array_equal(got[0], o.labels())
        assert np.array_equal(got[1], hist)
        assert np.array_equal(got[2], size)


@pytest.mark.parametrize("stop", [30, 72])
def test_resume_with_32_bit_pixel_labels(S, stop):
    """More than 65535 superpixels: pixel labels are stored in 32 bits; a run
    stopped at a block level (30) or at pixel level (72) resumes exactly."""
    import torch
    H, W, K, L, B, I = 600, 600, 70000, 2, 5, 4
    img = _img(H, W, 300, 303)
    rgb = torch.from_numpy(img).cuda()
    params = S.make_params(L, B, I, 1, 0)
    _say("snapshot 32-bit labels stop", stop)
    a = S.seeds_init(rgb, K, params)
    S.seeds_refine_phases(a, stop)
    b = S.seeds_init(rgb, K, params)
    S.seeds_restore(b, S.seeds_snapshot(a))
    S.seeds_refine(a)
    S.seeds_refine(b)
    for g, w in zip(_state(S, b, H, W, B), _state(S, a, H, W, B)):
        assert np.array_equal(g, w)
    S.seeds_destroy(a)
    S.seeds_destroy(b)


def test_second_refine_after_restore(S):
    import torch
    H, W, K, L, B, I = 120, 160, 50, 3, 5, 2
    img = _img(H, W, 14, 9)
    rgb = torch.from_numpy(img).cuda()
    params = S.make_params(L, B, I, 1, 0)
    a = S.seeds_init(rgb, K, params)
    S.seeds_refine(a)
    snap = S.seeds_snapshot(a)
    S.seeds_refine(a)   # I more pixel sweeps
    want = _state(S, a, H, W, B)
    S.seeds_destroy(a)
    b = S.seeds_init(rgb, K, params)
    S.seeds_restore(b, snap)
    S.seeds_refine(b)
    got = _state(S, b, H, W, B)
    S.seeds_destroy(b)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


@pytest.mark.parametrize("stop", [3, 50, 100])
def test_batch_resume(S, stop):
    import torch
    specs = [(90, 130, 30, 4, 201), (64, 64, 12, 2, 202), (120, 100, 40, 3, 203)]
    imgs = [_img(H, W, 10, sd) for H, W, _, _, sd in specs]
    rgbs = [torch.from_numpy(i).cuda() for i in imgs]
    Ks = [s[2] for s in specs]
    Ls = [s[3] for s in specs]
    params = S.make_params(4, 5, 3, 1, 0)
    _say("batch snapshot stop", stop)
    a = S.seeds_batch_init(rgbs, Ks, params, levels=Ls)
    S.seeds_refine_phases(a, stop)
    snap = S.seeds_snapshot(a)
    S.seeds_destroy(a)
    b = S.seeds_batch_init(rgbs, Ks, params, levels=Ls)
    S.seeds_restore(b, snap)
    S.seeds_refine(b)
    c = S.seeds_batch_init(rgbs, Ks, params, levels=Ls)
    S.seeds_refine(c)
    for i, (H, W, K, L, _) in enumerate(specs):
        got = _state(S, b, H, W, 5, i)
        want = _state(S, c, H, W, 5, i)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), i
        ref = oracle.seeds(imgs[i], K, L, 5, 3, 1, 0)
        assert np.array_equal(got[0], ref[0]), i
    S.seeds_destroy(b)
    S.seeds_destroy(c)


def test_restore_refuses_mismatched_snapshots(S):
    import torch
    rgb = torch.from_numpy(_img(64, 80, 8, 3)).cuda()
    a = S.seeds_init(rgb, 20, S.make_params(3, 5, 2, 1, 0))
    snap = S.seeds_snapshot(a)
    for K, L, B in ((30, 3, 5), (20, 2, 5), (20, 3, 4)):
        b = S.seeds_init(rgb, K, S.make_params(L, B, 2, 1, 0))
        with pytest.raises(S.SeedsError) as e:
            S.seeds_restore(b, snap)
        assert e.value.status == S.SEEDS_E_INVAL
        S.seeds_destroy(b)
    with pytest.raises(S.SeedsError):
        S.seeds_restore(a, b"\0" * len(snap))
    with pytest.raises(S.SeedsError):
        S.seeds_restore(a, snap[:-8])
    S.seeds_restore(a, snap)   # the context is still usable
    S.seeds_refine(a)
    S.seeds_sync(a)
    S.seeds_destroy(a)


def _boundary_from_labels(lab, s, cls):
    """Boundary units of class cls (-1: all) on the unit grid of side s, read
    from pixel labels (each unit's label is its top-left pixel's), and the
    pixels they cover."""
    H, W = lab.shape
    u = lab[::s, ::s]
    uh, uw = u.shape
    diff = np.zeros(u.shape, bool)
    diff[1:] |= u[1:] != u[:-1]
    diff[:-1] |= u[:-1] != u[1:]
    diff[:, 1:] |= u[:, 1:] != u[:, :-1]
    diff[:, :-1] |= u[:, :-1] != u[:, 1:]
    uy, ux = np.mgrid[0:uh, 0:uw]
    if cls >= 0:
        diff &= (3 * (uy % 3) + ux % 3) == cls
    cover = np.minimum(s, W - ux * s) * np.minimum(s, H - uy * s)
    return int(diff.sum()), int(cover[diff].sum())


def test_boundary_units_of_a_batch(S):
    import torch
    specs = [(90, 130, 30, 4, 211), (64, 64, 12, 2, 212)]
    rgbs = [torch.from_numpy(_img(H, W, 10, sd)).cuda() for H, W, _, _, sd in specs]
    ctx = S.seeds_batch_init(rgbs, [s[2] for s in specs], S.make_params(4, 5, 2, 1, 0),
                             levels=[s[3] for s in specs])
    try:
        S.seeds_refine_phases(ctx, 20)
        got = S.seeds_boundary_units(ctx, 3)
        for i, (H, W, _, L, _) in enumerate(specs):
            lab = torch.empty((H, W), dtype=torch.int32)
            S.seeds_batch_labels(ctx, i, lab)
            level = min(S.seeds_level(ctx), L - 1)
            assert got[i] == _boundary_from_labels(lab.numpy(), 1 << level, 3), i
        with pytest.raises(S.SeedsError):
            S.seeds_boundary_units(ctx, 0, S.seeds_level(ctx) + 1)
        with pytest.raises(S.SeedsError):
            S.seeds_boundary_units(ctx, 9)
    finally:
        S.seeds_destroy(ctx)


def test_boundary_units_match_the_definition(S):
    import torch
    H, W, K, L = 203, 317, 80, 4
    rgb = torch.from_numpy(_img(H, W, 25, 55)).cuda()
    ctx = S.seeds_init(rgb, K, S.make_params(L, 5, 2, 1, 0))
    try:
        for stop in (0, 7, 18, 30, 45, 54, 60, 72):
            if stop:
                S.seeds_refine_phases(ctx, stop - done)
            done = stop
            level = S.seeds_level(ctx)
            lab = torch.empty((H, W), dtype=torch.int32)
            S.seeds_labels(ctx, lab)
            for cls in (-1, 0, 4, 8):
                got = S.seeds_boundary_units(ctx, cls)[0]
                assert got == _boundary_from_labels(lab.numpy(), 1 << level, cls), (stop, cls)
                # finer grids, with the labels their units inherit
                for finer in range(level - 1, -1, -1):
                    got = S.seeds_boundary_units(ctx, cls, finer)[0]
                    want = _boundary_from_labels(lab.numpy(), 1 << finer, cls)
                    assert got == want, (stop, cls, finer)
    finally:
        S.seeds_destroy(ctx)
