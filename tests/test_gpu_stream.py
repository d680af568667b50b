"""GPU parity of the stream warm start: frame 0 runs the whole hierarchy,
every later frame keeps the previous labels, is re-binned and recounted, and
gets I pixel sweeps. Labels, histograms and sizes must equal the CPU oracle's
after every frame, bit for bit."""
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


def _read(S, ctx, H, W, B, image=None):
    import torch
    k = S.seeds_num_superpixels(ctx) if image is None else S.seeds_batch_num_superpixels(ctx, image)
    lab = torch.empty((H, W), dtype=torch.int32, device="cuda")
    hist = torch.empty((k, B ** 3), dtype=torch.int32)
    size = torch.empty((k,), dtype=torch.int32)
    if image is None:
        S.seeds_labels(ctx, lab)
        S.seeds_histograms(ctx, hist, size)
    else:
        S.seeds_batch_labels(ctx, image, lab)
        S.seeds_batch_histograms(ctx, image, hist, size)
    return lab.cpu().numpy(), hist.numpy(), size.numpy()


def _check(got, o, what):
    lab, hist, size = got
    ref = o.labels()
    bad = np.argwhere(lab != ref)
    assert bad.size == 0, f"{what}: {len(bad)} labels differ, first at {bad[:5].tolist()}"
    rh, rs = o.histograms()
    assert np.array_equal(hist, rh), what
    assert np.array_equal(size, rs), what


@pytest.mark.parametrize("mode", [0, 1, 2])
# the last two: superpixels of 2x2 and 4x4 pixels, so a warm-start tile meets
# more labels than its key table and slots hold (global-atomic path)
@pytest.mark.parametrize("shape", [(96, 128, 20, 24, 3), (270, 480, 60, 300, 4),
                                   (48, 200, 12, 2400, 1), (64, 192, 12, 768, 2)])
def test_stream_matches_oracle_frame_by_frame(S, mode, shape):
    import torch
    H, W, R, K, L = shape
    _say(f"stream {shape} mode {mode}")
    sc = synth.StreamScene(H=H, W=W, regions=R, frames=6, seed=21, noise_seed=2100)
    f0 = sc.frame(0)
    o = oracle.Oracle(f0, K, L, 5, 3, 1, 0)
    ctx = S.seeds_init(torch.from_numpy(f0).cuda(), K, S.make_params(L, 5, 3, 1, 0))
    try:
        S.seeds_set_launch_mode(ctx, mode)
        S.seeds_refine(ctx)
        o.run(-1)
        _check(_read(S, ctx, H, W, 5), o, "frame 0")
        for f in range(1, 6):
            fr = sc.frame(f)
            S.seeds_warm_start(ctx, torch.from_numpy(fr).cuda())
            S.seeds_refine(ctx)
            o.warm_start(fr)
            o.run(-1)
            got = _read(S, ctx, H, W, 5)
            _check(got, o, f"frame {f}")
            assert valid_partition(got[0], o.K)
        S.seeds_sync(ctx)
    finally:
        S.seeds_destroy(ctx)


def test_warm_start_before_pixel_level_is_refused(S):
    import torch
    _say("warm start refused")
    sc = synth.StreamScene(H=96, W=128, regions=20, frames=3, seed=21, noise_seed=2100)
    f0 = torch.from_numpy(sc.frame(0)).cuda()
    f1 = torch.from_numpy(sc.frame(1)).cuda()
    ctx = S.seeds_init(f0, 24, S.make_params(3, 5, 2, 1, 0))
    try:
        with pytest.raises(S.SeedsError) as e:
            S.seeds_warm_start(ctx, f1)
        assert e.value.status == S.SEEDS_E_STATE
        S.seeds_refine_phases(ctx, 10)           # still at a block level
        with pytest.raises(S.SeedsError):
            S.seeds_warm_start(ctx, f1)
        S.seeds_refine(ctx)                       # the context is still usable
        S.seeds_warm_start(ctx, f1)
        S.seeds_refine(ctx)
        o = oracle.Oracle(sc.frame(0), 24, 3, 5, 2, 1, 0)
        o.run(10)
        o.run(-1)
        o.warm_start(sc.frame(1))
        o.run(-1)
        _check(_read(S, ctx, 96, 128, 5), o, "after refusals")
    finally:
        S.seeds_destroy(ctx)


def test_batch_of_streams_matches_oracle(S):
    import torch
    _say("batch of streams")
    shapes = [(96, 128, 20, 24, 3), (120, 200, 30, 60, 4), (64, 96, 10, 12, 2)]
    scenes = [synth.StreamScene(H=H, W=W, regions=R, frames=4, seed=30 + i, noise_seed=3000 + 10 * i)
              for i, (H, W, R, _, _) in enumerate(shapes)]
    Ks = [s[3] for s in shapes]
    Ls = [s[4] for s in shapes]
    frames = [[torch.from_numpy(sc.frame(f)).cuda() for f in range(4)] for sc in scenes]
    ctx = S.seeds_batch_init([fr[0] for fr in frames], Ks, S.make_params(4, 5, 2, 1, 0), levels=Ls)
    os_ = [oracle.Oracle(sc.frame(0), K, L, 5, 2, 1, 0) for sc, K, L in zip(scenes, Ks, Ls)]
    try:
        S.seeds_refine(ctx)
        for o in os_:
            o.run(-1)
        for f in range(1, 4):
            S.seeds_batch_warm_start(ctx, [fr[f] for fr in frames])
            S.seeds_refine(ctx)
            for i, (o, sc) in enumerate(zip(os_, scenes)):
                o.warm_start(sc.frame(f))
                o.run(-1)
                H, W = shapes[i][:2]
                _check(_read(S, ctx, H, W, 5, image=i), o, f"stream {i} frame {f}")
    finally:
        S.seeds_destroy(ctx)


def test_4k_stream_frames_match_oracle(S):
    """The stream workload at its full size (3840 x 2160, K 5000, 4 levels):
    frame 0 and two warm-started frames against the oracle."""
    import torch
    _say("4k stream")
    sc = synth.StreamScene(frames=3)
    f0 = sc.frame(0)
    o = oracle.Oracle(f0, 5000, 4, 5, 4, 1, 0)
    ctx = S.seeds_init(torch.from_numpy(f0).cuda(), 5000, S.make_params(4, 5, 4, 1, 0))
    try:
        assert S.seeds_num_superpixels(ctx) == o.K == 4982
        S.seeds_refine(ctx)
        o.run(-1)
        _check(_read(S, ctx, 2160, 3840, 5), o, "frame 0")
        for f in (1, 2):
            fr = sc.frame(f)
            S.seeds_warm_start(ctx, torch.from_numpy(fr).cuda())
            S.seeds_refine(ctx)
            o.warm_start(fr)
            o.run(-1)
            _check(_read(S, ctx, 2160, 3840, 5), o, f"frame {f}")
    finally:
        S.seeds_destroy(ctx)
