"""The allocation-free entry point (seeds_segment_noalloc) against the
allocating path it stands for (seeds_init + seeds_refine + seeds_labels +
seeds_destroy), through the C ABI: labels bit for bit, on consecutive calls
that reuse the library's one device array, the second with a smaller image;
one case also against the CPU oracle."""
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


def _allocating(S, rgb, K, params):
    import torch
    ctx = S.seeds_init(rgb, K, params)
    try:
        S.seeds_refine(ctx)
        out = torch.empty(rgb.shape[:2], dtype=torch.int32, device=rgb.device)
        S.seeds_labels(ctx, out)
        S.seeds_sync(ctx)
    finally:
        S.seeds_destroy(ctx)
    return out.cpu().numpy()


def _noalloc(S, rgb, K, params):
    import torch
    out = torch.full(rgb.shape[:2], -7, dtype=torch.int32, device=rgb.device)
    S.seeds_segment_noalloc(rgb, K, params, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


# (H, W, regions, seed, K, levels, bins) pairs: the second image of each case
# is smaller than the first, so stale state of the first call would show
CASES = [
    ((1080, 1920, 400, 2, 1000, 4, 5), (321, 481, 30, 1, 200, 3, 5)),
    ((300, 500, 40, 11, 300, 3, 5), (97, 131, 12, 12, 40, 2, 5)),
    ((240, 320, 30, 21, 200, 4, 5), (61, 53, 6, 22, 9, 1, 5)),
    # more than 65535 superpixels (32-bit pixel labels; 2 bins per channel so
    # that their histograms fit the array), then 16-bit labels
    ((600, 600, 300, 23, 70000, 2, 2), (200, 300, 25, 24, 150, 3, 5)),
]


@pytest.mark.parametrize("rule", [0, 1], ids=["intersect", "exact"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_two_calls_match_the_allocating_path(S, case, rule):
    import torch
    for (H, W, R, seed, K, L, B) in CASES[case]:
        _say("noalloc", H, W, K, L, B, "rule", rule)
        rgb = torch.from_numpy(_img(H, W, R, seed)).cuda()
        params = S.make_params(L, B, 4, 1, rule)
        want = _allocating(S, rgb, K, params)
        got = _noalloc(S, rgb, K, params)
        assert np.array_equal(got, want), (H, W, K, L, rule)


def test_matches_the_oracle_after_a_larger_call(S):
    import torch
    big = torch.from_numpy(_img(720, 1280, 200, 31)).cuda()
    _noalloc(S, big, 800, S.make_params(4, 5, 4, 1, 0))
    img = _img(97, 131, 12, 7)
    _say("noalloc vs oracle 97x131")
    got = _noalloc(S, torch.from_numpy(img).cuda(), 40, S.make_params(3, 5, 2, 1, 0))
    ref, _, _ = oracle.seeds(img, 40, 3, 5, 2, 1, 0)
    assert np.array_equal(got, ref)


def test_strided_rows_and_repeat(S):
    import torch
    img = _img(200, 300, 25, 41)
    padded = torch.zeros((200, 320, 3), dtype=torch.uint8)
    padded[:, :300] = torch.from_numpy(img)
    rgb = padded.cuda()[:, :300]
    params = S.make_params(3, 5, 3, 1, 0)
    want = _allocating(S, torch.from_numpy(img).cuda(), 150, params)
    for _ in range(2):
        _say("noalloc strided 200x300")
        assert np.array_equal(_noalloc(S, rgb, 150, params), want)


def test_refuses_images_beyond_the_array(S):
    import torch
    rgb = torch.zeros((2160, 3840, 3), dtype=torch.uint8, device="cuda")
    out = torch.empty((2160, 3840), dtype=torch.int32, device="cuda")
    with pytest.raises(S.SeedsError) as e:
        S.seeds_segment_noalloc(rgb, 5000, S.make_params(4, 5, 4, 1, 0), out)
    assert e.value.status == S.SEEDS_E_INVAL
    assert "allocation-free" in str(e.value)
