"""Serving engine (continuous batching): each request's labels must equal a
single-image context's, and the oracle's, bit for bit, whatever else is in
flight, however arrivals interleave with the ticks, and when admission has to
wait for memory."""
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


def _solo(S, rgb, K, L, B, I, gamma):
    import torch
    ctx = S.seeds_init(rgb, K, S.make_params(L, B, I, gamma, 0))
    try:
        S.seeds_refine(ctx)
        out = torch.empty(rgb.shape[:2], dtype=torch.int32, device="cuda")
        S.seeds_labels(ctx, out)
        return out.cpu().numpy()
    finally:
        S.seeds_destroy(ctx)


def _serve(S, reqs, arrivals, params, host_out=False, max_ticks=100000, pageable=()):
    """reqs: list of (rgb tensor, K, L); arrivals[i]: tick at which request i
    is submitted. Returns labels per request and the server stats."""
    import torch
    srv = S.seeds_server_create(params)
    outs, ids, done = [], {}, set()
    try:
        for i, (rgb, _, _) in enumerate(reqs):
            shape = tuple(rgb.shape[:2])
            if host_out:
                outs.append(torch.empty(shape, dtype=torch.int32, pin_memory=i not in pageable))
            else:
                outs.append(torch.empty(shape, dtype=torch.int32, device="cuda"))
        order = sorted(range(len(reqs)), key=lambda i: arrivals[i])
        nxt, tick = 0, 0
        while len(done) < len(reqs):
            while nxt < len(order) and arrivals[order[nxt]] <= tick:
                i = order[nxt]
                rgb, K, L = reqs[i]
                ids[S.seeds_server_submit(srv, rgb, K, L, outs[i])] = i
                nxt += 1
            S.seeds_server_step(srv)
            done.update(ids[r] for r in S.seeds_server_poll(srv))
            tick += 1
            assert tick < max_ticks, "requests never completed"
        torch.cuda.synchronize()
        stats = S.seeds_server_get_stats(srv)
    finally:
        S.seeds_server_destroy(srv)
    return [o.cpu().numpy() for o in outs], stats


def _params(S, budget=1 << 30, inflight=64, I=3, levels=4, mapping=None, items=None):
    p = S.seeds_server_default_params()
    if mapping is not None:
        p.pixel_compaction, p.xcd_remap = mapping
    if items is not None:
        p.items_per_group = items
    p.iters_per_level = I
    p.max_levels = levels
    p.hbm_budget_bytes = budget
    p.max_inflight = inflight
    return p


SHAPES = [(97, 131, 12, 40, 3), (200, 160, 20, 60, 4), (64, 333, 9, 30, 2),
          (321, 481, 30, 200, 4), (33, 47, 4, 6, 1), (128, 128, 16, 64, 3)]


def _requests(shapes, seed0=500):
    import torch
    imgs = [synth.voronoi_image(H, W, R, 8.0, seed0 + i) for i, (H, W, R, _, _) in enumerate(shapes)]
    return imgs, [(torch.from_numpy(im).cuda(), K, L) for im, (_, _, _, K, L) in zip(imgs, shapes)]


@pytest.mark.parametrize("mapping,items", [((0, 0), 1), ((1, 1), 1), ((0, 1), 2), ((1, 0), 4),
                                           ((0, 0), 2), ((1, 1), 4)])
def test_staggered_arrivals_match_solo_and_oracle(S, mapping, items):
    _say(f"serve staggered {mapping} items {items}")
    imgs, reqs = _requests(SHAPES)
    arrivals = [0, 3, 17, 40, 41, 90]          # several join mid-hierarchy of others
    got, stats = _serve(S, reqs, arrivals, _params(S, mapping=mapping, items=items))
    assert stats["completed"] == len(reqs) and stats["peak_inflight"] >= 2
    for i, (im, (_, _, _, K, L)) in enumerate(zip(imgs, SHAPES)):
        ref, _, _ = oracle.seeds(im, K, L, 5, 3, 1, 0)
        assert np.array_equal(got[i], ref), f"request {i}"


def test_host_outputs_and_simultaneous_arrivals(S):
    _say("serve host outputs")
    imgs, reqs = _requests(SHAPES, seed0=600)
    # pinned outputs take the copy kernel, pageable ones (1 and 4) a plain copy
    got, _ = _serve(S, reqs, [0] * len(reqs), _params(S), host_out=True, pageable=(1, 4))
    for i, (rgb, K, L) in enumerate(reqs):
        assert np.array_equal(got[i], _solo(S, rgb, K, L, 5, 3, 1)), f"request {i}"


def test_admission_waits_for_memory(S):
    """A 64 MiB budget holds the pixels of two 1920x1080 images (14.5 MB each
    of a 38 MB pixel pool): six such requests cannot all be in flight, so the
    later ones wait for earlier ones to leave."""
    import torch
    _say("serve tight budget")
    imgs = [synth.voronoi_image(1080, 1920, 100, 8.0, 700 + i) for i in range(6)]
    reqs = [(torch.from_numpy(im).cuda(), 1000, 4) for im in imgs]
    got, stats = _serve(S, reqs, [0, 0, 0, 5, 9, 30], _params(S, budget=64 << 20, I=2))
    assert stats["peak_inflight"] == 2
    assert stats["peak_bytes_in_use"] <= stats["budget_bytes"]
    for i, (rgb, K, L) in enumerate(reqs):
        assert np.array_equal(got[i], _solo(S, rgb, K, L, 5, 2, 1)), f"request {i}"


def test_inflight_cap(S):
    _say("serve inflight cap")
    imgs, reqs = _requests(SHAPES, seed0=800)
    got, stats = _serve(S, reqs, [0] * len(reqs), _params(S, inflight=2))
    assert stats["peak_inflight"] <= 2
    for i, (rgb, K, L) in enumerate(reqs):
        assert np.array_equal(got[i], _solo(S, rgb, K, L, 5, 3, 1)), f"request {i}"


def test_many_small_requests_with_random_arrivals(S):
    import torch
    _say("serve many")
    rng = np.random.default_rng(9)
    shapes = []
    for i in range(40):
        H, W = int(rng.integers(24, 200)), int(rng.integers(24, 260))
        L = int(rng.integers(1, 5))
        while (1 << (L - 1)) > min(H, W):
            L -= 1
        K = int(max(1, min(int(rng.integers(4, 120)), (H * W) // (4 ** L))))
        shapes.append((H, W, int(rng.integers(2, 20)), K, L))
    imgs, reqs = _requests(shapes, seed0=900)
    arrivals = sorted(int(a) for a in rng.integers(0, 400, size=len(reqs)))
    got, _ = _serve(S, reqs, arrivals, _params(S, I=2))
    for i, (rgb, K, L) in enumerate(reqs):
        assert np.array_equal(got[i], _solo(S, rgb, K, L, 5, 2, 1)), f"request {i} {shapes[i]}"


def test_submit_checks(S):
    import torch
    _say("serve submit checks")
    srv = S.seeds_server_create(_params(S, budget=64 << 20, levels=3))
    try:
        rgb = torch.zeros((64, 64, 3), dtype=torch.uint8, device="cuda")
        out = torch.empty((64, 64), dtype=torch.int32, device="cuda")
        with pytest.raises(S.SeedsError):
            S.seeds_server_submit(srv, rgb, 16, 4, out)         # above max_levels
        big = torch.zeros((2160, 3840, 3), dtype=torch.uint8, device="cuda")
        with pytest.raises(S.SeedsError) as e:
            S.seeds_server_submit(srv, big, 4000, 3, torch.empty((2160, 3840), dtype=torch.int32,
                                                                  device="cuda"))
        assert "budget" in S.seeds_last_error()
        rid = S.seeds_server_submit(srv, rgb, 16, 3, out)       # still usable
        done = []
        while not done:
            S.seeds_server_step(srv)
            done = S.seeds_server_poll(srv)
        assert done == [rid]
    finally:
        S.seeds_server_destroy(srv)


def test_large_requests_in_the_mix(S):
    """Serving sizes of the request trace (640x480, 1080p, 4K) at once."""
    import torch
    _say("serve large mix")
    shapes = [(480, 640, 55, 153, 4), (1080, 1920, 377, 1036, 4), (2160, 3840, 1508, 4147, 4),
              (480, 640, 55, 153, 4), (1080, 1920, 377, 1036, 4)]
    imgs, reqs = _requests(shapes, seed0=1000)
    got, stats = _serve(S, reqs, [0, 0, 3, 20, 60], _params(S, budget=2 << 30, I=4))
    assert stats["peak_inflight"] >= 3
    for i, (rgb, K, L) in enumerate(reqs):
        assert np.array_equal(got[i], _solo(S, rgb, K, L, 5, 4, 1)), f"request {i} {shapes[i][:2]}"
    ref, _, _ = oracle.seeds(imgs[0], 153, 4, 5, 4, 1, 0)
    assert np.array_equal(got[0], ref)
