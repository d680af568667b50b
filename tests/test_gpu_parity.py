"""GPU parity: labels, colour histograms and sizes from the HIP library (through
the C ABI) must equal the CPU oracle's bit for bit, at the end of the schedule
and after every phase, on seeded synthetic images."""
import os
import sys

import numpy as np
import pytest

import oracle
from _defs import colour_histograms, valid_partition

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


# launch modes; "graph_ppl4" is the graph mode with four pixels per lane in
# the block phases of sides 2, 4 and 8 (tuning block_ppl = 4)
MODES = {"graph": 0, "steps": 1, "persistent": 2, "graph_ppl4": 3}
PPL4 = 3


@pytest.fixture(params=list(MODES))
def mode(request):
    return MODES[request.param]


def _set_mode(S, ctx, mode):
    S.seeds_set_tuning(ctx, block_ppl=4 if mode == PPL4 else 1)
    S.seeds_set_launch_mode(ctx, S.SEEDS_LAUNCH_GRAPH if mode == PPL4 else mode)


def _gpu_run(S, img, K, L, B, I, gamma, rule, max_phases=-1, mode=0):
    import torch
    rgb = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    ctx = S.seeds_init(rgb, K, S.make_params(L, B, I, gamma, rule))
    try:
        _set_mode(S, ctx, mode)
        if max_phases < 0:
            S.seeds_refine(ctx)
        else:
            S.seeds_refine_phases(ctx, max_phases)
        keff = S.seeds_num_superpixels(ctx)
        lab = torch.empty(img.shape[:2], dtype=torch.int32, device="cuda")
        S.seeds_labels(ctx, lab)
        hist = torch.empty((keff, B ** 3), dtype=torch.int32)
        size = torch.empty((keff,), dtype=torch.int32)
        S.seeds_histograms(ctx, hist, size)
        S.seeds_sync(ctx)
        return lab.cpu().numpy(), hist.numpy(), size.numpy(), S.seeds_level(ctx)
    finally:
        S.seeds_destroy(ctx)


def _compare(S, img, K, L, B=5, I=4, gamma=1, rule=0, max_phases=-1, check_valid=True, mode=0):
    _say(f"shape={img.shape[:2]} K={K} L={L} B={B} I={I} gamma={gamma} rule={rule} "
         f"max_phases={max_phases} mode={mode}")
    lab, hist, size, level = _gpu_run(S, img, K, L, B, I, gamma, rule, max_phases, mode)
    ref_lab, ref_hist, ref_size = oracle.seeds(img, K, L, B, I, gamma, rule, max_phases)
    assert lab.shape == ref_lab.shape
    bad = np.argwhere(lab != ref_lab)
    assert bad.size == 0, f"{len(bad)} labels differ, first at {bad[:5].tolist()}"
    assert np.array_equal(size, ref_size)
    assert np.array_equal(hist, ref_hist)
    # histograms must also agree with a recount of the GPU's own labels
    o = oracle.Oracle(img, K, L, B, I, gamma, rule)
    assert np.array_equal(hist, colour_histograms(lab, o.bins(), o.K, B ** 3))
    if check_valid:
        assert valid_partition(lab, o.K)
    return lab


# --------------------------------------------------------------------------

def test_small_image_full_schedule(S, mode):
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(97, 131, 12, 8.0, seed=7)
    _compare(S, img, K=40, L=3, B=5, I=2, mode=mode)


def test_481x321_workload(S, mode):
    from paper_1309_3848_amd import synth
    _compare(S, synth.single_481x321(), K=200, L=3, B=5, I=4, gamma=1, mode=mode)


@pytest.mark.parametrize("rule", [0, 1])
def test_1080p_workload(S, mode, rule):
    from paper_1309_3848_amd import synth
    _compare(S, synth.single_1080p(), K=1000, L=4, B=5, I=4, gamma=1, rule=rule,
             check_valid=False, mode=mode)


@pytest.mark.parametrize("case", range(16))
def test_random_configurations(S, case, mode):
    from paper_1309_3848_amd import synth
    rng = np.random.default_rng(500 + case)
    while True:
        L = int(rng.integers(1, 6))
        T = 1 << (L - 1)
        H = int(rng.integers(max(T, 3), 260))
        W = int(rng.integers(max(T, 3), 260))
        K = int(rng.integers(1, 300))
        if oracle.grid(H, W, K, L) is not None:
            break
    B = int(rng.integers(1, 7))
    I = int(rng.integers(0, 4))
    gamma = int(rng.choice([0, 1, 2, 7]))
    rule = int(rng.integers(0, 2))
    img = synth.voronoi_image(H, W, int(rng.integers(3, 40)), float(rng.uniform(2, 16)),
                              seed=600 + case)
    _compare(S, img, K, L, B, I, gamma, rule, mode=mode)


@pytest.mark.parametrize("rule", [0, 1])
def test_every_phase_matches(S, rule, mode):
    """Stop after 0, 1, 2, ... phases: the state (at whatever level) matches."""
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(75, 103, 10, 8.0, seed=31)
    total = 3 * 2 * 9
    for n in range(0, total + 1):
        _compare(S, img, K=30, L=3, B=4, I=2, gamma=1, rule=rule, max_phases=n,
                 check_valid=(n % 9 == 0), mode=mode)


@pytest.mark.parametrize("H,W,K,L", [
    (1, 1, 1, 1), (2, 2, 1, 2), (1, 57, 3, 1), (57, 1, 3, 1), (3, 200, 5, 2), (200, 3, 5, 2),
    (16, 16, 1, 5), (33, 65, 2, 1), (64, 64, 64, 3),
])
def test_edge_shapes(S, H, W, K, L, mode):
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(H, W, 4, 8.0, seed=H * 1000 + W)
    _compare(S, img, K, L, B=5, I=3, gamma=1, mode=mode)


@pytest.mark.parametrize("H,W,K,L", [
    (48, 200, 2400, 1), (48, 200, 2400, 2), (96, 256, 1536, 1), (96, 256, 384, 3), (50, 201, 600, 2),
])
def test_tiles_meeting_many_superpixels(S, H, W, K, L, mode):
    """Initial superpixels of 2x2 and 4x4 pixels: a 64 x 16 initialisation
    tile meets 64-256 of them and counts straight into the global histograms;
    8 x 8 superpixels (and a ragged 50 x 201 image) stay on the LDS path."""
    from paper_1309_3848_amd import synth
    assert oracle.grid(H, W, K, L) is not None
    img = synth.voronoi_image(H, W, 12, 8.0, seed=H * 7 + W + L)
    _compare(S, img, K, L, B=5, I=2, gamma=1, mode=mode)


def _junction_pixels(lab):
    """Pixels 2 or more cells inside the image whose four edge neighbours
    carry three labels other than their own."""
    H, W = lab.shape
    c = lab[2:H - 2, 2:W - 2]
    nbrs = [lab[1:H - 3, 2:W - 2], lab[2:H - 2, 3:W - 1], lab[3:H - 1, 2:W - 2], lab[2:H - 2, 1:W - 3]]
    count = np.zeros(c.shape, int)
    for i, n in enumerate(nbrs):
        new = n != c
        for m in nbrs[:i]:
            new &= n != m
        count += new
    return int((count >= 3).sum())


@pytest.mark.parametrize("gamma", [2, 7])
def test_pixel_decisions_at_junctions(S, gamma, mode):
    """Superpixels of about 3x3 pixels on a 96 x 640 image: the pixel sweeps
    decide many pixels with two and three candidate labels, in wavefronts whose
    pixels are all 2 or more cells inside the image (constant boundary-term
    weights: the image is wider than a wavefront's 190-pixel span) and in
    wavefronts touching the border (computed weights)."""
    from paper_1309_3848_amd import synth
    assert oracle.grid(96, 640, 6800, 2) is not None
    img = synth.voronoi_image(96, 640, 60, 14.0, seed=77 + gamma)
    lab = _compare(S, img, K=6800, L=2, B=4, I=3, gamma=gamma, mode=mode)
    assert _junction_pixels(lab) > 1000


@pytest.mark.parametrize("compaction", [1, 0])
@pytest.mark.parametrize("H,W", [
    (11, 189), (12, 190), (13, 191), (14, 192), (15, 193), (24, 194), (25, 195), (26, 196),
    (37, 383), (12, 384), (13, 385), (5, 577), (190, 14),
])
def test_pixel_tile_edges(S, H, W, compaction):
    """Pixel phases work on tiles of 64 x 4 class pixels (192 x 12 image pixels of
    one class, plus a 2-pixel window margin): shapes on both sides of the tile
    and window edges, with and without the compaction of movable pixels."""
    import torch
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(H, W, 9, 8.0, seed=H * 7919 + W)
    for K, L in ((6, 1), (12, 2)):
        _say(f"tile edges shape={H}x{W} K={K} L={L} compaction={compaction}")
        rgb = torch.from_numpy(img).cuda()
        ctx = S.seeds_init(rgb, K, S.make_params(L, 5, 3, 1, 0))
        try:
            S.seeds_set_tuning(ctx, compaction, 1)
            S.seeds_refine(ctx)
            lab = torch.empty((H, W), dtype=torch.int32, device="cuda")
            S.seeds_labels(ctx, lab)
            keff = S.seeds_num_superpixels(ctx)
            hist = torch.empty((keff, 125), dtype=torch.int32)
            size = torch.empty((keff,), dtype=torch.int32)
            S.seeds_histograms(ctx, hist, size)
            S.seeds_sync(ctx)
        finally:
            S.seeds_destroy(ctx)
        ref_lab, ref_hist, ref_size = oracle.seeds(img, K, L, 5, 3, 1, 0)
        bad = np.argwhere(lab.cpu().numpy() != ref_lab)
        assert bad.size == 0, f"{len(bad)} labels differ, first at {bad[:5].tolist()}"
        assert np.array_equal(hist.numpy(), ref_hist)
        assert np.array_equal(size.numpy(), ref_size)


def test_flat_and_two_colour_images(S, mode):
    img = np.full((64, 96, 3), 140, np.uint8)
    _compare(S, img, 24, 4, 5, 3, 0, mode=mode)
    img = np.zeros((32, 64, 3), np.uint8)
    img[:, :35] = (200, 40, 40)
    img[:, 35:] = (30, 30, 220)
    lab = _compare(S, img, 2, 3, 5, 12, 1, mode=mode)
    assert np.array_equal(lab, (np.arange(64)[None, :] >= 35).astype(np.int32).repeat(32, 0))


def test_largest_block_sizes(S, mode):
    """levels = 8: blocks of side 128, 64, 32, 16 use the multi-pixel-per-lane path."""
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(300, 530, 20, 8.0, seed=77)
    _compare(S, img, 4, 8, 5, 1, 1, mode=mode)
    _compare(S, img, 4, 8, 3, 2, 1, rule=1, mode=mode)


@pytest.mark.parametrize("rule", [0, 1])
def test_alternating_launch_modes(S, rule):
    """Phases run alternately by the persistent kernel, by per-step launches
    and by graphs with either block shape: each keeps the two histogram copies
    equal between calls."""
    import torch
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(110, 150, 14, 8.0, seed=91)
    rgb = torch.from_numpy(img).cuda()
    ctx = S.seeds_init(rgb, 36, S.make_params(3, 5, 3, 1, rule))
    o = oracle.Oracle(img, 36, 3, 5, 3, 1, rule)
    try:
        for i, n in enumerate([5, 4, 9, 1, 13, 2, 30, 100]):
            _set_mode(S, ctx, i % 4)
            _say(f"alternating step {i}: {n} phases mode {i % 4}")
            S.seeds_refine_phases(ctx, n)
            o.run(n)
            lab = torch.empty((110, 150), dtype=torch.int32)
            S.seeds_labels(ctx, lab)
            hist = torch.empty((o.K, 125), dtype=torch.int32)
            size = torch.empty((o.K,), dtype=torch.int32)
            S.seeds_histograms(ctx, hist, size)
            rh, rs = o.histograms()
            assert np.array_equal(lab.numpy(), o.labels())
            assert np.array_equal(hist.numpy(), rh) and np.array_equal(size.numpy(), rs)
    finally:
        S.seeds_destroy(ctx)


def test_determinism_and_repeat_refine(S):
    import torch
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(120, 170, 15, 8.0, seed=41)
    a = _gpu_run(S, img, 50, 3, 5, 3, 1, 0)
    b = _gpu_run(S, img, 50, 3, 5, 3, 1, 0)
    assert all(np.array_equal(x, y) for x, y in zip(a[:3], b[:3]))
    # a second refine runs I more pixel-level sweeps, like the oracle
    rgb = torch.from_numpy(img).cuda()
    ctx = S.seeds_init(rgb, 50, S.make_params(3, 5, 3, 1, 0))
    try:
        S.seeds_refine(ctx)
        S.seeds_refine(ctx)
        lab = torch.empty((120, 170), dtype=torch.int32)
        S.seeds_labels(ctx, lab)
    finally:
        S.seeds_destroy(ctx)
    o = oracle.Oracle(img, 50, 3, 5, 3, 1, 0)
    o.run()
    o.run()
    assert np.array_equal(lab.numpy(), o.labels())


def test_reinit_with_a_new_image(S):
    import torch
    from paper_1309_3848_amd import synth
    img1 = synth.voronoi_image(90, 140, 9, 8.0, seed=51)
    img2 = synth.voronoi_image(90, 140, 14, 6.0, seed=52)
    ctx = S.seeds_init(torch.from_numpy(img1).cuda(), 40, S.make_params(3, 5, 2, 1, 0))
    try:
        S.seeds_refine(ctx)
        S.seeds_reinit(ctx, torch.from_numpy(img2).cuda())
        S.seeds_refine(ctx)
        lab = torch.empty((90, 140), dtype=torch.int32)
        S.seeds_labels(ctx, lab)
    finally:
        S.seeds_destroy(ctx)
    ref, _, _ = oracle.seeds(img2, 40, 3, 5, 2, 1, 0)
    assert np.array_equal(lab.numpy(), ref)


def test_strided_rows(S):
    import torch
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(70, 90, 9, 8.0, seed=61)
    big = torch.zeros((70, 100, 3), dtype=torch.uint8)
    big[:, :90] = torch.from_numpy(img)
    view = big.cuda()[:, :90]           # row pitch 300 bytes, not 270
    ctx = S.seeds_init(view, 20, S.make_params(2, 5, 2, 1, 0))
    try:
        S.seeds_refine(ctx)
        lab = torch.empty((70, 90), dtype=torch.int32)
        S.seeds_labels(ctx, lab)
    finally:
        S.seeds_destroy(ctx)
    ref, _, _ = oracle.seeds(img, 20, 2, 5, 2, 1, 0)
    assert np.array_equal(lab.numpy(), ref)


@pytest.mark.parametrize("H,W,K,L", [(37, 53, 12, 2), (321, 481, 200, 4)])
def test_labels_into_outputs_at_every_alignment(S, H, W, K, L):
    """Device label readback at offsets 0..4 ints into a larger buffer (only
    offsets 0 and 4 allow 16-byte pieces; H W mod 4 = 1 leaves a ragged
    tail): the labels equal the oracle's and nothing around them is written."""
    import torch
    from paper_1309_3848_amd import synth
    _say(f"labels at every alignment {H}x{W}")
    img = synth.voronoi_image(H, W, 9, 8.0, seed=71)
    ref, _, _ = oracle.seeds(img, K, L, 5, 2, 1, 0)
    n = H * W
    ctx = S.seeds_init(torch.from_numpy(img).cuda(), K, S.make_params(L, 5, 2, 1, 0))
    try:
        S.seeds_refine(ctx)
        for off in range(5):
            buf = torch.full((n + 16,), -7, dtype=torch.int32, device="cuda")
            S.seeds_labels(ctx, buf[off:off + n].view(H, W))
            got = buf.cpu().numpy()
            assert np.array_equal(got[off:off + n].reshape(H, W), ref), f"offset {off}"
            assert (got[:off] == -7).all() and (got[off + n:] == -7).all(), f"offset {off}"
    finally:
        S.seeds_destroy(ctx)


@pytest.mark.parametrize("rule", [0, 1])
def test_graph_replays(S, rule):
    """The refinement graph is captured on the first refine and replayed by
    later ones (after reinit, and for the pixel-only second refine), with
    eager work and synchronisations in between; every replay must equal the
    oracle."""
    import torch
    from paper_1309_3848_amd import synth
    imgs = [synth.voronoi_image(100, 140, 12, 8.0, seed=200 + i) for i in range(3)]
    ctx = S.seeds_init(torch.from_numpy(imgs[0]).cuda(), 40, S.make_params(3, 5, 2, 1, rule))
    try:
        S.seeds_set_launch_mode(ctx, S.SEEDS_LAUNCH_GRAPH)
        for rep in range(6):
            img = imgs[rep % 3]
            _say(f"graph replay {rep}")
            S.seeds_reinit(ctx, torch.from_numpy(img).cuda())
            S.seeds_refine(ctx)
            junk = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")
            torch.cuda.synchronize()
            S.seeds_refine(ctx)  # pixel-only sweeps: a second cached graph
            lab = torch.empty((100, 140), dtype=torch.int32)
            S.seeds_labels(ctx, lab)
            hist = torch.empty((S.seeds_num_superpixels(ctx), 125), dtype=torch.int32)
            S.seeds_histograms(ctx, hist, None)
            o = oracle.Oracle(img, 40, 3, 5, 2, 1, rule)
            o.run()
            o.run()
            assert np.array_equal(lab.numpy(), o.labels()), rep
            assert np.array_equal(hist.numpy(), o.histograms()[0]), rep
            del junk
    finally:
        S.seeds_destroy(ctx)


@pytest.mark.parametrize("H,W,K,L", [(1024, 8191, 4000, 4), (8191, 1024, 3000, 3)])
def test_largest_image(S, H, W, K, L):
    """H * W just below the 2^23 limit, in both orientations."""
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(H, W, 300, 8.0, seed=77)
    _compare(S, img, K=K, L=L, B=5, I=2, gamma=1, rule=0, check_valid=False)


def test_image_at_the_limit_is_refused(S):
    import torch
    rgb = torch.zeros((2048, 4096, 3), dtype=torch.uint8, device="cuda")   # exactly 2^23 pixels
    with pytest.raises(S.SeedsError) as e:
        S.seeds_init(rgb, 1000, S.make_params(4, 5, 2, 1, 0))
    assert e.value.status == S.SEEDS_E_INVAL


@pytest.mark.parametrize("K,keff", [(70000, 69960), (65535, 65536), (65000, 65025)])
def test_label_width_on_both_sides_of_16_bits(S, mode, K, keff):
    """Pixel labels are stored in 16 bits up to 65535 superpixels and in 32
    bits above; both paths equal the oracle (tiny superpixels, two levels)."""
    from paper_1309_3848_amd import synth
    img = synth.voronoi_image(600, 600, 500, 8.0, seed=91)
    lab = _compare(S, img, K=K, L=2, B=5, I=2, gamma=1, rule=0, check_valid=False, mode=mode)
    assert lab.max() < keff
    gx, gy = S.seeds_grid(600, 600, K, 2)
    assert gx * gy == keff


def test_warm_start_with_32_bit_labels(S):
    """A stream whose superpixel count needs 32-bit labels: frame 0 and a
    warm-started frame 1 against the oracle."""
    import torch
    from paper_1309_3848_amd import synth
    sc = synth.StreamScene(H=600, W=600, regions=300, frames=2)
    f0, f1 = sc.frame(0), sc.frame(1)
    params = S.make_params(2, 5, 2, 1, 0)
    ctx = S.seeds_init(torch.from_numpy(f0).cuda(), 70000, params)
    try:
        assert S.seeds_num_superpixels(ctx) == 69960
        S.seeds_refine(ctx)
        S.seeds_warm_start(ctx, torch.from_numpy(f1).cuda())
        S.seeds_refine(ctx)
        lab = torch.empty((600, 600), dtype=torch.int32)
        S.seeds_labels(ctx, lab)
    finally:
        S.seeds_destroy(ctx)
    o = oracle.Oracle(f0, 70000, 2, 5, 2, 1, 0)
    o.run()
    o.warm_start(f1)
    o.run()
    assert np.array_equal(lab.numpy(), o.labels())
