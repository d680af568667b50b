"""C-ABI checks that run without a GPU: the library loads, exports every
function include/seeds.h declares, validates arguments before any device
work, and computes the superpixel grid exactly as the oracle does (the two
implementations share no code)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "seeds.h")


@pytest.fixture(scope="module")
def S():
    from paper_1309_3848_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=True)
    from paper_1309_3848_amd import seeds
    seeds.lib()
    return seeds


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(seeds_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("seeds_init", "seeds_refine", "seeds_labels", "seeds_num_superpixels",
                 "seeds_destroy", "seeds_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(S):
    L = ctypes.CDLL(S.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_default_params(S):
    p = S.seeds_default_params()
    assert (p.levels, p.bins_per_channel, p.iters_per_level, p.gamma, p.block_rule) == (4, 5, 4, 1, 0)


def test_grid_matches_oracle(S):
    rng = np.random.default_rng(5)
    for _ in range(4000):
        H, W = int(rng.integers(1, 2200)), int(rng.integers(1, 4000))
        if H * W >= 1 << 23:
            continue
        K, L = int(rng.integers(1, 6000)), int(rng.integers(1, 9))
        ref = oracle.grid(H, W, K, L)
        if (1 << (L - 1)) > min(H, W):
            ref = None
        try:
            got = S.seeds_grid(H, W, K, L)
        except S.SeedsError as e:
            assert e.status == S.SEEDS_E_INVAL
            got = None
        assert got == ref, (H, W, K, L)
    assert S.seeds_grid(321, 481, 200, 3) == (17, 12)
    assert S.seeds_grid(1080, 1920, 1000, 4) == (42, 24)
    assert S.seeds_grid(2160, 3840, 5000, 4) == (94, 53)


@pytest.mark.parametrize("H,W,K,kw,msg", [
    (0, 10, 4, {}, "empty"),
    (10, 0, 4, {}, "empty"),
    (4096, 2048, 4, {}, "2^23"),
    (20, 20, 0, {}, "num_superpixels"),
    (20, 20, 4, {"levels": 0}, "levels"),
    (20, 20, 4, {"levels": 9}, "levels"),
    (20, 20, 4, {"bins": 0}, "bins_per_channel"),
    (20, 20, 4, {"bins": 7}, "bins_per_channel"),
    (20, 20, 4, {"iters": -1}, "iters_per_level"),
    (20, 20, 4, {"gamma": -1}, "gamma"),
    (20, 20, 4, {"gamma": 70000}, "gamma"),
    (20, 20, 4, {"rule": 2}, "block_rule"),
    (20, 20, 4, {"levels": 6}, "top block"),
    (20, 20, 400, {"levels": 2}, "grid"),
])
def test_init_rejects_bad_arguments_before_device_work(S, H, W, K, kw, msg):
    import torch
    p = S.make_params(levels=kw.get("levels", 2), bins=kw.get("bins", 5),
                      iters=kw.get("iters", 2), gamma=kw.get("gamma", 1), rule=kw.get("rule", 0))
    ctx = ctypes.c_void_p()
    dummy = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    st = S.lib().seeds_init(ctypes.byref(ctx), dummy, H, W, 3 * max(W, 1), K, ctypes.byref(p), None)
    assert st == S.SEEDS_E_INVAL
    assert not ctx.value
    assert msg in S.seeds_last_error()


def test_null_arguments(S):
    L = S.lib()
    p = S.make_params()
    assert L.seeds_init(None, None, 8, 8, 24, 1, ctypes.byref(p), None) == S.SEEDS_E_INVAL
    ctx = ctypes.c_void_p()
    assert L.seeds_init(ctypes.byref(ctx), None, 8, 8, 24, 1, ctypes.byref(p), None) == S.SEEDS_E_INVAL
    assert "rgb" in S.seeds_last_error()
    assert L.seeds_init(ctypes.byref(ctx), ctypes.c_void_p(4096), 8, 8, 23, 1, ctypes.byref(p),
                        None) == S.SEEDS_E_INVAL
    assert "pitch" in S.seeds_last_error()
    assert L.seeds_refine(None, None) == S.SEEDS_E_INVAL
    assert L.seeds_labels(None, None, 0, None) == S.SEEDS_E_INVAL
    assert L.seeds_histograms(None, None, None, 0, None) == S.SEEDS_E_INVAL
    assert L.seeds_num_superpixels(None) == -1
    assert L.seeds_level(None) == -1
    assert L.seeds_destroy(None) == S.SEEDS_OK
    assert L.seeds_grid(10, 10, 4, 1, None, None) == S.SEEDS_E_INVAL


def test_init_without_a_device_reports_device_error(S):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = S.make_params(levels=2)
    ctx = ctypes.c_void_p()
    st = S.lib().seeds_init(ctypes.byref(ctx), ctypes.c_void_p(1 << 20), 16, 16, 48, 4,
                            ctypes.byref(p), None)
    assert st in (S.SEEDS_E_DEVICE, S.SEEDS_E_NOMEM)
    assert not ctx.value
    assert S.seeds_last_error()


def _images(S, specs):
    arr = (S.seeds_image * len(specs))()
    for i, (H, W, K, L, pitch, ptr) in enumerate(specs):
        arr[i] = S.seeds_image(ptr, H, W, pitch, K, L)
    return arr


@pytest.mark.parametrize("specs,count,msg", [
    ([], 0, "batch of 0"),
    ([(16, 16, 4, 2, 48, 1 << 20)], 4097, "batch of 4097"),
    ([(16, 16, 4, 2, 48, 1 << 20), (16, 16, 4, 2, 48, 0)], 2, "image 1: rgb"),
    ([(16, 16, 4, 2, 48, 1 << 20), (16, 16, 4, 2, 47, 1 << 20)], 2, "image 1: row pitch"),
    ([(16, 16, 4, 9, 48, 1 << 20)], 1, "image 0: levels 9"),
    ([(16, 16, 4, 2, 48, 1 << 20), (0, 16, 4, 2, 48, 1 << 20)], 2, "image 1: image size"),
    ([(16, 16, 4, 2, 48, 1 << 20), (16, 16, 400, 2, 48, 1 << 20)], 2, "image 1: "),
])
def test_batch_init_rejects_bad_images_before_device_work(S, specs, count, msg):
    p = S.make_params()
    ctx = ctypes.c_void_p()
    arr = _images(S, specs) if specs else None
    st = S.lib().seeds_batch_init(ctypes.byref(ctx), arr, count, ctypes.byref(p), None)
    assert st == S.SEEDS_E_INVAL
    assert not ctx.value
    assert msg in S.seeds_last_error()


def test_batch_null_arguments(S):
    L = S.lib()
    p = S.make_params()
    arr = _images(S, [(16, 16, 4, 2, 48, 1 << 20)])
    assert L.seeds_batch_init(None, arr, 1, ctypes.byref(p), None) == S.SEEDS_E_INVAL
    ctx = ctypes.c_void_p()
    assert L.seeds_batch_init(ctypes.byref(ctx), arr, 1, None, None) == S.SEEDS_E_INVAL
    assert L.seeds_batch_reinit(None, None, None, None) == S.SEEDS_E_INVAL
    assert L.seeds_batch_labels(None, 0, None, 0, None) == S.SEEDS_E_INVAL
    assert L.seeds_batch_histograms(None, 0, None, None, 0, None) == S.SEEDS_E_INVAL
    assert L.seeds_batch_num_superpixels(None, 0) == -1
    assert L.seeds_batch_count(None) == -1
    assert L.seeds_warm_start(None, None, 0, None) == S.SEEDS_E_INVAL
    assert L.seeds_batch_warm_start(None, None, None, None) == S.SEEDS_E_INVAL


def test_batch_init_without_a_device_reports_device_error(S):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = S.make_params(levels=2)
    arr = _images(S, [(16, 16, 4, 2, 48, 1 << 20), (20, 24, 6, 1, 72, 1 << 21)])
    ctx = ctypes.c_void_p()
    st = S.lib().seeds_batch_init(ctypes.byref(ctx), arr, 2, ctypes.byref(p), None)
    assert st in (S.SEEDS_E_DEVICE, S.SEEDS_E_NOMEM)
    assert not ctx.value


def test_quality_metrics_argument_checks(S):
    L = S.lib()
    q = S.seeds_quality()
    d = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    assert L.seeds_quality_metrics(None, d, 4, 4, 2, 2, 2, ctypes.byref(q), None) == S.SEEDS_E_INVAL
    assert L.seeds_quality_metrics(d, d, 4, 4, 2, 2, 2, None, None) == S.SEEDS_E_INVAL
    assert L.seeds_quality_metrics(d, d, 0, 4, 2, 2, 2, ctypes.byref(q), None) == S.SEEDS_E_INVAL
    assert L.seeds_quality_metrics(d, d, 4, 4, 0, 2, 2, ctypes.byref(q), None) == S.SEEDS_E_INVAL
    assert L.seeds_quality_metrics(d, d, 4, 4, 1 << 15, 1 << 14, 2, ctypes.byref(q),
                                   None) == S.SEEDS_E_INVAL
    assert "2^28" in S.seeds_last_error()
    assert L.seeds_quality_metrics(d, d, 4, 4, 2, 2, 0, ctypes.byref(q), None) == S.SEEDS_E_INVAL
    assert L.seeds_quality_metrics(d, d, 4, 4, 2, 2, 65, ctypes.byref(q), None) == S.SEEDS_E_INVAL


def test_server_argument_checks(S):
    L = S.lib()
    p = S.seeds_server_default_params()
    assert (p.bins_per_channel, p.iters_per_level, p.gamma, p.max_levels) == (5, 4, 1, 4)
    srv = ctypes.c_void_p()
    for field, bad in (("bins_per_channel", 7), ("iters_per_level", 0), ("gamma", -1),
                       ("max_levels", 9), ("max_inflight", 0), ("hbm_budget_bytes", 1 << 20),
                       ("pixel_compaction", 2), ("xcd_remap", -1), ("items_per_group", 3)):
        q = S.seeds_server_default_params()
        setattr(q, field, bad)
        assert L.seeds_server_create(ctypes.byref(srv), ctypes.byref(q), None) == S.SEEDS_E_INVAL
        assert not srv.value
    assert L.seeds_server_create(None, ctypes.byref(p), None) == S.SEEDS_E_INVAL
    assert L.seeds_server_submit(None, None, 8, 8, 24, 1, 1, None, 0, None) == S.SEEDS_E_INVAL
    assert L.seeds_server_step(None, None) == S.SEEDS_E_INVAL
    assert L.seeds_server_destroy(None) == S.SEEDS_OK


def test_server_without_a_device_reports_device_error(S):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = S.seeds_server_default_params()
    p.hbm_budget_bytes = 64 << 20
    srv = ctypes.c_void_p()
    assert S.lib().seeds_server_create(ctypes.byref(srv), ctypes.byref(p), None) in (
        S.SEEDS_E_DEVICE, S.SEEDS_E_NOMEM)
    assert not srv.value


def test_launch_floor_argument_checks(S):
    L = S.lib()
    us = (ctypes.c_double * 3)()
    assert L.seeds_launch_floor(900, 144, None, None) == S.SEEDS_E_INVAL
    for groups, launches in ((0, 144), (65537, 144), (900, 0), (900, 4097)):
        assert L.seeds_launch_floor(groups, launches, us, None) == S.SEEDS_E_INVAL
    assert b"outside" in S.lib().seeds_last_error()


def test_batch_labels_all_argument_checks(S):
    L = S.lib()
    outs = (ctypes.c_void_p * 1)()
    assert L.seeds_batch_labels_all(None, outs, None) == S.SEEDS_E_INVAL
    assert b"ctx is NULL" in S.lib().seeds_last_error()


def test_traffic_probe_argument_checks(S):
    L = S.lib()
    us = (ctypes.c_double * 3)()
    assert L.seeds_traffic_probe(1 << 19, None, None) == S.SEEDS_E_INVAL
    for lines in (0, 512, 1000, 3 << 18, (1 << 22) + 1, 1 << 23, -1024):
        assert L.seeds_traffic_probe(lines, us, None) == S.SEEDS_E_INVAL
    assert b"power of two" in S.lib().seeds_last_error()


def test_tuning_argument_checks(S):
    L = S.lib()
    t = S.seeds_tuning(1, 1)
    assert L.seeds_get_tuning(None, ctypes.byref(t)) == S.SEEDS_E_INVAL
    assert L.seeds_set_tuning(None, ctypes.byref(t)) == S.SEEDS_E_INVAL
    assert L.seeds_autotune(None, 3, None, None, None) == S.SEEDS_E_INVAL


def test_noalloc_argument_checks_before_device_work(S):
    L = S.lib()
    p = S.make_params(levels=4)
    d = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    assert L.seeds_segment_noalloc(None, 16, 16, 48, 4, ctypes.byref(p), d, None) == S.SEEDS_E_INVAL
    assert L.seeds_segment_noalloc(d, 16, 16, 48, 4, ctypes.byref(p), None, None) == S.SEEDS_E_INVAL
    assert L.seeds_segment_noalloc(d, 16, 16, 47, 4, ctypes.byref(p), d, None) == S.SEEDS_E_INVAL
    assert "pitch" in S.seeds_last_error()
    assert L.seeds_segment_noalloc(d, 16, 16, 48, 4, None, d, None) == S.SEEDS_E_INVAL
    assert L.seeds_segment_noalloc(d, 0, 16, 48, 4, ctypes.byref(p), d, None) == S.SEEDS_E_INVAL
    # a 4K frame's state (about 100 MB) exceeds the fixed array
    assert L.seeds_segment_noalloc(d, 2160, 3840, 3 * 3840, 5000, ctypes.byref(p), d,
                                   None) == S.SEEDS_E_INVAL
    assert "allocation-free" in S.seeds_last_error()


def test_fault_injection_argument_checks(S):
    L = S.lib()
    assert L.seeds_debug_inject_fault(2, 0) == S.SEEDS_E_INVAL
    assert L.seeds_debug_inject_fault(-1, 0) == S.SEEDS_E_INVAL
    assert L.seeds_debug_inject_fault(S.SEEDS_FAULT_ALLOC, -1) == S.SEEDS_OK
    assert L.seeds_debug_inject_fault(S.SEEDS_FAULT_LAUNCH, -1) == S.SEEDS_OK
