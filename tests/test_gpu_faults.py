"""Error paths, forced from the host (seeds_debug_inject_fault): an allocation
or a kernel launch reports a failure instead of running, so nothing faults on
the device. A failed allocation leaves no context behind; a failed launch
poisons the context or server (every later call but destroy returns
SEEDS_E_STATE), the caller's stream stays usable, and fresh contexts still
equal the oracle."""
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
    yield seeds
    seeds.seeds_debug_inject_fault(seeds.SEEDS_FAULT_ALLOC, -1)
    seeds.seeds_debug_inject_fault(seeds.SEEDS_FAULT_LAUNCH, -1)


@pytest.fixture
def img():
    from paper_1309_3848_amd import synth
    return synth.voronoi_image(97, 131, 12, 8.0, 7)


def _fresh_run_matches_oracle(S, img):
    import torch
    rgb = torch.from_numpy(img).cuda()
    ctx = S.seeds_init(rgb, 40, S.make_params(3, 5, 2, 1, 0))
    try:
        S.seeds_refine(ctx)
        lab = torch.empty(img.shape[:2], dtype=torch.int32)
        S.seeds_labels(ctx, lab)
    finally:
        S.seeds_destroy(ctx)
    ref, _, _ = oracle.seeds(img, 40, 3, 5, 2, 1, 0)
    assert np.array_equal(lab.numpy(), ref)


def _poisoned(S, ctx):
    import torch
    for call in (lambda: S.seeds_refine(ctx),
                 lambda: S.seeds_labels(ctx, torch.empty((4, 4), dtype=torch.int32)),
                 lambda: S.seeds_sync(ctx)):
        with pytest.raises(S.SeedsError) as e:
            call()
        assert e.value.status == S.SEEDS_E_STATE


def test_allocation_failure_in_init(S, img):
    import torch
    rgb = torch.from_numpy(img).cuda()
    for make in (lambda: S.seeds_init(rgb, 40, S.make_params(3, 5, 2, 1, 0)),
                 lambda: S.seeds_batch_init([rgb, rgb], 40, S.make_params(3, 5, 2, 1, 0))):
        S.seeds_debug_inject_fault(S.SEEDS_FAULT_ALLOC, 0)
        with pytest.raises(S.SeedsError) as e:
            make()
        assert e.value.status == S.SEEDS_E_NOMEM
    _fresh_run_matches_oracle(S, img)


def test_allocation_failure_in_server_create(S, img):
    p = S.seeds_server_default_params()
    p.hbm_budget_bytes = 64 << 20
    S.seeds_debug_inject_fault(S.SEEDS_FAULT_ALLOC, 0)
    with pytest.raises(S.SeedsError) as e:
        S.seeds_server_create(p)
    assert e.value.status == S.SEEDS_E_NOMEM
    srv = S.seeds_server_create(p)
    S.seeds_server_destroy(srv)


def test_launch_failure_at_init(S, img):
    import torch
    S.seeds_debug_inject_fault(S.SEEDS_FAULT_LAUNCH, 0)
    with pytest.raises(S.SeedsError) as e:
        S.seeds_init(torch.from_numpy(img).cuda(), 40, S.make_params(3, 5, 2, 1, 0))
    assert e.value.status == S.SEEDS_E_DEVICE
    _fresh_run_matches_oracle(S, img)


@pytest.mark.parametrize("mode", [0, 1, 2], ids=["graph", "steps", "persistent"])
@pytest.mark.parametrize("after", [0, 7, 40])
def test_launch_failure_in_refine_poisons_the_context(S, img, mode, after):
    import torch
    _say("launch fault mode", mode, "after", after)
    ctx = S.seeds_init(torch.from_numpy(img).cuda(), 40, S.make_params(3, 5, 2, 1, 0))
    S.seeds_set_launch_mode(ctx, mode)
    S.seeds_debug_inject_fault(S.SEEDS_FAULT_LAUNCH, after if mode != 2 else 0)
    with pytest.raises(S.SeedsError) as e:
        S.seeds_refine(ctx)
    assert e.value.status == S.SEEDS_E_DEVICE
    _poisoned(S, ctx)
    S.seeds_destroy(ctx)
    torch.cuda.current_stream().synchronize()
    _fresh_run_matches_oracle(S, img)


def test_launch_failure_in_warm_start(S, img):
    import torch
    rgb = torch.from_numpy(img).cuda()
    ctx = S.seeds_init(rgb, 40, S.make_params(3, 5, 2, 1, 0))
    S.seeds_refine(ctx)
    S.seeds_debug_inject_fault(S.SEEDS_FAULT_LAUNCH, 0)
    with pytest.raises(S.SeedsError) as e:
        S.seeds_warm_start(ctx, rgb)
    assert e.value.status == S.SEEDS_E_DEVICE
    _poisoned(S, ctx)
    S.seeds_destroy(ctx)
    _fresh_run_matches_oracle(S, img)


def test_launch_failure_in_a_server_tick(S, img):
    import torch
    p = S.seeds_server_default_params()
    p.hbm_budget_bytes = 64 << 20
    srv = S.seeds_server_create(p)
    rgb = torch.from_numpy(img).cuda()
    out = torch.empty(img.shape[:2], dtype=torch.int32, device="cuda")
    S.seeds_server_submit(srv, rgb, 40, 3, out)
    S.seeds_server_step(srv)
    S.seeds_debug_inject_fault(S.SEEDS_FAULT_LAUNCH, 0)
    with pytest.raises(S.SeedsError) as e:
        S.seeds_server_step(srv)
    assert e.value.status == S.SEEDS_E_DEVICE
    for call in (lambda: S.seeds_server_step(srv), lambda: S.seeds_server_poll(srv)):
        with pytest.raises(S.SeedsError) as e:
            call()
        assert e.value.status == S.SEEDS_E_STATE
    S.seeds_server_destroy(srv)
    _fresh_run_matches_oracle(S, img)
