"""Benchmark: SEEDS refinement throughput on one MI355X.

A step is the whole hot path for one image already resident in HBM:
re-initialise the context from the image (quantise, grid, colour histograms),
run the full refinement schedule (all block levels, then pixel level), and
write the labels to a device buffer. Workload: one 1920 x 1080 synthetic image
(400 Voronoi regions + gradient + Gaussian noise sigma 8), K = 1000 requested
(1008 on the grid), 4 levels, 5 bins per channel, 4 sweeps per level, gamma 1,
Prop. 1 block rule.

Prints one JSON line (rank 0). `roofline` reports the refine kernel against
the HBM roofline with the algorithmic bytes of the schedule; `cpu_baseline`
times the CPU oracle on the same image and checks the GPU labels against it.
Before the warm-up the context's launch mapping is autotuned (seeds_autotune;
the mapping never changes a result), unless --no-autotune.

`--workload stream4k` measures a 300-frame 3840 x 2160 video stream: frame 0
runs the whole hierarchy, every later frame is warm-started from the previous
labels (re-binned, recounted, 4 pixel sweeps); K = 5000, 4 levels, 5 bins.
Every frame is resident in HBM before timing; value is frames x pixels over
the wall time of the pass, latency is per frame.

`--workload quality` refines 20 481 x 321 images (K = 200) three ways - the
initial grid, pixel-level updates only (one level), SEEDS with 3 levels - and
reports the metrics of Sec. 6.1 (UE, CUE, ASA, BR with eps 2) against the
images' Voronoi region maps, computed on the device.

`--workload serve` replays a request trace through the serving engine:
Poisson arrivals at 2000 requests/s of 640x480 (70%), 1920x1080 (25%) and
3840x2160 (5%) images, K = pixels/2000, 4 levels; 500 warm-up requests, then
4000 timed ones. Latency runs from a request's arrival to its labels in host
memory; value is the timed requests' pixels over the time from the first
timed arrival to the last completion. The line also gives the plain path
(single-image contexts back to back) on the same requests.

`--workload batch64` measures the mixed batch instead: 64 synthetic images,
W ~ U{320..1920}, H ~ U{240..1080}, 50-600 Voronoi regions, noise sigma in
[4,16], K ~ U{200..2000} clamped to N/256, 3-4 levels, 5 bins, 4 sweeps,
gamma 1, Prop. 1 rule, refined by one batch context (one launch per phase for
all images). A step re-initialises all 64 images, refines them and writes
their labels to device buffers. The line also reports the same images run
one after another through single-image contexts (the plain path).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

H, W, K, LEVELS, BINS, ITERS, GAMMA, RULE = 1080, 1920, 1000, 4, 5, 4, 1, 0
HBM_PEAK_GBS = 8000.0
METRIC = "Mpixel/s SEEDS refine (bit-exact vs oracle) + p50/p99 latency; % HBM peak"


def phase_bytes(h: int, w: int, level: int, cls: int) -> float:
    """Algorithmic bytes of one phase launch: the unit-label plane of the level
    (4 B per unit; the neighbourhoods of one class cover the whole plane) and
    the colour bins of the class's units (1 B per pixel of those units). Moved
    labels and histogram deltas are a few percent and not counted."""
    s = 1 << level
    uw, uh = -(-w // s), -(-h // s)
    cw = (uw - cls % 3 + 2) // 3 if cls % 3 < uw else 0
    ch = (uh - cls // 3 + 2) // 3 if cls // 3 < uh else 0
    px_per_unit = s * s
    return 4.0 * uw * uh + 1.0 * cw * ch * px_per_unit


def schedule_bytes(h: int, w: int, levels: int, iters: int):
    """(phase launches, algorithmic bytes of all phases, of init, of output)."""
    launches, total = 0, 0.0
    for lev in range(levels - 1, -1, -1):
        for _ in range(iters):
            for c in range(9):
                total += phase_bytes(h, w, lev, c)
                launches += 1
    n = h * w
    top = 1 << (levels - 1)
    init = 3.0 * n + 1.0 * n + 4.0 * (-(-h // top) * -(-w // top))
    out = 8.0 * n
    return launches, total, init, out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_phase_1080p_traffic.json")
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_phase_batch64_traffic.json")
STREAM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_phase_stream4k_traffic.json")
KERNEL_SOURCES = ["seeds_phase.h", "seeds_phase.hip", "seeds_device.h", "seeds_internal.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1309_3848_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per phase launch of a workload from the committed rocprofv3
    FETCH_SIZE and WRITE_SIZE runs, or None when the kernel sources changed
    since."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t.get("traffic_bytes_per_launch")


LDS_FILE = os.path.join(ROOT, "profiles", "k_phase_1080p_lds.json")
# LDS atomics: one wavefront instruction of 64 32-bit lanes moves 256 B
# through a CU's 128 B/clock LDS pipe, so at most one every two clocks per CU
LDS_ATOMIC_PEAK_GINST = 256 * 2.4 / 2


def measured_lds():
    """LDS counters per phase launch from the committed rocprofv3 run, or None
    when the kernel sources changed since."""
    try:
        with open(LDS_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t


def _percentiles(lat):
    lat = sorted(lat)
    return lat[len(lat) // 2], lat[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]


def run_batch(args) -> int:
    import numpy as np
    import torch

    from paper_1309_3848_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=True)
    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    specs = synth.batch_mixed(64)
    imgs = [synth.voronoi_image(s["H"], s["W"], s["regions"], s["sigma"], s["seed"])
            for s in specs]
    rgbs = [torch.from_numpy(im).to(dev) for im in imgs]
    Ks = [s["K"] for s in specs]
    Ls = [s["levels"] for s in specs]
    npx = sum(s["H"] * s["W"] for s in specs)
    outs = [torch.empty((s["H"], s["W"]), dtype=torch.int32, device=dev) for s in specs]
    stream = torch.cuda.current_stream()
    params = S.make_params(max(Ls), BINS, ITERS, GAMMA, RULE)
    ctx = S.seeds_batch_init(rgbs, Ks, params, levels=Ls, stream=stream)
    tuning = None
    if not args.no_autotune:
        chosen, ms = S.seeds_autotune(ctx, 3, stream)
        tuning = {"chosen": chosen, "refine_ms_per_variant": [round(m, 3) for m in ms]}

    def step():
        S.seeds_batch_reinit(ctx, rgbs, stream)
        S.seeds_refine(ctx, stream)
        for i in range(len(specs)):
            S.seeds_batch_labels(ctx, i, outs[i], stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    p50, p99 = _percentiles([a.elapsed_time(b) for a, b in zip(starts, ends)])
    ms_per_step = wall * 1e3 / args.steps

    reps = max(5, args.steps // 2)
    r0 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    r1 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    for i in range(reps):
        S.seeds_batch_reinit(ctx, rgbs, stream)
        r0[i].record(stream)
        S.seeds_refine(ctx, stream)
        r1[i].record(stream)
    for i in range(len(specs)):
        S.seeds_batch_labels(ctx, i, outs[i], stream)
    torch.cuda.synchronize()
    refine_ms = sum(a.elapsed_time(b) for a, b in zip(r0, r1)) / reps
    S.seeds_sync(ctx, stream)
    S.seeds_destroy(ctx)
    gpu_labels = [o.cpu().numpy() for o in outs]

    # the plain path: the same images through single-image contexts, in turn
    solo = [S.seeds_init(r, k, S.make_params(l, BINS, ITERS, GAMMA, RULE), stream)
            for r, k, l in zip(rgbs, Ks, Ls)]

    def solo_step():
        for c, r, o in zip(solo, rgbs, outs):
            S.seeds_reinit(c, r, stream)
            S.seeds_refine(c, stream)
            S.seeds_labels(c, o, stream)

    for _ in range(max(2, args.warmup // 4)):
        solo_step()
    torch.cuda.synchronize()
    solo_steps = max(3, args.steps // 4)
    t1 = time.perf_counter()
    for _ in range(solo_steps):
        solo_step()
    torch.cuda.synchronize()
    solo_ms = (time.perf_counter() - t1) * 1e3 / solo_steps
    solo_same = all(bool(np.array_equal(o.cpu().numpy(), g)) for o, g in zip(outs, gpu_labels))
    for c in solo:
        S.seeds_destroy(c)

    # algorithmic bytes of all phase launches (each image over its own levels)
    launches = max(Ls) * ITERS * 9
    refine_bytes = sum(schedule_bytes(s["H"], s["W"], s["levels"], ITERS)[1] for s in specs)
    per_launch = refine_bytes / launches
    phase_us = refine_ms * 1e3 / launches
    achieved = per_launch / (phase_us * 1e-6) / 1e9
    result = {
        "metric": METRIC, "value": round(npx * args.steps / wall / 1e6, 2), "unit": "Mpixel/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batch of 64 mixed RGB u8 images (W 320-1920, H 240-1080, "
                               "50-600 Voronoi regions, noise sigma 4-16, seeds 3000+i); K 200-2000 "
                               "clamped to N/256, 3-4 levels, 5 bins/channel, 4 sweeps/level, "
                               "gamma 1, Prop. 1 block rule; one batch context",
                   "images": len(specs), "megapixels": round(npx / 1e6, 3),
                   "step": "batch reinit + refine + labels of every image (device)"},
        "p50_ms": round(p50, 4), "p99_ms": round(p99, 4),
        "images_per_s": round(len(specs) * args.steps / wall, 1), "tuning": tuning,
        "plain_path": {"ms_per_batch": round(solo_ms, 4),
                       "value": round(npx / (solo_ms * 1e-3) / 1e6, 2), "unit": "Mpixel/s",
                       "labels_equal_to_batch": solo_same},
        "roofline": {"bound": "hbm", "kernel": "k_phase (batch variant; one phase of every "
                                               "image per launch)",
                     "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 6),
                     "traffic": measured_traffic(BATCH_TRAFFIC_FILE),
                     "algorithmic_bytes_per_launch": int(per_launch),
                     "launches_per_batch": launches, "avg_launch_us": round(phase_us, 3),
                     "refine_ms": round(refine_ms, 4)},
    }
    if not args.no_cpu_baseline:
        import oracle
        order = np.argsort([s["H"] * s["W"] for s in specs])
        # the smallest, median and largest image first, then others in turn
        # until about cpu_seconds of oracle work
        sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
        sample += [i for i in range(len(specs)) if i not in sample]
        t2 = time.perf_counter()
        px, same, used = 0, True, []
        for i in sample:
            if len(used) >= 3 and time.perf_counter() - t2 >= args.cpu_seconds:
                break
            ref, _, _ = oracle.seeds(imgs[i], Ks[i], Ls[i], BINS, ITERS, GAMMA, RULE)
            px += imgs[i].shape[0] * imgs[i].shape[1]
            same &= bool(np.array_equal(gpu_labels[i], ref))
            used.append(i)
        cpu_s = time.perf_counter() - t2
        result["cpu_baseline"] = {
            "value": round(px / cpu_s / 1e6, 3), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(used)} images of the batch ({px / 1e6:.1f} Mpx; first the smallest, "
                      f"median and largest), full runs, single-threaded C oracle, {cpu_s:.1f} s"}
        result["bitexact_vs_oracle"] = same
    print(json.dumps(result), flush=True)
    return 0


def run_stream(args) -> int:
    import concurrent.futures as cf

    import numpy as np
    import torch

    from paper_1309_3848_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=True)
    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    SH, SW, SK = 2160, 3840, 5000
    nfr = args.frames
    scene = synth.StreamScene(H=SH, W=SW, regions=1500, frames=nfr)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        host = list(ex.map(scene.frame, range(nfr)))
    gen_s = time.perf_counter() - t0
    frames = [torch.from_numpy(f).to(dev) for f in host]   # every frame resident in HBM
    out = torch.empty((SH, SW), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    params = S.make_params(LEVELS, BINS, ITERS, GAMMA, RULE)

    def cold(ctx, f):
        S.seeds_reinit(ctx, frames[f], stream)
        S.seeds_refine(ctx, stream)
        S.seeds_labels(ctx, out, stream)

    def warm(ctx, f):
        S.seeds_warm_start(ctx, frames[f], stream)
        S.seeds_refine(ctx, stream)
        S.seeds_labels(ctx, out, stream)

    ctx = S.seeds_init(frames[0], SK, params, stream)
    keff = S.seeds_num_superpixels(ctx)
    tuning = None
    if not args.no_autotune:
        chosen, ms = S.seeds_autotune(ctx, 3, stream)
        tuning = {"chosen": chosen, "refine_ms_per_variant": [round(m, 3) for m in ms]}
    # warm-up on the first frames, then the timed pass over the whole stream
    for f in range(min(args.warmup, nfr)):
        (cold if f == 0 else warm)(ctx, f)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(nfr)]
    labels_kept = {}
    t1 = time.perf_counter()
    for f in range(nfr):
        ev[f][0].record(stream)
        (cold if f == 0 else warm)(ctx, f)
        ev[f][1].record(stream)
        if f < 2:
            labels_kept[f] = out.clone()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    lat = [a.elapsed_time(b) for a, b in ev]
    p50, p99 = _percentiles(lat[1:])
    # refine alone on warm frames, for the per-launch duration of the pixel phases
    reps = max(5, min(30, nfr - 1))
    r = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
         for _ in range(reps)]
    for i in range(reps):
        S.seeds_warm_start(ctx, frames[1 + i % (nfr - 1)], stream)
        r[i][0].record(stream)
        S.seeds_refine(ctx, stream)
        r[i][1].record(stream)
    torch.cuda.synchronize()
    refine_ms = sum(a.elapsed_time(b) for a, b in r) / reps
    # the same frames each refined from scratch (the whole hierarchy)
    cold_reps = min(20, nfr)
    c = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
         for _ in range(cold_reps)]
    for i in range(cold_reps):
        c[i][0].record(stream)
        cold(ctx, i)
        c[i][1].record(stream)
    torch.cuda.synchronize()
    cold_p50, _ = _percentiles([a.elapsed_time(b) for a, b in c])
    S.seeds_sync(ctx, stream)
    S.seeds_destroy(ctx)
    labels_kept = {f: t.cpu().numpy() for f, t in labels_kept.items()}

    launches = ITERS * 9
    per_launch = sum(phase_bytes(SH, SW, 0, cl) for cl in range(9)) / 9
    phase_us = refine_ms * 1e3 / launches
    achieved = per_launch / (phase_us * 1e-6) / 1e9
    npx = SH * SW
    result = {
        "metric": METRIC, "value": round(npx * nfr / wall / 1e6, 2), "unit": "Mpixel/s",
        "n_gpus": 1, "steps": nfr, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / nfr, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"stream of {nfr} frames 3840x2160 RGB u8: 1500-region Voronoi "
                               "scene translated 2 px/frame, fresh noise sigma 8 per frame "
                               "(scene seed 4, noise seeds 4000+f); K=5000 (4982 on the grid), "
                               "4 levels, 5 bins/channel, 4 sweeps/level, gamma 1, Prop. 1 rule; "
                               "frame 0 full hierarchy, later frames warm-started (labels kept, "
                               "re-binned, recounted, 4 pixel sweeps)",
                   "H": SH, "W": SW, "K": SK, "K_eff": keff, "frames": nfr,
                   "step": "one frame: warm start + refine + labels (device)"},
        "p50_ms": round(p50, 4), "p99_ms": round(p99, 4),
        "frame0_ms": round(lat[0], 4), "frames_per_s": round(nfr / wall, 1), "tuning": tuning,
        "cold_per_frame_p50_ms": round(cold_p50, 4),
        "frame_generation_s": round(gen_s, 1),
        "roofline": {"bound": "hbm", "kernel": "k_phase (pixel-level phase of one 4K frame)",
                     "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 6),
                     "traffic": measured_traffic(STREAM_TRAFFIC_FILE),
                     "algorithmic_bytes_per_launch": int(per_launch),
                     "launches_per_frame": launches, "avg_launch_us": round(phase_us, 3),
                     "refine_ms": round(refine_ms, 4)},
    }
    if not args.no_cpu_baseline:
        import oracle
        t2 = time.perf_counter()
        o = oracle.Oracle(host[0], SK, LEVELS, BINS, ITERS, GAMMA, RULE)
        o.run(-1)
        same = bool(np.array_equal(o.labels(), labels_kept[0]))
        t_cold = time.perf_counter() - t2
        o.warm_start(host[1])
        o.run(-1)
        same &= bool(np.array_equal(o.labels(), labels_kept[1]))
        cpu_s = time.perf_counter() - t2
        result["cpu_baseline"] = {
            "value": round(2 * npx / cpu_s / 1e6, 3), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": f"frames 0 (full hierarchy, {t_cold:.1f} s) and 1 (warm start, "
                      f"{cpu_s - t_cold:.1f} s) of the stream, single-threaded C oracle"}
        result["bitexact_vs_oracle"] = same
    print(json.dumps(result), flush=True)
    return 0


def run_quality(args) -> int:
    import numpy as np
    import torch

    from paper_1309_3848_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=True)
    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    QH, QW, QK, QR, n = 321, 481, 200, 30, 20
    pairs = [synth.voronoi_image(QH, QW, QR, 8.0, sd, return_regions=True) for sd in range(1, n + 1)]
    rgbs = [torch.from_numpy(im).to(dev) for im, _ in pairs]
    truths = [torch.from_numpy(reg).to(dev) for _, reg in pairs]
    stream = torch.cuda.current_stream()
    outs = [torch.empty((QH, QW), dtype=torch.int32, device=dev) for _ in range(n)]
    methods = {"grid": (3, 0), "sph": (1, -1), "seeds": (3, -1)}   # (levels, phases)
    quality, labels_of, timing, keff_of = {}, {}, {}, {}
    for name, (L, phases) in methods.items():
        ctx = S.seeds_batch_init(rgbs, QK, S.make_params(L, BINS, ITERS, GAMMA, RULE),
                                 levels=L, stream=stream)

        def step():
            S.seeds_batch_reinit(ctx, rgbs, stream)
            if phases < 0:
                S.seeds_refine(ctx, stream)
            for i in range(n):
                S.seeds_batch_labels(ctx, i, outs[i], stream)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        timing[name] = e0.elapsed_time(e1) / args.steps
        keff = keff_of[name] = S.seeds_batch_num_superpixels(ctx, 0)
        S.seeds_destroy(ctx)
        qs = [S.seeds_quality_metrics(outs[i], truths[i], keff, QR, 2, stream) for i in range(n)]
        labels_of[name] = [o.cpu().numpy() for o in outs]
        quality[name] = {
            "UE": round(float(np.mean([q["ue"] / q["N"] for q in qs])), 5),
            "CUE": round(float(np.mean([q["cue"] / q["N"] for q in qs])), 5),
            "ASA": round(float(np.mean([q["asa"] / q["N"] for q in qs])), 5),
            "BR_eps2": round(float(np.mean([q["br_hits"] / q["br_total"] for q in qs])), 5),
        }
    # the metric kernels themselves, on the SEEDS labels
    lab_dev = [torch.from_numpy(l).to(dev) for l in labels_of["seeds"]]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        for i in range(n):
            S.seeds_quality_metrics(lab_dev[i], truths[i], keff_of["seeds"], QR, 2, stream)
    metric_ms = (time.perf_counter() - t0) * 1e3 / (reps * n)
    npx = QH * QW * n
    result = {
        "metric": METRIC, "value": round(npx / (timing["seeds"] * 1e-3) / 1e6, 2),
        "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(timing["seeds"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{n} images 481x321 RGB u8 (30 Voronoi regions, noise sigma 8, "
                               "seeds 1-20) with their Voronoi region maps as ground truth; "
                               "K=200, 5 bins, 4 sweeps, gamma 1, Prop. 1 rule; one batch context "
                               "per method; metrics of Sec. 6.1 on the device (BR with eps 2)",
                   "methods": {"grid": "initial grid, no refinement (3 levels)",
                               "sph": "pixel-level updates only (1 level)",
                               "seeds": "3 levels (block sides 4, 2, then pixels)"},
                   "step": "batch reinit + refine + labels of 20 images (device)"},
        "quality": quality,
        "ms_per_batch": {k: round(v, 4) for k, v in timing.items()},
        "metric_call_ms": round(metric_ms, 4),
    }
    if not args.no_cpu_baseline:
        import oracle
        t2 = time.perf_counter()
        same, done = True, 0
        while done < n and (done < 3 or time.perf_counter() - t2 < args.cpu_seconds):
            i = done
            ref, _, _ = oracle.seeds(pairs[i][0], QK, 3, BINS, ITERS, GAMMA, RULE)
            same &= bool(np.array_equal(ref, labels_of["seeds"][i]))
            q_cpu = oracle.quality(ref, pairs[i][1], keff_of["seeds"], QR, 2)
            q_gpu = S.seeds_quality_metrics(lab_dev[i], truths[i], keff_of["seeds"], QR, 2, stream)
            same &= q_cpu == q_gpu
            done += 1
        cpu_s = time.perf_counter() - t2
        result["cpu_baseline"] = {
            "value": round(done * QH * QW / cpu_s / 1e6, 3), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": f"images 1-{done}: full oracle runs (3 levels) and oracle metrics, "
                      f"single-threaded C oracle, {cpu_s:.1f} s"}
        result["bitexact_vs_oracle"] = same
    print(json.dumps(result), flush=True)
    return 0


def run_serve(args) -> int:
    import numpy as np
    import torch

    from paper_1309_3848_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=True)
    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rate, n_warm, n_timed = args.rate, args.warm_requests, args.requests
    classes = [(480, 640, 0.70, 24), (1080, 1920, 0.25, 8), (2160, 3840, 0.05, 2)]
    # a pool of distinct images per size (results depend only on the image,
    # so requests reuse them); region counts scale with the area
    pool, pool_np = [], []
    for ci, (H, W, _, cnt) in enumerate(classes):
        imgs = [synth.voronoi_image(H, W, max(30, H * W // 5500), 8.0, 5000 + 100 * ci + j)
                for j in range(cnt)]
        pool_np.append(imgs)
        pool.append([torch.from_numpy(im).to(dev) for im in imgs])
    # the request trace: Poisson arrivals, size class by its share
    rng = np.random.Generator(np.random.PCG64(5))
    total = n_warm + n_timed
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=total))
    cls_of = rng.choice(len(classes), size=total, p=[c[2] for c in classes])
    pick = [int(rng.integers(0, classes[c][3])) for c in cls_of]
    K_of = [classes[c][0] * classes[c][1] // 2000 for c in cls_of]
    # pinned host outputs, reused once a request is reported
    free_out = [[torch.empty((H, W), dtype=torch.int32, pin_memory=True) for _ in range(n)]
                for (H, W, _, _), n in zip(classes, (192, 96, 24))]
    stream = torch.cuda.current_stream()
    params = S.seeds_server_default_params()
    params.iters_per_level, params.max_levels = ITERS, LEVELS
    params.hbm_budget_bytes, params.max_inflight = args.budget_gib << 30, 1024
    srv = S.seeds_server_create(params, stream)
    done_at = np.full(total, np.nan)
    owner, out_of = {}, {}
    kept = {}
    nxt, completed = 0, 0
    t0 = time.perf_counter()
    while completed < total:
        now = time.perf_counter() - t0
        while nxt < total and arrivals[nxt] <= now:
            c = cls_of[nxt]
            if not free_out[c]:
                break
            out = free_out[c].pop()
            rid = S.seeds_server_submit(srv, pool[c][pick[nxt]], K_of[nxt], LEVELS, out)
            owner[rid], out_of[rid] = nxt, out
            nxt += 1
        pending = S.seeds_server_step(srv) if (owner or nxt < total) else 0
        for rid in S.seeds_server_poll(srv):
            i = owner.pop(rid)
            done_at[i] = time.perf_counter() - t0
            out = out_of.pop(rid)
            if len(kept) < 12 and cls_of[i] == 0 and pick[i] not in kept:
                kept[pick[i]] = out.clone()       # a few results for the checks below
            free_out[cls_of[i]].append(out)
            completed += 1
        if pending == 0 and nxt < total and not owner:
            wait = arrivals[nxt] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001))
    stats = S.seeds_server_get_stats(srv)
    S.seeds_server_destroy(srv)
    lat = (done_at - arrivals)[n_warm:] * 1e3
    px = np.array([classes[c][0] * classes[c][1] for c in cls_of])
    span = done_at[n_warm:].max() - arrivals[n_warm]
    served_mpx = px[n_warm:].sum() / span / 1e6
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    # the plain path on the same requests: single-image contexts one after
    # another; its latency under the same arrivals follows from a FIFO queue
    ctxs = {}
    outs_dev = [torch.empty((H, W), dtype=torch.int32, device=dev) for (H, W, _, _) in classes]
    for c, (H, W, _, cnt) in enumerate(classes):
        for j in range(cnt):
            ctxs[c, j] = S.seeds_init(pool[c][j], H * W // 2000,
                                      S.make_params(LEVELS, BINS, ITERS, GAMMA, RULE), stream)
    def plain(i):
        c, j = cls_of[i], pick[i]
        S.seeds_reinit(ctxs[c, j], pool[c][j], stream)
        S.seeds_refine(ctxs[c, j], stream)
        S.seeds_labels(ctxs[c, j], outs_dev[c], stream)
    for i in range(min(50, total)):
        plain(i)
    torch.cuda.synchronize()
    service = {}
    for c in range(len(classes)):
        idx = [i for i in range(n_warm, total) if cls_of[i] == c][:40]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in idx:
            plain(i)
        e1.record(stream)
        torch.cuda.synchronize()
        service[c] = e0.elapsed_time(e1) / max(1, len(idx)) / 1e3
    plain_same = True
    for j, lab in kept.items():
        S.seeds_reinit(ctxs[0, j], pool[0][j], stream)
        S.seeds_refine(ctxs[0, j], stream)
        S.seeds_labels(ctxs[0, j], outs_dev[0], stream)
        plain_same &= bool(torch.equal(outs_dev[0].cpu(), lab))
    for cx in ctxs.values():
        S.seeds_destroy(cx)
    finish, plain_lat = 0.0, []
    for i in range(total):
        finish = max(finish, arrivals[i]) + service[cls_of[i]]
        if i >= n_warm:
            plain_lat.append((finish - arrivals[i]) * 1e3)
    plain_span = finish - arrivals[n_warm]
    result = {
        "metric": METRIC, "value": round(served_mpx, 2), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": n_timed, "warmup": n_warm, "ms_per_step": round(span * 1e3 / n_timed, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals at {rate:g} req/s of RGB u8 images, "
                               "70% 640x480, 25% 1920x1080, 5% 3840x2160 (Voronoi + gradient + "
                               "noise sigma 8; a pool of 24/8/2 distinct images per size); "
                               "K = pixels/2000, 4 levels, 5 bins, 4 sweeps, gamma 1, Prop. 1 "
                               "rule; labels to pinned host memory; continuous batching server "
                               f"with a {args.budget_gib} GiB budget",
                   "rate_req_s": rate, "offered_mpx_s": round(float(px.mean()) * rate / 1e6, 1),
                   "requests_timed": n_timed, "requests_warmup": n_warm,
                   "step": "one request, arrival to labels in host memory"},
        "p50_ms": round(p50, 3), "p99_ms": round(p99, 3),
        "server": {"ticks": stats["ticks"], "peak_inflight": stats["peak_inflight"],
                   "peak_bytes_in_use": stats["peak_bytes_in_use"]},
        "plain_path": {"value": round(px[n_warm:].sum() / plain_span / 1e6, 2),
                       "unit": "Mpixel/s", "p50_ms": round(float(np.percentile(plain_lat, 50)), 3),
                       "p99_ms": round(float(np.percentile(plain_lat, 99)), 3),
                       "service_ms": {f"{classes[c][1]}x{classes[c][0]}": round(v * 1e3, 3)
                                      for c, v in service.items()},
                       "note": "single-image contexts back to back; latency from a FIFO queue "
                               "over the same arrivals and measured service times",
                       "labels_equal_to_served": plain_same},
    }
    if not args.no_cpu_baseline:
        import oracle
        t2 = time.perf_counter()
        same, used = True, 0
        for j, lab in kept.items():
            if used >= 2 and time.perf_counter() - t2 >= args.cpu_seconds:
                break
            ref, _, _ = oracle.seeds(pool_np[0][j], 480 * 640 // 2000, LEVELS, BINS, ITERS,
                                     GAMMA, RULE)
            same &= bool(np.array_equal(ref, lab.numpy()))
            used += 1
        cpu_s = time.perf_counter() - t2
        result["cpu_baseline"] = {
            "value": round(used * 480 * 640 / cpu_s / 1e6, 3), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{used} served 640x480 requests recomputed by the single-threaded C "
                      f"oracle, {cpu_s:.1f} s"}
        result["bitexact_vs_oracle"] = same
    print(json.dumps(result), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: requests per second")
    ap.add_argument("--requests", type=int, default=4000, help="serve: timed requests")
    ap.add_argument("--warm-requests", type=int, default=500, help="serve: warm-up requests")
    ap.add_argument("--budget-gib", type=int, default=8, help="serve: server memory budget")
    ap.add_argument("--workload", choices=["single1080p", "batch64", "stream4k", "quality", "serve"],
                    default="single1080p")
    ap.add_argument("--frames", type=int, default=300, help="stream4k: frames of the stream")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch mapping instead of timing the four settings "
                         "(seeds_autotune) before the warm-up")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 64 MiB device-to-device copy (a known amount of HBM "
                         "traffic for scaling profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(images are independent: several GPUs would each refine their own images)", file=sys.stderr)
        return 2
    if args.workload == "serve":
        args.steps = args.requests if args.steps is None else args.steps
        args.warmup = args.warm_requests if args.warmup is None else args.warmup
        return run_serve(args)
    if args.workload == "quality":
        args.steps = 20 if args.steps is None else args.steps
        args.warmup = 3 if args.warmup is None else args.warmup
        return run_quality(args)
    if args.workload == "stream4k":
        args.warmup = 3 if args.warmup is None else args.warmup
        return run_stream(args)
    if args.workload == "batch64":
        args.steps = 20 if args.steps is None else args.steps
        args.warmup = 3 if args.warmup is None else args.warmup
        return run_batch(args)
    args.steps = 200 if args.steps is None else args.steps
    args.warmup = 20 if args.warmup is None else args.warmup

    import numpy as np
    import torch

    from paper_1309_3848_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=True)
    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    img = synth.single_1080p()
    rgb = torch.from_numpy(img).to(dev)
    out = torch.empty((H, W), dtype=torch.int32, device=dev)
    params = S.make_params(LEVELS, BINS, ITERS, GAMMA, RULE)
    stream = torch.cuda.current_stream()
    ctx = S.seeds_init(rgb, K, params, stream)
    keff = S.seeds_num_superpixels(ctx)
    tuning = None
    if not args.no_autotune:
        chosen, ms = S.seeds_autotune(ctx, 5, stream)
        tuning = {"chosen": chosen, "refine_ms_per_variant": [round(m, 4) for m in ms]}

    def step():
        S.seeds_reinit(ctx, rgb, stream)
        S.seeds_refine(ctx, stream)
        S.seeds_labels(ctx, out, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    p50, p99 = _percentiles([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ms_per_step = wall * 1e3 / args.steps
    mpx = H * W * args.steps / wall / 1e6

    # refine launch alone, timed with events on the stream it runs on
    reps = max(10, args.steps // 4)
    r0 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    r1 = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    for i in range(reps):
        S.seeds_reinit(ctx, rgb, stream)
        r0[i].record(stream)
        S.seeds_refine(ctx, stream)
        r1[i].record(stream)
    S.seeds_labels(ctx, out, stream)
    torch.cuda.synchronize()
    refine_ms = sum(a.elapsed_time(b) for a, b in zip(r0, r1)) / reps
    launches, refine_bytes, init_bytes, out_bytes = schedule_bytes(H, W, LEVELS, ITERS)
    # the refine call is the phase launches plus 3 level transitions and one
    # final replay (about 2% of its time): charging it all to the phase
    # kernel keeps the per-launch duration an upper bound
    phase_us = refine_ms * 1e3 / launches
    per_launch = refine_bytes / launches
    achieved = per_launch / (phase_us * 1e-6) / 1e9
    traffic = measured_traffic()
    lds = measured_lds()
    lds_atomics = None
    if lds is not None:
        per = lds["lds_atomic_insts_per_launch"]
        rate = per / (phase_us * 1e-6) / 1e9
        lds_atomics = {"achieved": round(rate, 3), "peak": LDS_ATOMIC_PEAK_GINST,
                       "unit": "G wavefront-instructions/s", "frac": round(rate / LDS_ATOMIC_PEAK_GINST, 6),
                       "per_launch": per, "bank_conflict_frac": lds["bank_conflict_frac"],
                       "source": "profiles/k_phase_1080p_lds.json (rocprofv3 SQ_INSTS_LDS_ATOMIC)"}
    gpu_labels = out.cpu().numpy()
    S.seeds_destroy(ctx)

    result = {
        "metric": METRIC, "value": round(mpx, 2), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "single 1920x1080 RGB u8 image, 400 Voronoi regions + gradient + "
                               "noise sigma 8 (seed 2); K=1000 (1008 on the grid), 4 levels, "
                               "5 bins/channel, 4 sweeps/level, gamma 1, Prop. 1 block rule",
                   "H": H, "W": W, "K": K, "K_eff": keff, "levels": LEVELS, "bins": BINS,
                   "iters": ITERS, "gamma": GAMMA, "block_rule": "intersect",
                   "step": "reinit + refine + labels (device)"},
        "p50_ms": round(p50, 4), "p99_ms": round(p99, 4), "tuning": tuning,
        "hbm_frac_step": round((refine_bytes + init_bytes + out_bytes) / (ms_per_step * 1e-3)
                               / 1e9 / HBM_PEAK_GBS, 6),
        "algorithmic_bytes_per_step": int(refine_bytes + init_bytes + out_bytes),
        "roofline": {"bound": "hbm", "kernel": "k_phase (one phase of the schedule per launch; block-level and pixel-level variants)",
                     "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
                     "algorithmic_bytes_per_launch": int(per_launch),
                     "launches_per_image": launches, "avg_launch_us": round(phase_us, 3),
                     "refine_ms": round(refine_ms, 4)},
        "lds_atomics": lds_atomics,
    }

    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        n = 0
        ref = None
        while True:
            ref, _, _ = oracle.seeds(img, K, LEVELS, BINS, ITERS, GAMMA, RULE)
            n += 1
            if time.perf_counter() - t1 >= args.cpu_seconds or n >= 20:
                break
        cpu_s = time.perf_counter() - t1
        result["cpu_baseline"] = {
            "value": round(H * W * n / cpu_s / 1e6, 3), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n} full runs of the same 1920x1080 image (quantise+grid+refine), "
                      f"single-threaded C oracle, {cpu_s:.1f} s",
        }
        result["bitexact_vs_oracle"] = bool(np.array_equal(gpu_labels, ref))
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
