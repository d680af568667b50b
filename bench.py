"""Benchmark: SEEDS refinement throughput on one MI355X.

The default run prints one JSON line. Its headline (`value`, `ms_per_step`,
`roofline`, `cpu_baseline`) is the single 1920 x 1080 image: a step is the
whole hot path for the image already resident in HBM - re-initialise the
context from the image (quantise, grid, colour histograms), run the full
refinement schedule (all block levels, then pixel level) and write the labels
to a device buffer. Workload: 400 Voronoi regions + gradient + Gaussian noise
sigma 8, K = 1000 requested (1008 on the grid), 4 levels, 5 bins per channel,
4 sweeps per level, gamma 1, Prop. 1 block rule.

The same line nests the other workloads under `workloads`, each measured in
this run with its own step counts, roofline and CPU baseline:
  c1_481x321  the small single image (481 x 321, K 200, 3 levels);
  batch64     64 mixed images in one batch context (one launch per phase for
              all images), against the same images through single-image
              contexts one after another (the plain path);
  stream4k    300 frames of 3840 x 2160, frame 0 from scratch, later frames
              warm-started (labels kept, re-binned, recounted, 4 pixel sweeps);
  serve       Poisson arrivals at 2000 requests/s (70% 640x480, 25% 1080p, 5%
              4K) through the continuous-batching server, against the plain
              path under the same arrivals; latency from arrival to labels in
              host memory.
`--workload NAME` runs one of them alone (or `quality`: the metrics of
Sec. 6.1 for the grid, pixel-only updates and SEEDS; `single4k`: the 4K
stream's first frame as a single image refined from scratch, K 5000, a size
at which the block phases can be profiled; `traffic_probe`: the 64 MiB
calibration copy and the library's traffic probes, kernels of known traffic
for reading profiler byte counters) and prints its line.

Roofline. `roofline.achieved` is the algorithmic bytes of one k_phase launch
over the launch's average duration. Algorithmic bytes follow the byte model
of the method: per sweep of a level, its unit-label plane once (4 B per unit)
plus the colour bins of the boundary units (1 B per pixel they cover; only
those are proposed, Sec. 5.2), plus 4 B per moved unit where counted. The
boundary units of every phase are counted on the device (seeds_boundary_units)
in an untimed pass over the same schedule. The duration is the event-timed
refine call divided by its phase launches (level transitions and the final
replay included, so the rate is a lower bound). `structural_bytes_per_launch`
is what a launch reads by construction: the whole label plane of its level
(every class's 5 x 5 windows or 3 x 3 rings cover it) plus its class's bins.

CPU baseline. The plain C oracle, single-threaded (median of 5 runs where a
run takes seconds, else a bounded sample), and its OpenMP build (the units of
a phase decided in parallel, identical results) on all host cores; the host's
core count and CPU model are recorded. The paper's own figure (30 Hz on one
core of a 2.8 GHz i7 at 481 x 321) is given as context.
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
PAPER_CONTEXT = {
    "value": round(481 * 321 * 30 / 1e6, 2), "unit": "Mpixel/s",
    "what": "the paper's real-time claim (Sec. 6): 30 Hz on 481x321 images on one core of an "
            "Intel i7 at 2.8 GHz (LAB colour, random proposals, another machine: context only)"}


# ---- byte model ---------------------------------------------------------------

def units_of(h: int, w: int, level: int):
    s = 1 << level
    return -(-w // s), -(-h // s)


def class_units(uw: int, uh: int, cls: int) -> int:
    cw = (uw - cls % 3 + 2) // 3 if cls % 3 < uw else 0
    ch = (uh - cls // 3 + 2) // 3 if cls // 3 < uh else 0
    return cw * ch


def structural_phase_bytes(h: int, w: int, level: int, cls: int, lab_bytes: float = 4.0) -> float:
    """What one phase launch reads by construction: the whole unit-label plane
    of its level and the bins of its class's units."""
    uw, uh = units_of(h, w, level)
    return lab_bytes * uw * uh + 1.0 * class_units(uw, uh, cls) * (1 << level) ** 2


def fixed_bytes(h: int, w: int, levels: int, lab_bytes: float = 2.0):
    """(init, materialised pixel labels, output) bytes of one image: RGB read +
    bins write + top-block labels; the pixel-label plane written once (2 B per
    pixel in 16 bits); 4 B per pixel of int32 output."""
    n = h * w
    tw, th = units_of(h, w, levels - 1)
    return (3.0 * n + 1.0 * n + 4.0 * tw * th, (lab_bytes * n if levels > 1 else 0.0), 4.0 * n)


def schedule_profile(S, ctx, dims, levels_walk, iters, moves=False, energy=False, stream=None):
    """Walk the next phases of ctx one at a time (untimed) and count, on the
    device, the boundary units of every phase of every image taking part.

    dims: per image (H, W, L); levels_walk: the levels the schedule visits
    (each I sweeps of 9 classes). With `moves` the labels before and after each
    phase are compared (moved pixels / s^2 = moved units); with `energy` H' and
    G' are read after each level (single images). Returns the per-launch
    algorithmic and structural bytes and per-level figures."""
    import torch
    n = len(dims)
    dev = torch.device("cuda:0")
    # pixel labels are stored in 16 bits up to 65535 superpixels (the library's
    # choice for the whole context); block grids in 32
    lab16 = all(S.seeds_batch_num_superpixels(ctx, i) <= 65535 for i in range(n))
    labs = [torch.empty((h, w), dtype=torch.int32, device=dev) for h, w, _ in dims] if moves else None
    before = None
    total, struct, launches = 0.0, 0.0, 0
    per_level = []
    for lvl in levels_walk:
        side = 1 << lvl
        rec = {"side": side, "phases": 0, "boundary_pixels": 0, "pixels": 0, "moved_units": 0,
               "bytes": 0.0}
        part = [i for i, (_, _, L) in enumerate(dims) if L - 1 >= lvl]
        for _ in range(iters):
            for cls in range(9):
                b = S.seeds_boundary_units(ctx, cls, lvl, stream)
                if moves:
                    before = []
                    for i in part:
                        S.seeds_batch_labels(ctx, i, labs[i], stream)
                        before.append(labs[i].clone())
                S.seeds_refine_phases(ctx, 1, stream)
                launches += 1
                rec["phases"] += 1
                for q, i in enumerate(part):
                    h, w, _ = dims[i]
                    uw, uh = units_of(h, w, lvl)
                    mv = 0.0
                    if moves:
                        S.seeds_batch_labels(ctx, i, labs[i], stream)
                        mv = float((labs[i] != before[q]).sum().item()) / (side * side)
                        rec["moved_units"] += mv
                    lb = 2.0 if (lvl == 0 and lab16) else 4.0
                    total += lb * uw * uh / 9.0 + b[i][1] + lb * mv
                    rec["bytes"] += lb * uw * uh / 9.0 + b[i][1] + lb * mv
                    struct += structural_phase_bytes(h, w, lvl, cls, lb)
                    rec["boundary_pixels"] += b[i][1]
        rec["pixels"] = sum(dims[i][0] * dims[i][1] for i in part)
        # boundary fraction per sweep: pixels of boundary units over all pixels
        rec["beta"] = round(rec["boundary_pixels"] / max(1, rec["pixels"] * iters), 4)
        if energy and n == 1:
            h_e, g_e = S.seeds_energy(ctx, stream)
            rec["H_prime"], rec["G_prime"] = h_e, g_e
            rec["E_prime"] = h_e + (GAMMA * g_e if lvl == 0 else 0)
        rec["moved_units"] = round(rec["moved_units"]) if moves else None
        rec["algorithmic_bytes_per_launch"] = int(rec.pop("bytes") / max(1, rec["phases"]))
        per_level.append(rec)
    torch.cuda.synchronize()
    return {"launches": launches, "bytes": total, "bytes_per_launch": total / max(1, launches),
            "structural_bytes_per_launch": struct / max(1, launches), "levels": per_level,
            "pixel_label_bytes": 2 if lab16 else 4}


def roofline(kernel, prof, avg_launch_us, traffic=None):
    if prof is None:   # --skip-byte-pass (profiler runs): no boundary counts
        return {"bound": "hbm", "kernel": kernel, "achieved": None, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": None, "traffic": traffic,
                "avg_launch_us": round(avg_launch_us, 3), "note": "byte pass skipped"}
    achieved = prof["bytes_per_launch"] / (avg_launch_us * 1e-6) / 1e9
    st_achieved = prof["structural_bytes_per_launch"] / (avg_launch_us * 1e-6) / 1e9
    r = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
         "algorithmic_bytes_per_launch": int(prof["bytes_per_launch"]),
         "avg_launch_us": round(avg_launch_us, 3),
         "duration": "event-timed refine call / phase launches (level transitions and the "
                     "final replay included)",
         "structural_bytes_per_launch": int(prof["structural_bytes_per_launch"]),
         "structural_frac": round(st_achieved / HBM_PEAK_GBS, 6),
         "per_level": [{k: v for k, v in rec.items() if k not in ("pixels",)}
                       for rec in prof["levels"]]}
    if traffic:
        r["traffic_over_algorithmic"] = round(traffic / prof["bytes_per_launch"], 2)
        r["traffic_over_structural"] = round(traffic / prof["structural_bytes_per_launch"], 2)
    return r


# ---- measured traffic and LDS counters from committed profiles -----------------

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_phase_1080p_traffic.json")
STREAM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_phase_stream4k_traffic.json")
LDS_FILE = os.path.join(ROOT, "profiles", "k_phase_1080p_lds.json")
KERNEL_SOURCES = ["seeds_phase.h", "seeds_phase.hip", "seeds_device.h", "seeds_internal.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1309_3848_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile_json(path):
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    return t if t.get("kernel_source_sha256") == kernel_source_hash() else None


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per phase launch from the committed rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs, or None when the kernel sources changed since."""
    t = _profile_json(path)
    return t.get("traffic_bytes_per_launch") if t else None


def _percentiles(lat):
    lat = sorted(lat)
    return lat[len(lat) // 2], lat[min(len(lat) - 1, int(round(0.99 * (len(lat) - 1))))]


# ---- CPU baseline ----------------------------------------------------------------

def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"nproc": nproc, "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def cpu_single(img, k, levels, budget_s, want=None):
    """Oracle on one image: median of 5 serial runs (fewer if one run exceeds
    the budget) and median of 5 all-core runs. want: GPU labels to compare."""
    import numpy as np

    import oracle
    npx = img.shape[0] * img.shape[1]
    omp = oracle.lib_omp()
    out = {}
    for name, cdll in (("serial", None), ("all_cores", omp)):
        times, same = [], True
        while len(times) < 5:
            t0 = time.perf_counter()
            ref, _, _ = oracle.seeds(img, k, levels, BINS, ITERS, GAMMA, RULE, cdll=cdll)
            times.append(time.perf_counter() - t0)
            if want is not None:
                same &= bool(np.array_equal(ref, want))
            if sum(times) > budget_s:
                break
        out[name] = (times, same)
    ts, same_s = out["serial"]
    ta, same_a = out["all_cores"]
    return {
        "value": round(npx / _median(ts) / 1e6, 3), "unit": "Mpixel/s", "cores": 1,
        "kind": "oracle",
        "sample": f"median of {len(ts)} full runs (quantise+grid+refine) of the {img.shape[1]}x"
                  f"{img.shape[0]} image, single-threaded C oracle ({_median(ts):.3f} s per run)",
        "all_cores": {"value": round(npx / _median(ta) / 1e6, 3), "unit": "Mpixel/s",
                      "cores": omp.oracle_threads(), "kind": "oracle (OpenMP build)",
                      "sample": f"median of {len(ta)} full runs ({_median(ta):.3f} s per run)"},
        "host": host_info(), "paper_context": PAPER_CONTEXT,
    }, same_s and same_a


# ---- single image (C1, C2) -------------------------------------------------------

def run_single(args, img, k, levels, name, steps, warmup, traffic_file=None, lds_file=None):
    import numpy as np
    import torch

    from paper_1309_3848_amd import seeds as S

    dev = torch.device("cuda:0")
    h, w, _ = img.shape
    rgb = torch.from_numpy(img).to(dev)
    out = torch.empty((h, w), dtype=torch.int32, device=dev)
    params = S.make_params(levels, BINS, ITERS, GAMMA, RULE)
    stream = torch.cuda.current_stream()
    ctx = S.seeds_init(rgb, k, params, stream)
    keff = S.seeds_num_superpixels(ctx)
    tuning = apply_tuning(S, ctx, args)
    if tuning is None and not args.no_autotune:
        chosen, ms = S.seeds_autotune(ctx, 5, stream)
        tuning = {"chosen": chosen, "ms_per_variant": [round(m, 4) for m in ms]}

    def step():
        S.seeds_reinit(ctx, rgb, stream)
        S.seeds_refine(ctx, stream)
        S.seeds_labels(ctx, out, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    p50, p99 = _percentiles([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ms_per_step = wall * 1e3 / steps

    # refine call alone, timed with events on the stream it runs on
    reps = max(10, steps // 4)
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
    gpu_labels = out.cpu().numpy()
    # untimed pass: boundary units, moves and energies of every phase
    prof = None
    if not args.skip_byte_pass:
        S.seeds_reinit(ctx, rgb, stream)
        prof = schedule_profile(S, ctx, [(h, w, levels)], list(range(levels - 1, -1, -1)), ITERS,
                                moves=True, energy=True, stream=stream)
    if args.copy_calibration:
        # a known amount of traffic for scaling profiler byte counters
        src = torch.empty(64 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    S.seeds_destroy(ctx)
    launches = levels * ITERS * 9
    avg_us = refine_ms * 1e3 / launches
    init_b, mat_b, out_b = fixed_bytes(h, w, levels)
    step_bytes = init_b + (prof["bytes"] if prof else 0.0) + mat_b + out_b
    traffic = measured_traffic(traffic_file) if traffic_file else None
    result = {
        "metric": METRIC, "value": round(h * w * steps / wall / 1e6, 2), "unit": "Mpixel/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": name, "H": h, "W": w, "K": k, "K_eff": keff, "levels": levels,
                   "bins": BINS, "iters": ITERS, "gamma": GAMMA, "block_rule": "intersect",
                   "step": "reinit + refine + labels (device)"},
        "p50_ms": round(p50, 4), "p99_ms": round(p99, 4), "tuning": tuning,
        "refine_ms": round(refine_ms, 4), "launches_per_image": launches,
        "algorithmic_bytes_per_step": int(step_bytes) if prof else None,
        "algorithmic_bytes_per_pixel": round(step_bytes / (h * w), 2) if prof else None,
        "hbm_frac_step": (round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 6)
                          if prof else None),
        "roofline": roofline("k_phase (one phase of the schedule per launch; block-level and "
                             "pixel-level variants)", prof, avg_us, traffic),
    }
    if lds_file:
        lds = _profile_json(lds_file)
        if lds is not None:
            per = lds["lds_atomic_insts_per_launch"]
            rate = per / (avg_us * 1e-6) / 1e9
            result["lds_atomics"] = {"achieved": round(rate, 3), "unit": "G wavefront-instructions/s",
                                     "per_launch": per, "bank_conflict_frac": lds["bank_conflict_frac"],
                                     "source": os.path.relpath(lds_file, ROOT)}
    if not args.no_cpu_baseline:
        cb, same = cpu_single(img, k, levels, args.cpu_seconds, gpu_labels)
        result["cpu_baseline"] = cb
        result["bitexact_vs_oracle"] = same
    return result


def apply_tuning(S, ctx, args):
    """--tuning c,r,items,init_rows,warm_rows[,block_ppl]: set that mapping (no
    autotuning)."""
    if not args.tuning:
        return None
    S.seeds_set_tuning(ctx, *(int(v) for v in args.tuning.split(",")))
    return {"chosen": S.seeds_get_tuning(ctx), "set": True}


def lds_peak(S, result, stream):
    """Measured LDS-atomic throughput (project microbenchmark) as the peak of
    the `lds_atomics` object."""
    la = result.get("lds_atomics")
    if la is None:
        return
    peak = S.seeds_lds_atomic_rate(stream)
    la["peak"] = round(peak, 3)
    la["frac"] = round(la["achieved"] / peak, 6)
    la["peak_source"] = "seeds_lds_atomic_rate: every lane of 4096 workgroups adds to its own " \
                        "LDS word, conflict free (measured live)"


def pixel_tiles(h, w):
    """Workgroups of a class-0 pixel-level launch: tiles of 64 x 4 pixels of one class."""
    return -(-(-(-w // 3)) // 64) * -(-(-(-h // 3)) // 4)


def launch_floor(S, result, h, w, stream, launches=None, groups=None):
    """Latency floor of the image's phase launches (project microbenchmark
    with the same grid and launch count): empty launches, one round of window
    loads, and two dependent rounds plus atomics, against k_phase's average
    launch. A batch passes the sum of its images' tiles as `groups`."""
    rf = result.get("roofline") or {}
    groups = groups or pixel_tiles(h, w)
    launches = launches or result.get("launches_per_image") or 144
    us = S.seeds_launch_floor(groups, launches, stream)
    rf["launch_floor_us"] = {"empty": round(us[0], 3), "one_round_trip": round(us[1], 3),
                             "two_round_trips": round(us[2], 3), "groups": groups,
                             "launches": launches,
                             "source": "seeds_launch_floor (measured live)"}
    if rf.get("avg_launch_us"):
        rf["frac_of_launch_floor"] = round(us[2] / rf["avg_launch_us"], 3)
        if us[2] > rf["avg_launch_us"]:
            rf["launch_floor_us"]["note"] = (
                "the two-round skeleton loads five table cells in every lane and a 7 KB window "
                "per workgroup; here it takes longer than the phase, so it is bound by its own "
                "loads, not by latency, and only the empty launch bounds the phase")


# ---- batch (C3) -------------------------------------------------------------------

def run_batch(args) -> dict:
    import numpy as np
    import torch

    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    dev = torch.device("cuda:0")
    steps, warmup = args.batch_steps, args.batch_warmup
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
    tuning = apply_tuning(S, ctx, args)
    if tuning is None and not args.no_autotune:
        chosen, ms = S.seeds_autotune(ctx, 3, stream)
        tuning = {"chosen": chosen, "ms_per_variant": [round(m, 4) for m in ms]}

    def step():
        S.seeds_batch_reinit(ctx, rgbs, stream)
        S.seeds_refine(ctx, stream)
        S.seeds_batch_labels_all(ctx, outs, stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    p50, p99 = _percentiles([a.elapsed_time(b) for a, b in zip(starts, ends)])
    ms_per_step = wall * 1e3 / steps

    reps = max(5, steps // 2)
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
    gpu_labels = [o.cpu().numpy() for o in outs]
    dims = [(s["H"], s["W"], s["levels"]) for s in specs]
    prof = None
    if not args.skip_byte_pass:
        S.seeds_batch_reinit(ctx, rgbs, stream)
        prof = schedule_profile(S, ctx, dims, list(range(max(Ls) - 1, -1, -1)), ITERS,
                                stream=stream)
    S.seeds_sync(ctx, stream)
    S.seeds_destroy(ctx)

    # the plain path: the same images through single-image contexts, in turn
    solo = [S.seeds_init(r, k, S.make_params(l, BINS, ITERS, GAMMA, RULE), stream)
            for r, k, l in zip(rgbs, Ks, Ls)]

    def solo_step():
        for c, r, o in zip(solo, rgbs, outs):
            S.seeds_reinit(c, r, stream)
            S.seeds_refine(c, stream)
            S.seeds_labels(c, o, stream)

    for _ in range(2):
        solo_step()
    torch.cuda.synchronize()
    solo_steps = max(3, steps // 4)
    t1 = time.perf_counter()
    for _ in range(solo_steps):
        solo_step()
    torch.cuda.synchronize()
    solo_ms = (time.perf_counter() - t1) * 1e3 / solo_steps
    solo_same = all(bool(np.array_equal(o.cpu().numpy(), g)) for o, g in zip(outs, gpu_labels))
    for c in solo:
        S.seeds_destroy(c)

    launches = max(Ls) * ITERS * 9
    avg_us = refine_ms * 1e3 / launches
    fixed = [fixed_bytes(s["H"], s["W"], s["levels"]) for s in specs]
    step_bytes = sum(sum(f) for f in fixed) + (prof["bytes"] if prof else 0.0)
    solo_mpx = npx / (solo_ms * 1e-3) / 1e6
    value = npx * steps / wall / 1e6
    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpixel/s",
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms_per_step, 4),
        "config": {"workload": "batch of 64 mixed RGB u8 images (W 320-1920, H 240-1080, "
                               "50-600 Voronoi regions, noise sigma 4-16, seeds 3000+i); K 200-2000 "
                               "clamped to N/256, 3-4 levels, 5 bins/channel, 4 sweeps/level, "
                               "gamma 1, Prop. 1 block rule; one batch context",
                   "images": len(specs), "megapixels": round(npx / 1e6, 3),
                   "step": "batch reinit + refine + labels of every image (device)"},
        "p50_ms": round(p50, 4), "p99_ms": round(p99, 4),
        "images_per_s": round(len(specs) * steps / wall, 1), "tuning": tuning,
        "refine_ms": round(refine_ms, 4), "launches_per_batch": launches,
        "hbm_frac_step": (round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 6)
                          if prof else None),
        "plain_path": {"ms_per_batch": round(solo_ms, 4), "value": round(solo_mpx, 2),
                       "unit": "Mpixel/s", "labels_equal_to_batch": solo_same,
                       "hbm_frac_step": (round(step_bytes / (solo_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                               6) if prof else None),
                       "speedup_of_batch": round(value / solo_mpx, 2)},
        "roofline": roofline("k_phase (batch variant; one phase of every image per launch)",
                             prof, avg_us, None),
    }
    result["roofline"]["traffic_note"] = "not measured: see the batch profile notes"
    launch_floor(S, result, 0, 0, stream, launches=launches,
                 groups=min(sum(pixel_tiles(s["H"], s["W"]) for s in specs), 65536))
    if not args.no_cpu_baseline:
        import oracle
        order = np.argsort([s["H"] * s["W"] for s in specs])
        # the smallest, median and largest image first, then others in turn
        sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
        sample += [i for i in range(len(specs)) if i not in sample]
        res = {}
        for name, cdll in (("serial", None), ("all_cores", oracle.lib_omp())):
            t2 = time.perf_counter()
            px, same, used = 0, True, []
            for i in sample:
                if len(used) >= 3 and time.perf_counter() - t2 >= args.cpu_seconds:
                    break
                ref, _, _ = oracle.seeds(imgs[i], Ks[i], Ls[i], BINS, ITERS, GAMMA, RULE, cdll=cdll)
                px += imgs[i].shape[0] * imgs[i].shape[1]
                same &= bool(np.array_equal(gpu_labels[i], ref))
                used.append(i)
            res[name] = (px, time.perf_counter() - t2, len(used), same)
        px, cs, nu, same = res["serial"]
        pa, ca, na, same_a = res["all_cores"]
        result["cpu_baseline"] = {
            "value": round(px / cs / 1e6, 3), "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"{nu} images of the batch ({px / 1e6:.1f} Mpx; first the smallest, median "
                      f"and largest), full runs, single-threaded C oracle, {cs:.1f} s",
            "all_cores": {"value": round(pa / ca / 1e6, 3), "unit": "Mpixel/s",
                          "cores": oracle.lib_omp().oracle_threads(),
                          "kind": "oracle (OpenMP build)",
                          "sample": f"{na} images in the same order ({pa / 1e6:.1f} Mpx), {ca:.1f} s"},
            "host": host_info(), "paper_context": PAPER_CONTEXT}
        result["bitexact_vs_oracle"] = same and same_a
    return result


# ---- stream (C4) ------------------------------------------------------------------

def run_stream(args) -> dict:
    import concurrent.futures as cf

    import numpy as np
    import torch

    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    dev = torch.device("cuda:0")
    SH, SW, SK = 2160, 3840, 5000
    nfr = args.frames
    warmup = 3
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
    tuning = apply_tuning(S, ctx, args)
    if tuning is None and not args.no_autotune:
        chosen, ms = S.seeds_autotune(ctx, 3, stream)
        tuning = {"chosen": chosen, "ms_per_variant": [round(m, 4) for m in ms]}
    for f in range(min(warmup, nfr)):
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
    # boundary units of the pixel phases of a warm frame (untimed)
    prof = None
    if not args.skip_byte_pass:
        S.seeds_warm_start(ctx, frames[min(5, nfr - 1)], stream)
        prof = schedule_profile(S, ctx, [(SH, SW, LEVELS)], [0], ITERS, moves=True,
                                stream=stream)
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

    avg_us = refine_ms * 1e3 / (ITERS * 9)
    npx = SH * SW
    result = {
        "metric": METRIC, "value": round(npx * nfr / wall / 1e6, 2), "unit": "Mpixel/s",
        "steps": nfr, "warmup": warmup, "ms_per_step": round(wall * 1e3 / nfr, 4),
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
        "refine_ms": round(refine_ms, 4),
        "roofline": roofline("k_phase (pixel-level phase of one warm 4K frame)", prof, avg_us,
                             measured_traffic(STREAM_TRAFFIC_FILE)),
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
        del o
        # all cores: the first frames of the stream (up to 30) within the budget
        omp = oracle.lib_omp()
        t3 = time.perf_counter()
        o = oracle.Oracle(host[0], SK, LEVELS, BINS, ITERS, GAMMA, RULE, cdll=omp)
        o.run(-1)
        same &= bool(np.array_equal(o.labels(), labels_kept[0]))
        done = 1
        while done < min(30, nfr) and time.perf_counter() - t3 < args.cpu_seconds:
            o.warm_start(host[done])
            o.run(-1)
            if done == 1:
                same &= bool(np.array_equal(o.labels(), labels_kept[1]))
            done += 1
        omp_s = time.perf_counter() - t3
        result["cpu_baseline"] = {
            "value": round(2 * npx / cpu_s / 1e6, 3), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": f"frames 0 (full hierarchy, {t_cold:.1f} s) and 1 (warm start, "
                      f"{cpu_s - t_cold:.1f} s) of the stream, single-threaded C oracle",
            "all_cores": {"value": round(done * npx / omp_s / 1e6, 3), "unit": "Mpixel/s",
                          "cores": omp.oracle_threads(), "kind": "oracle (OpenMP build)",
                          "sample": f"frames 0-{done - 1} of the stream (frame 0 full hierarchy, "
                                    f"then warm starts), {omp_s:.1f} s"},
            "host": host_info(), "paper_context": PAPER_CONTEXT}
        result["bitexact_vs_oracle"] = same
    launch_floor(S, result, SH, SW, stream, launches=ITERS * 9)  # a warm frame's pixel phases
    return result


# ---- serving (C5) -----------------------------------------------------------------

SERVE_CLASSES = [(480, 640, 0.70, 24), (1080, 1920, 0.25, 8), (2160, 3840, 0.05, 2)]


def _serve_trace(rate, total):
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(5))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=total))
    cls_of = rng.choice(len(SERVE_CLASSES), size=total, p=[c[2] for c in SERVE_CLASSES])
    pick = [int(rng.integers(0, SERVE_CLASSES[c][3])) for c in cls_of]
    return arrivals, cls_of, pick


def run_serve(args) -> dict:
    import numpy as np
    import torch

    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    dev = torch.device("cuda:0")
    rate, n_warm, n_timed = args.rate, args.warm_requests, args.requests
    classes = SERVE_CLASSES
    # a pool of distinct images per size (results depend only on the image,
    # so requests reuse them); region counts scale with the area
    pool, pool_np = [], []
    for ci, (h, w, _, cnt) in enumerate(classes):
        imgs = [synth.voronoi_image(h, w, max(30, h * w // 5500), 8.0, 5000 + 100 * ci + j)
                for j in range(cnt)]
        pool_np.append(imgs)
        pool.append([torch.from_numpy(im).to(dev) for im in imgs])
    total = n_warm + n_timed
    arrivals, cls_of, pick = _serve_trace(rate, total)
    K_of = [classes[c][0] * classes[c][1] // 2000 for c in cls_of]
    px = np.array([classes[c][0] * classes[c][1] for c in cls_of])
    stream = torch.cuda.current_stream()

    def pinned_outputs():
        return [[torch.empty((h, w), dtype=torch.int32, pin_memory=True) for _ in range(n)]
                for (h, w, _, _), n in zip(classes, (192, 96, 24))]

    # ---- the server
    free_out = pinned_outputs()
    params = S.seeds_server_default_params()
    params.iters_per_level, params.max_levels = ITERS, LEVELS
    params.hbm_budget_bytes, params.max_inflight = args.budget_gib << 30, 1024
    params.items_per_group = args.serve_items
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
    span = done_at[n_warm:].max() - arrivals[n_warm]
    served_mpx = px[n_warm:].sum() / span / 1e6
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    # ---- the plain path under the same arrivals: one single-image context per
    # pool image, each request re-initialised, refined and its labels copied to
    # its pinned host output in arrival order on one stream; a request
    # completes when an event after its copy has passed
    ctxs = {}
    for c, (h, w, _, cnt) in enumerate(classes):
        for j in range(cnt):
            ctxs[c, j] = S.seeds_init(pool[c][j], h * w // 2000,
                                      S.make_params(LEVELS, BINS, ITERS, GAMMA, RULE), stream)
    outs_dev = [torch.empty((h, w), dtype=torch.int32, device=dev) for (h, w, _, _) in classes]
    free_out = pinned_outputs()

    def plain(i, out):
        c, j = cls_of[i], pick[i]
        S.seeds_reinit(ctxs[c, j], pool[c][j], stream)
        S.seeds_refine(ctxs[c, j], stream)
        S.seeds_labels(ctxs[c, j], outs_dev[c], stream)
        out.copy_(outs_dev[c], non_blocking=True)

    for i in range(min(50, total)):          # capture every context's graph
        plain(i, free_out[cls_of[i]][0])
    torch.cuda.synchronize()
    plain_done = np.full(total, np.nan)
    inflight = []                            # (request, event, output)
    nxt = 0
    t0 = time.perf_counter()
    while nxt < total or inflight:
        now = time.perf_counter() - t0
        while nxt < total and arrivals[nxt] <= now and free_out[cls_of[nxt]]:
            out = free_out[cls_of[nxt]].pop()
            plain(nxt, out)
            ev = torch.cuda.Event()
            ev.record(stream)
            inflight.append((nxt, ev, out))
            nxt += 1
        while inflight and inflight[0][1].query():
            i, _, out = inflight.pop(0)
            plain_done[i] = time.perf_counter() - t0
            free_out[cls_of[i]].append(out)
        if not inflight and nxt < total:
            wait = arrivals[nxt] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001))
    plain_lat = (plain_done - arrivals)[n_warm:] * 1e3
    plain_span = plain_done[n_warm:].max() - arrivals[n_warm]
    plain_same = True
    for j, lab in kept.items():
        S.seeds_reinit(ctxs[0, j], pool[0][j], stream)
        S.seeds_refine(ctxs[0, j], stream)
        S.seeds_labels(ctxs[0, j], outs_dev[0], stream)
        plain_same &= bool(torch.equal(outs_dev[0].cpu(), lab))
    for cx in ctxs.values():
        S.seeds_destroy(cx)
    torch.cuda.synchronize()
    del free_out
    result = {
        "metric": METRIC, "value": round(served_mpx, 2), "unit": "Mpixel/s",
        "steps": n_timed, "warmup": n_warm, "ms_per_step": round(span * 1e3 / n_timed, 4),
        "config": {"workload": f"serving: Poisson arrivals at {rate:g} req/s of RGB u8 images, "
                               "70% 640x480, 25% 1920x1080, 5% 3840x2160 (Voronoi + gradient + "
                               "noise sigma 8; a pool of 24/8/2 distinct images per size); "
                               "K = pixels/2000, 4 levels, 5 bins, 4 sweeps, gamma 1, Prop. 1 "
                               "rule; labels to pinned host memory; continuous batching server "
                               f"with a {args.budget_gib} GiB budget",
                   "rate_req_s": rate, "offered_mpx_s": round(float(px.mean()) * rate / 1e6, 1),
                   "items_per_group": args.serve_items,
                   "requests_timed": n_timed, "requests_warmup": n_warm,
                   "step": "one request, arrival to labels in host memory"},
        "p50_ms": round(p50, 3), "p99_ms": round(p99, 3),
        "server": {"ticks": stats["ticks"], "peak_inflight": stats["peak_inflight"],
                   "peak_bytes_in_use": stats["peak_bytes_in_use"]},
        "plain_path": {"value": round(px[n_warm:].sum() / plain_span / 1e6, 2),
                       "unit": "Mpixel/s", "p50_ms": round(float(np.percentile(plain_lat, 50)), 3),
                       "p99_ms": round(float(np.percentile(plain_lat, 99)), 3),
                       "note": "single-image contexts, one request at a time in arrival order on "
                               "one stream, replayed under the same arrival times; labels to "
                               "pinned host memory",
                       "labels_equal_to_served": plain_same},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_serve(args, pool_np, kept, arrivals, cls_of, pick)
        result["bitexact_vs_oracle"] = result["cpu_baseline"].pop("labels_equal")
    return result


def cpu_serve(args, pool_np, kept, arrivals, cls_of, pick):
    """The same trace's first requests through a pool of nproc oracle workers
    (threads; the oracle runs outside the interpreter lock), each request
    submitted at its arrival time."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    info = host_info()
    nw = info["nproc"] or 1
    oracle.lib()
    classes = SERVE_CLASSES
    n = min(len(arrivals), args.cpu_serve_requests)

    def job(i):
        c, j = cls_of[i], pick[i]
        h, w = classes[c][0], classes[c][1]
        ref, _, _ = oracle.seeds(pool_np[c][j], h * w // 2000, LEVELS, BINS, ITERS, GAMMA, RULE)
        return ref, time.perf_counter()

    t0 = time.perf_counter()
    futs = []
    with cf.ThreadPoolExecutor(max_workers=nw) as ex:
        for i in range(n):
            wait = arrivals[i] - arrivals[0] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            futs.append(ex.submit(job, i))
        res = [f.result() for f in futs]
    lat = [(res[i][1] - t0 - (arrivals[i] - arrivals[0])) * 1e3 for i in range(n)]
    span = max(r[1] for r in res) - t0
    px = sum(classes[cls_of[i]][0] * classes[cls_of[i]][1] for i in range(n))
    same = True
    for i in range(n):
        if cls_of[i] == 0 and pick[i] in kept:
            same &= bool(np.array_equal(res[i][0], kept[pick[i]].numpy()))
    return {"value": round(px / span / 1e6, 3), "unit": "Mpixel/s", "cores": nw,
            "kind": "oracle (pool of single-threaded workers)",
            "sample": f"the trace's first {n} requests ({px / 1e6:.1f} Mpx), each submitted at its "
                      f"arrival time to {nw} oracle workers; {span:.1f} s",
            "p50_ms": round(float(np.percentile(lat, 50)), 1),
            "p99_ms": round(float(np.percentile(lat, 99)), 1),
            "host": info, "paper_context": PAPER_CONTEXT, "labels_equal": same}


# ---- quality (Sec. 6.1 metrics) ---------------------------------------------------

def run_quality(args) -> dict:
    import numpy as np
    import torch

    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    dev = torch.device("cuda:0")
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
                      f"single-threaded C oracle, {cpu_s:.1f} s", "host": host_info()}
        result["bitexact_vs_oracle"] = same
    return result


# ---- entry ------------------------------------------------------------------------

def _line(result: dict) -> dict:
    """Contract fields common to every printed line."""
    base = {"n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "int32", "data": "synthetic"}
    out = {k: result[k] for k in ("metric", "value", "unit")}
    out.update(base)
    out.update({k: v for k, v in result.items() if k not in out})
    return out


def run_traffic_probe(S, torch, stream, lines=1 << 19):
    """Kernels of known traffic for reading profiler byte counters: the 64 MiB
    device copy the phase profiles are scaled by, then the library's three
    traffic probes over 64 MiB of 128-byte lines (a coalesced read, one
    scattered 4-byte read per line, one scattered 4-byte atomic per line).
    Run under rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE."""
    src = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    us = S.seeds_traffic_probe(lines, stream)
    return {"workload": "traffic probes", "copy_bytes": 64 << 20, "lines": lines,
            "line_bytes": 128, "buffer_bytes": lines * 128,
            "us": {"k_probe_stream": round(us[0], 2), "k_probe_scatter": round(us[1], 2),
                   "k_probe_atomic": round(us[2], 2)}}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["all", "single1080p", "c1", "single4k", "batch64",
                                           "stream4k", "quality", "serve", "traffic_probe"],
                    default="all",
                    help="all (default): the 1080p headline with the other workloads nested")
    ap.add_argument("--steps", type=int, default=None, help="headline steps (default 200)")
    ap.add_argument("--warmup", type=int, default=None, help="headline warm-up (default 20)")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=300, help="stream4k: frames of the stream")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: requests per second")
    ap.add_argument("--requests", type=int, default=4000, help="serve: timed requests")
    ap.add_argument("--warm-requests", type=int, default=500, help="serve: warm-up requests")
    ap.add_argument("--budget-gib", type=int, default=8, help="serve: server memory budget")
    ap.add_argument("--serve-items", type=int, default=2,
                    help="serve: work items per workgroup of the server's phase launches")
    ap.add_argument("--cpu-serve-requests", type=int, default=200,
                    help="serve: requests of the trace replayed through the oracle workers")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch mapping instead of timing the four settings "
                         "(seeds_autotune) before the warm-up")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tuning", default=None,
                    help="pixel_compaction,xcd_remap,items_per_group,init_rows,warm_rows[,block_ppl] "
                         "to set instead of "
                         "autotuning (for profiler runs of the tuned mapping)")
    ap.add_argument("--skip", default="", help="comma-separated nested workloads to leave out")
    ap.add_argument("--skip-byte-pass", action="store_true",
                    help="leave out the untimed phase-by-phase pass that counts boundary units "
                         "(for profiler runs: its hook kernels would mix into the statistics)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="single image: also run one 64 MiB device-to-device copy (a known "
                         "amount of HBM traffic for scaling profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(images are independent: several GPUs would each refine their own images)",
              file=sys.stderr)
        return 2

    import torch

    from paper_1309_3848_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build(force=True)
    from paper_1309_3848_amd import seeds as S
    from paper_1309_3848_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(torch.device("cuda:0"))
    steps = 200 if args.steps is None else args.steps
    warmup = 20 if args.warmup is None else args.warmup
    c2_name = ("single 1920x1080 RGB u8 image, 400 Voronoi regions + gradient + noise sigma 8 "
               "(seed 2); K=1000 (1008 on the grid), 4 levels, 5 bins/channel, 4 sweeps/level, "
               "gamma 1, Prop. 1 block rule")
    c1_name = ("single 481x321 RGB u8 image, 30 Voronoi regions + gradient + noise sigma 8 "
               "(seed 1); K=200 (204 on the grid), 3 levels, 5 bins/channel, 4 sweeps/level, "
               "gamma 1, Prop. 1 block rule")
    stream = torch.cuda.current_stream()
    if args.workload == "traffic_probe":
        print(json.dumps(run_traffic_probe(S, torch, stream)), flush=True)
        return 0
    if args.workload == "quality":
        args.steps, args.warmup = (20 if args.steps is None else args.steps), warmup
        print(json.dumps(_line(run_quality(args))), flush=True)
        return 0
    single = {"single1080p": ("c2", synth.single_1080p(), K, LEVELS, c2_name),
              "c1": ("c1", synth.single_481x321(), 200, 3, c1_name)}
    if args.workload == "single4k":  # the 4K stream's first frame, refined from scratch
        single["single4k"] = ("4k", synth.StreamScene(H=2160, W=3840, regions=1500, frames=1).frame(0),
                              5000, LEVELS, "single 3840x2160 RGB u8 image: frame 0 of the 4K stream "
                              "scene (1500 Voronoi regions, noise sigma 8, seeds 4 / 4000); K=5000, "
                              "4 levels, 5 bins/channel, 4 sweeps/level, gamma 1, Prop. 1 block rule")
    if args.workload in single:
        _, img, k, lv, name = single[args.workload]
        r = run_single(args, img, k, lv, name, steps, warmup,
                       TRAFFIC_FILE if args.workload == "single1080p" else None,
                       LDS_FILE if args.workload == "single1080p" else None)
        lds_peak(S, r, stream)
        launch_floor(S, r, img.shape[0], img.shape[1], stream)
        print(json.dumps(_line(r)), flush=True)
        return 0
    if args.workload != "all":
        fn = {"batch64": run_batch, "stream4k": run_stream, "serve": run_serve}[args.workload]
        print(json.dumps(_line(fn(args))), flush=True)
        return 0

    t_all = time.perf_counter()
    head = run_single(args, synth.single_1080p(), K, LEVELS, c2_name, steps, warmup, TRAFFIC_FILE,
                      LDS_FILE)
    lds_peak(S, head, stream)
    launch_floor(S, head, 1080, 1920, stream)
    print(f"[bench] 1080p done in {time.perf_counter() - t_all:.1f} s", file=sys.stderr, flush=True)
    skip = set(filter(None, args.skip.split(",")))
    nested = {}
    jobs = [("c1_481x321", lambda: run_single(args, synth.single_481x321(), 200, 3, c1_name,
                                              steps, warmup)),
            ("batch64", lambda: run_batch(args)),
            ("stream4k", lambda: run_stream(args)),
            ("serve", lambda: run_serve(args))]
    for key, fn in jobs:
        if key in skip:
            continue
        t = time.perf_counter()
        nested[key] = fn()
        nested[key]["wall_s"] = round(time.perf_counter() - t, 1)
        print(f"[bench] {key} done in {nested[key]['wall_s']} s", file=sys.stderr, flush=True)
    head["workloads"] = nested
    head["bench_wall_s"] = round(time.perf_counter() - t_all, 1)
    print(json.dumps(_line(head)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
