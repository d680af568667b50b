"""Python binding of libseeds (C ABI in include/seeds.h).

Argument marshalling only: every step of the refinement runs in the HIP
library. PyTorch supplies device memory (tensor data pointers) and streams.
There is no fallback: if libseeds.so is missing or cannot be loaded, calls
raise.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so that libseeds shares torch's HIP runtime

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libseeds.so")

SEEDS_OK = 0
SEEDS_E_INVAL = -1
SEEDS_E_NOMEM = -2
SEEDS_E_DEVICE = -3
SEEDS_E_STATE = -4
SEEDS_BLOCK_INTERSECT = 0
SEEDS_BLOCK_EXACT = 1
SEEDS_LAUNCH_GRAPH = 0
SEEDS_LAUNCH_STEPS = 1
SEEDS_LAUNCH_PERSISTENT = 2


class SeedsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libseeds status {status}: {msg}")
        self.status = status


class seeds_params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("bins_per_channel", ctypes.c_int32),
                ("iters_per_level", ctypes.c_int32), ("gamma", ctypes.c_int32),
                ("block_rule", ctypes.c_int32)]


SEEDS_MAX_BATCH = 4096


class seeds_server_params(ctypes.Structure):
    _fields_ = [("bins_per_channel", ctypes.c_int32), ("iters_per_level", ctypes.c_int32),
                ("gamma", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("pixel_compaction", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("items_per_group", ctypes.c_int32)]


class seeds_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "admitted", "completed", "ticks", "queued", "inflight", "peak_inflight",
        "bytes_in_use", "peak_bytes_in_use", "budget_bytes")]


class seeds_tuning(ctypes.Structure):
    _fields_ = [("pixel_compaction", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("items_per_group", ctypes.c_int32), ("init_rows", ctypes.c_int32),
                ("warm_rows", ctypes.c_int32), ("block_ppl", ctypes.c_int32)]


SEEDS_TUNE_VARIANTS = 21


class seeds_quality(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("pixels", "ue", "asa", "cue", "br_hits", "br_total")]


class seeds_image(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("row_pitch_bytes", ctypes.c_int64), ("num_superpixels", ctypes.c_int32),
                ("levels", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int
        PI = ctypes.POINTER(ctypes.c_int32)
        sig = {
            "seeds_default_params": ([ctypes.POINTER(seeds_params)], S),
            "seeds_grid": ([I32, I32, I32, I32, PI, PI], S),
            "seeds_init": ([ctypes.POINTER(P), P, I32, I32, I64, I32, ctypes.POINTER(seeds_params), P], S),
            "seeds_reinit": ([P, P, I64, P], S),
            "seeds_refine": ([P, P], S),
            "seeds_refine_phases": ([P, I32, PI, P], S),
            "seeds_labels": ([P, P, I32, P], S),
            "seeds_num_superpixels": ([P], I32),
            "seeds_histograms": ([P, P, P, I32, P], S),
            "seeds_level": ([P], I32),
            "seeds_set_launch_mode": ([P, I32], S),
            "seeds_sync": ([P, P], S),
            "seeds_batch_init": ([ctypes.POINTER(P), ctypes.POINTER(seeds_image), I32,
                                  ctypes.POINTER(seeds_params), P], S),
            "seeds_batch_reinit": ([P, ctypes.POINTER(P), ctypes.POINTER(I64), P], S),
            "seeds_batch_count": ([P], I32),
            "seeds_warm_start": ([P, P, I64, P], S),
            "seeds_batch_warm_start": ([P, ctypes.POINTER(P), ctypes.POINTER(I64), P], S),
            "seeds_batch_labels": ([P, I32, P, I32, P], S),
            "seeds_batch_labels_all": ([P, P, P], S),
            "seeds_batch_histograms": ([P, I32, P, P, I32, P], S),
            "seeds_batch_num_superpixels": ([P, I32], I32),
            "seeds_energy": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), P], S),
            "seeds_batch_energy": ([P, I32, ctypes.POINTER(I64), ctypes.POINTER(I64), P], S),
            "seeds_quality_metrics": ([P, P, I32, I32, I32, I32, I32, ctypes.POINTER(seeds_quality),
                                       P], S),
            "seeds_server_default_params": ([ctypes.POINTER(seeds_server_params)], S),
            "seeds_server_create": ([ctypes.POINTER(P), ctypes.POINTER(seeds_server_params), P], S),
            "seeds_server_submit": ([P, P, I32, I32, I64, I32, I32, P, I32,
                                     ctypes.POINTER(I64)], S),
            "seeds_server_step": ([P, PI], S),
            "seeds_server_poll": ([P, ctypes.POINTER(I64), I32, PI], S),
            "seeds_server_get_stats": ([P, ctypes.POINTER(seeds_server_stats)], S),
            "seeds_server_destroy": ([P], S),
            "seeds_get_tuning": ([P, ctypes.POINTER(seeds_tuning)], S),
            "seeds_set_tuning": ([P, ctypes.POINTER(seeds_tuning)], S),
            "seeds_autotune": ([P, I32, ctypes.POINTER(seeds_tuning),
                                ctypes.POINTER(ctypes.c_float), P], S),
            "seeds_segment_noalloc": ([P, I32, I32, I64, I32, ctypes.POINTER(seeds_params), P, P],
                                      S),
            "seeds_boundary_units": ([P, I32, I32, ctypes.POINTER(I64), ctypes.POINTER(I64), P],
                                     S),
            "seeds_snapshot_size": ([P, ctypes.POINTER(I64)], S),
            "seeds_snapshot": ([P, P, I64, P], S),
            "seeds_restore": ([P, P, I64, P], S),
            "seeds_lds_atomic_rate": ([ctypes.POINTER(ctypes.c_double), P], S),
            "seeds_launch_floor": ([I32, I32, ctypes.POINTER(ctypes.c_double), P], S),
            "seeds_traffic_probe": ([I64, ctypes.POINTER(ctypes.c_double), P], S),
            "seeds_debug_inject_fault": ([I32, I32], S),
            "seeds_destroy": ([P], S),
            "seeds_last_error": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != SEEDS_OK:
        raise SeedsError(status, lib().seeds_last_error().decode())


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


# ---- the C ABI, one function each -------------------------------------------

def seeds_default_params() -> seeds_params:
    p = seeds_params()
    _check(lib().seeds_default_params(ctypes.byref(p)))
    return p


def seeds_grid(H: int, W: int, num_superpixels: int, levels: int):
    gx, gy = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().seeds_grid(H, W, num_superpixels, levels, ctypes.byref(gx), ctypes.byref(gy)))
    return gx.value, gy.value


def seeds_init(rgb: torch.Tensor, num_superpixels: int, params: seeds_params, stream=None):
    """rgb: H x W x 3 uint8 CUDA tensor (rows may be strided). Returns a ctx handle."""
    _check_rgb(rgb)
    H, W, _ = rgb.shape
    ctx = ctypes.c_void_p()
    _check(lib().seeds_init(ctypes.byref(ctx), rgb.data_ptr(), H, W, rgb.stride(0),
                            num_superpixels, ctypes.byref(params), _stream(stream)))
    return ctx


def _check_rgb(rgb: torch.Tensor) -> None:
    if rgb.dtype != torch.uint8 or rgb.dim() != 3 or rgb.shape[2] != 3 or not rgb.is_cuda:
        raise ValueError("rgb must be an H x W x 3 uint8 device tensor")
    if rgb.stride(2) != 1 or rgb.stride(1) != 3:
        raise ValueError("rgb pixels must be interleaved R,G,B bytes")


def seeds_reinit(ctx, rgb: torch.Tensor, stream=None) -> None:
    _check_rgb(rgb)
    _check(lib().seeds_reinit(ctx, rgb.data_ptr(), rgb.stride(0), _stream(stream)))


def seeds_batch_init(images, num_superpixels, params: seeds_params, levels=None, stream=None):
    """images: list of H x W x 3 uint8 device tensors; num_superpixels and
    levels: one int for all images or one per image (levels default to
    params.levels). Returns a ctx handle."""
    n = len(images)
    ks = list(num_superpixels) if hasattr(num_superpixels, "__len__") else [num_superpixels] * n
    if levels is None:
        levels = params.levels
    ls = list(levels) if hasattr(levels, "__len__") else [levels] * n
    if len(ks) != n or len(ls) != n:
        raise ValueError("one num_superpixels and one levels value per image")
    arr = (seeds_image * max(n, 1))()
    for i, rgb in enumerate(images):
        _check_rgb(rgb)
        arr[i] = seeds_image(rgb.data_ptr(), rgb.shape[0], rgb.shape[1], rgb.stride(0), ks[i], ls[i])
    ctx = ctypes.c_void_p()
    _check(lib().seeds_batch_init(ctypes.byref(ctx), arr, n, ctypes.byref(params),
                                  _stream(stream)))
    return ctx


def _image_tables(ctx, images):
    n = len(images)
    if n != seeds_batch_count(ctx):
        raise ValueError(f"context holds {seeds_batch_count(ctx)} images, got {n}")
    ptrs = (ctypes.c_void_p * max(n, 1))()
    pitches = (ctypes.c_int64 * max(n, 1))()
    for i, rgb in enumerate(images):
        _check_rgb(rgb)
        ptrs[i] = rgb.data_ptr()
        pitches[i] = rgb.stride(0)
    return ptrs, pitches


def seeds_batch_reinit(ctx, images, stream=None) -> None:
    ptrs, pitches = _image_tables(ctx, images)
    _check(lib().seeds_batch_reinit(ctx, ptrs, pitches, _stream(stream)))


def seeds_warm_start(ctx, rgb: torch.Tensor, stream=None) -> None:
    """Next frame of a stream: keep the labels, re-bin, recount; the next
    seeds_refine runs I pixel sweeps."""
    _check_rgb(rgb)
    _check(lib().seeds_warm_start(ctx, rgb.data_ptr(), rgb.stride(0), _stream(stream)))


def seeds_batch_warm_start(ctx, images, stream=None) -> None:
    ptrs, pitches = _image_tables(ctx, images)
    _check(lib().seeds_batch_warm_start(ctx, ptrs, pitches, _stream(stream)))


def seeds_batch_count(ctx) -> int:
    return lib().seeds_batch_count(ctx)


def seeds_batch_labels(ctx, image: int, out: torch.Tensor, stream=None) -> torch.Tensor:
    if out.dtype != torch.int32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor")
    _check(lib().seeds_batch_labels(ctx, image, out.data_ptr(), 0 if out.is_cuda else 1,
                                    _stream(stream)))
    return out


def seeds_batch_labels_all(ctx, outs, stream=None) -> list:
    """Labels of every image into the device tensors `outs` (one per image,
    contiguous int32 of that image's H x W), written in stream order."""
    for o in outs:
        if o.dtype != torch.int32 or not o.is_contiguous() or not o.is_cuda:
            raise ValueError("outs must be contiguous int32 device tensors")
    ptrs = (ctypes.c_void_p * max(1, len(outs)))(*[o.data_ptr() for o in outs])
    if len(outs) != seeds_batch_count(ctx):
        raise ValueError(f"{len(outs)} outputs for {seeds_batch_count(ctx)} images")
    _check(lib().seeds_batch_labels_all(ctx, ptrs, _stream(stream)))
    return outs


def seeds_batch_num_superpixels(ctx, image: int) -> int:
    return lib().seeds_batch_num_superpixels(ctx, image)


def seeds_batch_histograms(ctx, image: int, hist: torch.Tensor | None,
                           size: torch.Tensor | None, stream=None):
    host = _host_flag(hist, size)
    _check(lib().seeds_batch_histograms(ctx, image, hist.data_ptr() if hist is not None else None,
                                        size.data_ptr() if size is not None else None,
                                        1 if host else 0, _stream(stream)))
    return hist, size


def seeds_refine(ctx, stream=None) -> None:
    _check(lib().seeds_refine(ctx, _stream(stream)))


def seeds_refine_phases(ctx, max_phases: int, stream=None) -> int:
    done = ctypes.c_int32()
    _check(lib().seeds_refine_phases(ctx, max_phases, ctypes.byref(done), _stream(stream)))
    return done.value


def seeds_labels(ctx, out: torch.Tensor, stream=None) -> torch.Tensor:
    """Write H x W int32 labels into out (device or host tensor, contiguous)."""
    if out.dtype != torch.int32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 tensor")
    _check(lib().seeds_labels(ctx, out.data_ptr(), 0 if out.is_cuda else 1, _stream(stream)))
    return out


def seeds_num_superpixels(ctx) -> int:
    return lib().seeds_num_superpixels(ctx)


def seeds_level(ctx) -> int:
    return lib().seeds_level(ctx)


def _host_flag(hist, size) -> bool:
    host = None
    for t in (hist, size):
        if t is not None:
            if t.dtype != torch.int32 or not t.is_contiguous():
                raise ValueError("histogram outputs must be contiguous int32 tensors")
            host = (not t.is_cuda) if host is None else host
            if host != (not t.is_cuda):
                raise ValueError("hist and size must both be on the device or both on the host")
    return bool(host)


def seeds_histograms(ctx, hist: torch.Tensor | None, size: torch.Tensor | None, stream=None):
    host = _host_flag(hist, size)
    _check(lib().seeds_histograms(ctx, hist.data_ptr() if hist is not None else None,
                                  size.data_ptr() if size is not None else None,
                                  1 if host else 0, _stream(stream)))
    return hist, size


def seeds_energy(ctx, stream=None) -> tuple:
    """(H', G') of the context's state in count form (exact integers)."""
    h, g = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().seeds_energy(ctx, ctypes.byref(h), ctypes.byref(g), _stream(stream)))
    return h.value, g.value


def seeds_batch_energy(ctx, image: int, stream=None) -> tuple:
    h, g = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().seeds_batch_energy(ctx, image, ctypes.byref(h), ctypes.byref(g), _stream(stream)))
    return h.value, g.value


def seeds_boundary_units(ctx, cls: int = -1, level: int = -1, stream=None):
    """Per image: (boundary units, pixels they cover) of class cls (-1: all)
    on the unit grid of `level` (-1: the image's current level)."""
    n = seeds_batch_count(ctx)
    units = (ctypes.c_int64 * max(n, 1))()
    pixels = (ctypes.c_int64 * max(n, 1))()
    _check(lib().seeds_boundary_units(ctx, level, cls, units, pixels, _stream(stream)))
    return [(units[i], pixels[i]) for i in range(n)]


def seeds_snapshot(ctx, stream=None) -> bytes:
    """The context's whole state (bins, labels, histograms, sizes, cursor)."""
    n = ctypes.c_int64()
    _check(lib().seeds_snapshot_size(ctx, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().seeds_snapshot(ctx, buf, n.value, _stream(stream)))
    return buf.raw


def seeds_restore(ctx, snap: bytes, stream=None) -> None:
    buf = ctypes.create_string_buffer(snap, len(snap))
    _check(lib().seeds_restore(ctx, buf, len(snap), _stream(stream)))


def seeds_set_launch_mode(ctx, mode: int) -> None:
    _check(lib().seeds_set_launch_mode(ctx, mode))


def seeds_sync(ctx, stream=None) -> None:
    _check(lib().seeds_sync(ctx, _stream(stream)))


def seeds_destroy(ctx) -> None:
    _check(lib().seeds_destroy(ctx))


def seeds_quality_metrics(labels: torch.Tensor, truth: torch.Tensor, num_labels: int,
                          num_truth: int, eps: int = 2, stream=None) -> dict:
    """UE, CUE, ASA and BR numerators (Sec. 6.1) of device int32 label maps;
    keys N, ue, asa, cue, br_hits, br_total."""
    for t in (labels, truth):
        if t.dtype != torch.int32 or t.dim() != 2 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("labels and truth must be contiguous H x W int32 device tensors")
    if labels.shape != truth.shape:
        raise ValueError("labels and truth differ in shape")
    q = seeds_quality()
    H, W = labels.shape
    _check(lib().seeds_quality_metrics(labels.data_ptr(), truth.data_ptr(), H, W, num_labels,
                                       num_truth, eps, ctypes.byref(q), _stream(stream)))
    return dict(N=q.pixels, ue=q.ue, asa=q.asa, cue=q.cue, br_hits=q.br_hits,
                br_total=q.br_total)


def seeds_server_default_params() -> seeds_server_params:
    p = seeds_server_params()
    _check(lib().seeds_server_default_params(ctypes.byref(p)))
    return p


def seeds_server_create(params: seeds_server_params, stream=None):
    srv = ctypes.c_void_p()
    _check(lib().seeds_server_create(ctypes.byref(srv), ctypes.byref(params), _stream(stream)))
    return srv


def seeds_server_submit(srv, rgb: torch.Tensor, num_superpixels: int, levels: int,
                        out: torch.Tensor) -> int:
    """Queue rgb (H x W x 3 uint8 device tensor); labels go to out (H x W int32,
    device or pinned host tensor). Returns the request id."""
    _check_rgb(rgb)
    if out.dtype != torch.int32 or not out.is_contiguous() or tuple(out.shape) != tuple(rgb.shape[:2]):
        raise ValueError("out must be a contiguous H x W int32 tensor")
    rid = ctypes.c_int64()
    _check(lib().seeds_server_submit(srv, rgb.data_ptr(), rgb.shape[0], rgb.shape[1],
                                     rgb.stride(0), num_superpixels, levels, out.data_ptr(),
                                     0 if out.is_cuda else 1, ctypes.byref(rid)))
    return rid.value


def seeds_server_step(srv) -> int:
    pending = ctypes.c_int32()
    _check(lib().seeds_server_step(srv, ctypes.byref(pending)))
    return pending.value


def seeds_server_poll(srv, max_ids: int = 1024) -> list:
    ids = (ctypes.c_int64 * max_ids)()
    n = ctypes.c_int32()
    _check(lib().seeds_server_poll(srv, ids, max_ids, ctypes.byref(n)))
    return [ids[i] for i in range(n.value)]


def seeds_server_get_stats(srv) -> dict:
    st = seeds_server_stats()
    _check(lib().seeds_server_get_stats(srv, ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in seeds_server_stats._fields_}


def seeds_server_destroy(srv) -> None:
    _check(lib().seeds_server_destroy(srv))


def _tuning_dict(t: seeds_tuning) -> dict:
    return {f: getattr(t, f) for f, _ in seeds_tuning._fields_}


def seeds_get_tuning(ctx) -> dict:
    t = seeds_tuning()
    _check(lib().seeds_get_tuning(ctx, ctypes.byref(t)))
    return _tuning_dict(t)


def seeds_set_tuning(ctx, pixel_compaction: int = 0, xcd_remap: int = 1,
                     items_per_group: int = 1, init_rows: int = 16, warm_rows: int = 16,
                     block_ppl: int = 1) -> None:
    t = seeds_tuning(pixel_compaction, xcd_remap, items_per_group, init_rows, warm_rows,
                     block_ppl)
    _check(lib().seeds_set_tuning(ctx, ctypes.byref(t)))


def seeds_autotune(ctx, reps: int = 3, stream=None):
    """Time the launch mappings and initialisation tiles, keep the fastest; the
    context comes back freshly initialised. Returns (chosen dict, medians in
    ms per variant, SEEDS_TUNE_VARIANTS entries)."""
    t = seeds_tuning()
    ms = (ctypes.c_float * SEEDS_TUNE_VARIANTS)()
    _check(lib().seeds_autotune(ctx, reps, ctypes.byref(t), ms, _stream(stream)))
    return _tuning_dict(t), [ms[i] for i in range(SEEDS_TUNE_VARIANTS)]


def seeds_segment_noalloc(rgb: torch.Tensor, num_superpixels: int, params: seeds_params,
                          out: torch.Tensor, stream=None) -> torch.Tensor:
    """Allocation-free init + refine + labels of one image into out (H x W
    int32 device tensor); all state lives in the library's fixed device
    array, so calls on one device must not overlap."""
    _check_rgb(rgb)
    H, W, _ = rgb.shape
    if (out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous()
            or tuple(out.shape) != (H, W)):
        raise ValueError("out must be a contiguous H x W int32 device tensor")
    _check(lib().seeds_segment_noalloc(rgb.data_ptr(), H, W, rgb.stride(0), num_superpixels,
                                       ctypes.byref(params), out.data_ptr(), _stream(stream)))
    return out


def seeds_lds_atomic_rate(stream=None) -> float:
    """Measured LDS-atomic throughput, G wavefront instructions per second."""
    r = ctypes.c_double()
    _check(lib().seeds_lds_atomic_rate(ctypes.byref(r), _stream(stream)))
    return r.value


def seeds_launch_floor(groups: int, launches: int = 144, stream=None) -> list:
    """Microseconds per launch of graph-captured launches of `groups`
    workgroups doing nothing, one round of window loads, and two dependent
    rounds plus atomics (the latency floor of a phase launch)."""
    us = (ctypes.c_double * 3)()
    _check(lib().seeds_launch_floor(groups, launches, us, _stream(stream)))
    return [us[0], us[1], us[2]]


def seeds_traffic_probe(lines: int = 1 << 19, stream=None) -> list:
    """Event-timed microseconds of the three traffic probes over `lines`
    128-byte lines: a coalesced read of the buffer, one scattered 4-byte read
    per line, one scattered 4-byte atomic add per line."""
    us = (ctypes.c_double * 3)()
    _check(lib().seeds_traffic_probe(lines, us, _stream(stream)))
    return [us[0], us[1], us[2]]


SEEDS_FAULT_ALLOC = 0
SEEDS_FAULT_LAUNCH = 1


def seeds_debug_inject_fault(kind: int, after: int) -> None:
    """Test hook: the operation of `kind` after `after` more ones fails (on the
    host; nothing runs on the device); after < 0 disarms."""
    _check(lib().seeds_debug_inject_fault(kind, after))


def seeds_last_error() -> str:
    return lib().seeds_last_error().decode()


# ---- convenience --------------------------------------------------------------

def make_params(levels: int = 4, bins: int = 5, iters: int = 4, gamma: int = 1,
                rule: int = SEEDS_BLOCK_INTERSECT) -> seeds_params:
    return seeds_params(levels, bins, iters, gamma, rule)


def superpixels(rgb: torch.Tensor, num_superpixels: int, params: seeds_params,
                stream=None) -> torch.Tensor:
    """One-shot: init, refine and return device int32 labels (H x W)."""
    ctx = seeds_init(rgb, num_superpixels, params, stream)
    try:
        seeds_refine(ctx, stream)
        out = torch.empty(rgb.shape[:2], dtype=torch.int32, device=rgb.device)
        seeds_labels(ctx, out, stream)
    finally:
        seeds_destroy(ctx)
    return out
