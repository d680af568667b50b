// C ABI of libseeds: argument checks, the superpixel grid, context memory and
// the refinement schedule (levels x sweeps x nine unit classes).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <new>

#include "seeds.h"
#include "seeds_internal.h"

using namespace seeds;

namespace {

thread_local char g_err[512] = "";

seeds_status fail(seeds_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

}  // namespace

// A refinement captured as a HIP graph, replayed while the schedule starts
// from the same cursor.
struct CachedGraph {
    bool valid = false;
    Sched start{}, end{};
    int start_bl = 0, end_bl = 0;
    int32_t phases = 0;
    hipGraphExec_t exec = nullptr;
};

constexpr int kGraphSlots = 4;

struct seeds_ctx {
    Dims d;
    int device;
    void *slab;  // one device allocation holding every buffer
    Buffers b;
    PersistentGeom geom;
    int log_groups, log_cap;  // move-log shape of the per-phase launches
    int mode;    // seeds_launch_mode
    hipStream_t capture;      // private stream used only to capture graphs
    CachedGraph graphs[kGraphSlots];
    int next_slot;
    // state of the partition: the unit grid of sched.level holds the labels
    // (bl[cur_bl] for block levels, b.lab for pixels); sched also holds the
    // next phase of the schedule
    Sched sched;
    int cur_bl;
    bool cold;      // the first, hierarchical schedule is still running
    bool poisoned;  // a device error happened: only destroy is allowed
    uint32_t stamp; // phase counter, stamps move sources for the drop rule
    hipStream_t last_stream;
};

namespace {

seeds_status device_error(seeds_ctx *ctx, hipError_t e, const char *what) {
    if (ctx) ctx->poisoned = true;
    return fail(SEEDS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Superpixel grid (Sec. 5.1): gx = round(sqrt(K W / H)) with halves rounding
// up, i.e. the largest g >= 1 with (2g - 1)^2 H <= 4 K W; gy = round(K / gx).
bool grid_of(int64_t H, int64_t W, int64_t K, int *gx_out, int *gy_out) {
    const int64_t rhs = 4 * K * W;
    int64_t g = (int64_t)std::floor(std::sqrt((double)K * (double)W / (double)H) + 0.5);
    if (g < 1) g = 1;
    while ((2 * g + 1) * (2 * g + 1) * H <= rhs) ++g;
    while (g > 1 && (2 * g - 1) * (2 * g - 1) * H > rhs) --g;
    int64_t gy = K / g + (2 * (K % g) >= g ? 1 : 0);
    if (gy < 1) gy = 1;
    *gx_out = (int)g;
    *gy_out = (int)gy;
    return true;
}

seeds_status check_params(int32_t H, int32_t W, int32_t K, const seeds_params *p, Dims *d) {
    if (!p) return fail(SEEDS_E_INVAL, "params is NULL");
    if (H < 1 || W < 1) return fail(SEEDS_E_INVAL, "image size %d x %d is empty", W, H);
    if ((int64_t)H * W >= (int64_t)1 << 23)
        return fail(SEEDS_E_INVAL, "image of %lld pixels exceeds the 2^23 - 1 limit",
                    (long long)H * W);
    if (K < 1) return fail(SEEDS_E_INVAL, "num_superpixels %d < 1", K);
    if (p->levels < 1 || p->levels > 8)
        return fail(SEEDS_E_INVAL, "levels %d outside [1,8]", p->levels);
    if (p->bins_per_channel < 1 || p->bins_per_channel > 6)
        return fail(SEEDS_E_INVAL, "bins_per_channel %d outside [1,6]", p->bins_per_channel);
    if (p->iters_per_level < 0) return fail(SEEDS_E_INVAL, "iters_per_level %d < 0", p->iters_per_level);
    if (p->gamma < 0 || p->gamma > 65536) return fail(SEEDS_E_INVAL, "gamma %d outside [0,65536]", p->gamma);
    if (p->block_rule != SEEDS_BLOCK_INTERSECT && p->block_rule != SEEDS_BLOCK_EXACT)
        return fail(SEEDS_E_INVAL, "unknown block_rule %d", p->block_rule);
    const int T = 1 << (p->levels - 1);
    if (T > (H < W ? H : W))
        return fail(SEEDS_E_INVAL, "top block side %d exceeds the image side", T);
    int gx, gy;
    grid_of(H, W, K, &gx, &gy);
    const int bw = (W + T - 1) / T, bh = (H + T - 1) / T;
    if (gx > bw || gy > bh)
        return fail(SEEDS_E_INVAL, "%d x %d superpixel grid does not fit %d x %d top blocks", gx,
                    gy, bw, bh);
    d->H = H;
    d->W = W;
    d->B = p->bins_per_channel;
    d->nb = d->B * d->B * d->B;
    d->hs = hist_stride(d->nb);
    d->L = p->levels;
    d->I = p->iters_per_level;
    d->gamma = p->gamma;
    d->rule = p->block_rule;
    d->gx = gx;
    d->gy = gy;
    d->K = gx * gy;
    d->T = T;
    return SEEDS_OK;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Layout of the context's single device allocation. The two histogram
// copies are contiguous, and so are the two size copies.
struct Layout {
    size_t bins, lab, bl0, bl1, hist, src, pend, log, log_n, sync, total;
};

Layout layout_of(const Dims &d, const PersistentGeom &g, int phase_groups_, int phase_cap) {
    const size_t N = (size_t)d.H * d.W;
    const size_t blk = d.L > 1 ? (size_t)units_w(d, 1) * units_h(d, 1) : 0;
    const size_t pend = (size_t)class_cols(d.W, 0) * class_rows(d.H, 0);  // largest class
    Layout l;
    size_t off = 0;
    l.bins = off; off += align_up(N);
    l.lab = off;  off += align_up(N * 4);
    l.bl0 = off;  off += align_up(blk * 4);
    l.bl1 = off;  off += align_up(blk * 4);
    l.hist = off; off += align_up(2 * ((size_t)d.K * d.hs + d.K) * 4);
    l.src = off;  off += align_up((size_t)d.K * 4);
    l.pend = off; off += align_up(pend * 4);
    const size_t entries = std::max((size_t)g.groups * g.log_cap, (size_t)phase_groups_ * phase_cap);
    l.log = off;  off += align_up(2 * entries * 8);
    l.log_n = off; off += align_up(2 * (size_t)std::max(g.groups, phase_groups_) * 4);
    l.sync = off; off += align_up(4 * 4);
    l.total = off;
    return l;
}

int32_t *current_units(seeds_ctx *ctx) {
    return ctx->sched.level == 0 ? ctx->b.lab : ctx->b.bl[ctx->cur_bl];
}

seeds_status start_schedule(seeds_ctx *ctx, const uint8_t *rgb, int64_t pitch, hipStream_t s) {
    const Dims &d = ctx->d;
    ctx->cur_bl = 0;
    int32_t *top = d.L > 1 ? ctx->b.bl[0] : ctx->b.lab;
    hipError_t e = launch_init(d, ctx->b, rgb, pitch, top, s);
    if (e != hipSuccess) return device_error(ctx, e, "init launch");
    ctx->sched.level = d.L - 1;
    ctx->sched.cur_level = d.L - 1;
    ctx->sched.cur_sweep = 0;
    ctx->sched.cur_class = 0;
    ctx->cold = true;
    ctx->last_stream = s;
    return SEEDS_OK;
}

// Split the current level's blocks into their 2x2 children (per-step path).
hipError_t descend_steps(seeds_ctx *ctx, hipStream_t s) {
    const Dims &d = ctx->d;
    const int from = ctx->sched.level;
    if (from == 1) return launch_expand(d, ctx->b.bl[ctx->cur_bl], 1, ctx->b.lab, s);
    hipError_t e = launch_upsample(ctx->b.bl[ctx->cur_bl], units_w(d, from), units_h(d, from),
                                   ctx->b.bl[1 - ctx->cur_bl], units_w(d, from - 1),
                                   units_h(d, from - 1), s);
    ctx->cur_bl = 1 - ctx->cur_bl;
    return e;
}

// Enqueue the schedule from the current cursor as per-phase launches (at
// most max_phases phases; < 0: all), ending with the replay that makes both
// histogram copies equal again.
seeds_status enqueue_phases(seeds_ctx *ctx, int32_t max_phases, int32_t *done_out, hipStream_t s) {
    const Dims &d = ctx->d;
    const bool exact = d.rule == SEEDS_BLOCK_EXACT;
    int32_t done = 0;
    int par = 0, prev_groups = 0;
    uint32_t stamp = 0;
    hipError_t e = hipSuccess;
    if (exact) e = launch_fill(ctx->b.src, 0, d.K, s);
    for (;;) {
        if (e != hipSuccess) return device_error(ctx, e, "phase launch");
        int cls;
        const SchedOp op = sched_next(d, ctx->sched, max_phases < 0 ? -1 : max_phases - done, &cls);
        if (op == OP_END) break;
        if (op == OP_DESCEND) {
            e = descend_steps(ctx, s);
        } else {
            const int level = ctx->sched.level;
            ++stamp;
            if (level > 0 && exact) {
                e = launch_phase_kernel(d, ctx->b, ctx->log_groups, ctx->log_cap, level, cls, par,
                                        1, stamp, ctx->cur_bl, prev_groups, s);
                if (e == hipSuccess)
                    e = launch_phase_kernel(d, ctx->b, ctx->log_groups, ctx->log_cap, level, cls,
                                            par, 2, stamp, ctx->cur_bl, 0, s);
            } else {
                e = launch_phase_kernel(d, ctx->b, ctx->log_groups, ctx->log_cap, level, cls, par,
                                        0, stamp, ctx->cur_bl, prev_groups, s);
            }
            prev_groups = phase_groups(d, level, cls);
            par ^= 1;
            ++done;
        }
        sched_done(ctx->sched, op);
    }
    if (done > 0)
        e = launch_phase_kernel(d, ctx->b, ctx->log_groups, ctx->log_cap, -1, 0, par ^ 1, 0, 0, 0,
                                prev_groups, s);
    if (e != hipSuccess) return device_error(ctx, e, "replay launch");
    if (done_out) *done_out = done;
    return SEEDS_OK;
}

bool same_sched(const Sched &a, const Sched &b) {
    return a.level == b.level && a.cur_level == b.cur_level && a.cur_sweep == b.cur_sweep &&
           a.cur_class == b.cur_class;
}

// Full refinement from the current cursor through a cached graph (captured
// on the first call from this cursor).
seeds_status run_graph(seeds_ctx *ctx, int32_t *done_out, hipStream_t s) {
    for (auto &g : ctx->graphs)
        if (g.valid && same_sched(g.start, ctx->sched) && g.start_bl == ctx->cur_bl) {
            hipError_t e = hipGraphLaunch(g.exec, s);
            if (e != hipSuccess) return device_error(ctx, e, "hipGraphLaunch");
            ctx->sched = g.end;
            ctx->cur_bl = g.end_bl;
            if (done_out) *done_out = g.phases;
            return SEEDS_OK;
        }
    CachedGraph &g = ctx->graphs[ctx->next_slot];
    ctx->next_slot = (ctx->next_slot + 1) % kGraphSlots;
    if (g.valid) {
        (void)hipGraphExecDestroy(g.exec);
        g.valid = false;
    }
    g.start = ctx->sched;
    g.start_bl = ctx->cur_bl;
    hipError_t e = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return device_error(ctx, e, "hipStreamBeginCapture");
    int32_t done = 0;
    seeds_status st = enqueue_phases(ctx, -1, &done, ctx->capture);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->capture, &graph);
    if (st != SEEDS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return device_error(ctx, e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return device_error(ctx, e, "hipGraphInstantiate");
    g.end = ctx->sched;
    g.end_bl = ctx->cur_bl;
    g.phases = done;
    g.valid = true;
    e = hipGraphLaunch(g.exec, s);
    if (e != hipSuccess) return device_error(ctx, e, "hipGraphLaunch");
    if (done_out) *done_out = done;
    return SEEDS_OK;
}

seeds_status run_schedule(seeds_ctx *ctx, int32_t max_phases, int32_t *done_out, hipStream_t s) {
    const Dims &d = ctx->d;
    if (!ctx->cold && ctx->sched.cur_level < 0) {  // finished: another I pixel sweeps
        ctx->sched.cur_level = 0;
        ctx->sched.cur_sweep = 0;
        ctx->sched.cur_class = 0;
    }
    int32_t done = 0;
    seeds_status st = SEEDS_OK;
    if (ctx->mode == SEEDS_LAUNCH_PERSISTENT) {
        // one launch; the host walks the same schedule to keep its cursor
        const Sched start = ctx->sched;
        const int start_bl = ctx->cur_bl;
        int ops = 0;
        for (;;) {
            int cls;
            const SchedOp op = sched_next(d, ctx->sched, max_phases < 0 ? -1 : max_phases - done, &cls);
            if (op == OP_END) break;
            if (op == OP_DESCEND && ctx->sched.level > 1) ctx->cur_bl ^= 1;
            if (op == OP_PHASE) ++done;
            sched_done(ctx->sched, op);
            ++ops;
        }
        if (ops) {
            hipError_t e = hipSuccess;
            if (d.rule == SEEDS_BLOCK_EXACT) e = launch_fill(ctx->b.src, 0, d.K, s);
            if (e == hipSuccess)
                e = launch_refine(d, ctx->b, ctx->geom, start, start_bl, max_phases, 0, s);
            if (e != hipSuccess) return device_error(ctx, e, "persistent refine launch");
        }
    } else if (ctx->mode == SEEDS_LAUNCH_GRAPH && max_phases < 0) {
        st = run_graph(ctx, &done, s);
    } else {
        st = enqueue_phases(ctx, max_phases, &done, s);
    }
    if (st != SEEDS_OK) return st;
    if (ctx->sched.cur_level < 0) ctx->cold = false;
    ctx->last_stream = s;
    if (done_out) *done_out = done;
    return SEEDS_OK;
}

// Device-side failure flag of the persistent kernel (barrier time-out or a
// full move log); read after the stream has drained.
seeds_status check_device_flag(seeds_ctx *ctx, hipStream_t s) {
    uint32_t flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, ctx->b.sync + 2, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "synchronise");
    if (flag) {
        ctx->poisoned = true;
        return fail(SEEDS_E_DEVICE, flag == 2 ? "persistent kernel: move log overflow"
                                              : "persistent kernel: grid barrier timed out");
    }
    return SEEDS_OK;
}

}  // namespace

extern "C" {

seeds_status seeds_default_params(seeds_params *p) {
    if (!p) return fail(SEEDS_E_INVAL, "params is NULL");
    p->levels = 4;
    p->bins_per_channel = 5;
    p->iters_per_level = 4;
    p->gamma = 1;
    p->block_rule = SEEDS_BLOCK_INTERSECT;
    return SEEDS_OK;
}

seeds_status seeds_grid(int32_t H, int32_t W, int32_t K, int32_t levels, int32_t *gx,
                        int32_t *gy) {
    if (!gx || !gy) return fail(SEEDS_E_INVAL, "output pointer is NULL");
    seeds_params p;
    seeds_default_params(&p);
    p.levels = levels;
    Dims d;
    seeds_status st = check_params(H, W, K, &p, &d);
    if (st != SEEDS_OK) return st;
    *gx = d.gx;
    *gy = d.gy;
    return SEEDS_OK;
}

seeds_status seeds_init(seeds_ctx **out, const uint8_t *rgb, int32_t H, int32_t W,
                        int64_t row_pitch_bytes, int32_t num_superpixels, const seeds_params *p,
                        void *hip_stream) {
    if (!out) return fail(SEEDS_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!rgb) return fail(SEEDS_E_INVAL, "rgb is NULL");
    Dims d;
    seeds_status st = check_params(H, W, num_superpixels, p, &d);
    if (st != SEEDS_OK) return st;
    if (row_pitch_bytes < 3 * (int64_t)W)
        return fail(SEEDS_E_INVAL, "row pitch %lld < 3 W", (long long)row_pitch_bytes);
    seeds_ctx *ctx = new (std::nothrow) seeds_ctx();
    if (!ctx) return fail(SEEDS_E_NOMEM, "host allocation failed");
    ctx->d = d;
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) {
        delete ctx;
        return fail(SEEDS_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    ctx->geom = persistent_geometry(d, ctx->device, 2);
    phase_log_shape(d, &ctx->log_groups, &ctx->log_cap);
    ctx->mode = SEEDS_LAUNCH_GRAPH;
    ctx->next_slot = 0;
    e = hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete ctx;
        return fail(SEEDS_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    const Layout l = layout_of(d, ctx->geom, ctx->log_groups, ctx->log_cap);
    e = hipMalloc(&ctx->slab, l.total);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(ctx->capture);
        delete ctx;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? SEEDS_E_NOMEM : SEEDS_E_DEVICE,
                    "hipMalloc(%zu): %s", l.total, hipGetErrorString(e));
    }
    char *base = (char *)ctx->slab;
    ctx->b.bins = (uint8_t *)(base + l.bins);
    ctx->b.lab = (int32_t *)(base + l.lab);
    ctx->b.bl[0] = (int32_t *)(base + l.bl0);
    ctx->b.bl[1] = (int32_t *)(base + l.bl1);
    ctx->b.hist[0] = (int32_t *)(base + l.hist);
    ctx->b.hist[1] = ctx->b.hist[0] + (size_t)d.K * d.hs + d.K;
    ctx->b.size[0] = ctx->b.hist[0] + (size_t)d.K * d.hs;
    ctx->b.size[1] = ctx->b.hist[1] + (size_t)d.K * d.hs;
    ctx->b.src = (int32_t *)(base + l.src);
    ctx->b.pend = (int32_t *)(base + l.pend);
    ctx->b.log = (int2 *)(base + l.log);
    ctx->b.log_n = (int32_t *)(base + l.log_n);
    ctx->b.sync = (uint32_t *)(base + l.sync);
    ctx->stamp = 0;
    e = launch_fill(ctx->b.src, 0, d.K, (hipStream_t)hip_stream);
    if (e == hipSuccess) e = launch_fill((int32_t *)ctx->b.sync, 0, 4, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
        (void)hipFree(ctx->slab);
        (void)hipStreamDestroy(ctx->capture);
        delete ctx;
        return fail(SEEDS_E_DEVICE, "init fill: %s", hipGetErrorString(e));
    }
    st = start_schedule(ctx, rgb, row_pitch_bytes, (hipStream_t)hip_stream);
    if (st != SEEDS_OK) {
        (void)hipStreamSynchronize((hipStream_t)hip_stream);
        (void)hipFree(ctx->slab);
        (void)hipStreamDestroy(ctx->capture);
        delete ctx;
        return st;
    }
    *out = ctx;
    return SEEDS_OK;
}

seeds_status seeds_reinit(seeds_ctx *ctx, const uint8_t *rgb, int64_t row_pitch_bytes,
                          void *hip_stream) {
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (ctx->poisoned) return fail(SEEDS_E_STATE, "context is poisoned by an earlier device error");
    if (!rgb) return fail(SEEDS_E_INVAL, "rgb is NULL");
    if (row_pitch_bytes < 3 * (int64_t)ctx->d.W)
        return fail(SEEDS_E_INVAL, "row pitch %lld < 3 W", (long long)row_pitch_bytes);
    return start_schedule(ctx, rgb, row_pitch_bytes, (hipStream_t)hip_stream);
}

seeds_status seeds_refine_phases(seeds_ctx *ctx, int32_t max_phases, int32_t *phases_done,
                                 void *hip_stream) {
    if (phases_done) *phases_done = 0;
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (ctx->poisoned) return fail(SEEDS_E_STATE, "context is poisoned by an earlier device error");
    return run_schedule(ctx, max_phases, phases_done, (hipStream_t)hip_stream);
}

seeds_status seeds_refine(seeds_ctx *ctx, void *hip_stream) {
    return seeds_refine_phases(ctx, -1, nullptr, hip_stream);
}

seeds_status seeds_labels(const seeds_ctx *cctx, int32_t *out, int32_t out_is_host,
                          void *hip_stream) {
    seeds_ctx *ctx = const_cast<seeds_ctx *>(cctx);
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (!out) return fail(SEEDS_E_INVAL, "out is NULL");
    if (ctx->poisoned) return fail(SEEDS_E_STATE, "context is poisoned by an earlier device error");
    hipStream_t s = (hipStream_t)hip_stream;
    const Dims &d = ctx->d;
    const size_t bytes = (size_t)d.H * d.W * 4;
    int32_t *dst = out;
    void *stage = nullptr;
    hipError_t e;
    if (out_is_host) {
        e = hipMallocAsync(&stage, bytes, s);
        if (e != hipSuccess) return device_error(nullptr, e, "hipMallocAsync");
        dst = (int32_t *)stage;
    }
    if (ctx->sched.level == 0)
        e = hipMemcpyAsync(dst, ctx->b.lab, bytes, hipMemcpyDeviceToDevice, s);
    else
        e = launch_expand(d, ctx->b.bl[ctx->cur_bl], ctx->sched.level, dst, s);
    if (e == hipSuccess && out_is_host) e = hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, s);
    if (out_is_host) {
        hipError_t e2 = hipFreeAsync(stage, s);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) return device_error(ctx, e, "labels copy");
    if (out_is_host) return check_device_flag(ctx, s);
    return SEEDS_OK;
}

int32_t seeds_num_superpixels(const seeds_ctx *ctx) { return ctx ? ctx->d.K : -1; }

int32_t seeds_level(const seeds_ctx *ctx) { return ctx ? ctx->sched.level : -1; }

seeds_status seeds_set_launch_mode(seeds_ctx *ctx, int32_t mode) {
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (mode != SEEDS_LAUNCH_GRAPH && mode != SEEDS_LAUNCH_PERSISTENT && mode != SEEDS_LAUNCH_STEPS)
        return fail(SEEDS_E_INVAL, "unknown launch mode %d", mode);
    ctx->mode = mode;
    return SEEDS_OK;
}

seeds_status seeds_sync(seeds_ctx *ctx, void *hip_stream) {
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (ctx->poisoned) return fail(SEEDS_E_STATE, "context is poisoned by an earlier device error");
    return check_device_flag(ctx, (hipStream_t)hip_stream);
}

seeds_status seeds_histograms(const seeds_ctx *cctx, int32_t *hist, int32_t *size,
                              int32_t out_is_host, void *hip_stream) {
    seeds_ctx *ctx = const_cast<seeds_ctx *>(cctx);
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (ctx->poisoned) return fail(SEEDS_E_STATE, "context is poisoned by an earlier device error");
    hipStream_t s = (hipStream_t)hip_stream;
    const Dims &d = ctx->d;
    const hipMemcpyKind kind = out_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    // pixel phases do not maintain the sizes: derive them from the histograms
    hipError_t e = launch_sizes(d, ctx->b, s);
    if (e == hipSuccess && hist)
        e = hipMemcpy2DAsync(hist, (size_t)d.nb * 4, ctx->b.hist[0], (size_t)d.hs * 4,
                             (size_t)d.nb * 4, d.K, kind, s);
    if (e == hipSuccess && size)
        e = hipMemcpyAsync(size, ctx->b.size[0], (size_t)d.K * 4, kind, s);
    if (e == hipSuccess && out_is_host) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "histogram copy");
    if (out_is_host) return check_device_flag(ctx, s);
    return SEEDS_OK;
}

seeds_status seeds_destroy(seeds_ctx *ctx) {
    if (!ctx) return SEEDS_OK;
    // the stream must drain before the memory goes (also after a device error)
    hipError_t e = hipStreamSynchronize(ctx->last_stream);
    for (auto &g : ctx->graphs)
        if (g.valid) (void)hipGraphExecDestroy(g.exec);
    hipError_t e2 = hipFree(ctx->slab);
    (void)hipStreamDestroy(ctx->capture);
    delete ctx;
    if (e != hipSuccess) return fail(SEEDS_E_DEVICE, "destroy: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(SEEDS_E_DEVICE, "hipFree: %s", hipGetErrorString(e2));
    return SEEDS_OK;
}

const char *seeds_last_error(void) { return g_err; }

}  // extern "C"
