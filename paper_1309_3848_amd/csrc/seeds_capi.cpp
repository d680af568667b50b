// C ABI of libseeds: argument checks, the superpixel grid, context memory and
// the refinement schedule (levels x sweeps x nine unit classes).
//
// A context holds one image (seeds_init) or a batch (seeds_batch_init). The
// images of a batch follow one schedule aligned at its end: with Lmax the
// most levels of any image, the schedule walks levels Lmax-1 .. 0 and an
// image of L levels takes part from level L-1 down, exactly as it would on
// its own. All images taking part in a step are at the same level and class,
// so one launch per phase serves the whole batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "seeds.h"
#include "seeds_internal.h"

using namespace seeds;

namespace seeds {

// Text of the last failure on this thread (seeds_last_error).
thread_local char g_err[512] = "";

seeds_status set_error(seeds_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

}  // namespace seeds

namespace {

seeds_status fail(seeds_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

// A refinement captured as a HIP graph, replayed while the schedule starts
// from the same cursor.
struct CachedGraph {
    bool valid = false;
    Sched start{}, end{};
    int32_t phases = 0;
    hipGraphExec_t exec = nullptr;
};

constexpr int kGraphSlots = 4;

// Workgroups of one launch: the map (device array of (image, rank) per
// logical workgroup; nullptr for a single image) and their number.
struct LaunchMap {
    const int2 *map = nullptr;
    int groups = 0;
};

}  // namespace

struct seeds_ctx {
    int device = 0;
    int nimg = 0;
    std::vector<ImageDesc> imgs;  // host copies of the image descriptors
    Dims top{};                   // shared parameters; L = the most levels of any image
    void *slab = nullptr;         // one device allocation holding every arena and table
    Arenas ar{};
    int64_t state_elems = 0;      // elements of one state copy (all images)
    int64_t src_elems = 0;
    ImageDesc *d_imgs = nullptr;  // device copy of imgs
    const uint8_t **d_rgb = nullptr;  // batch: device table of image pointers
    int64_t *d_pitch = nullptr;       // batch: device table of row pitches
    std::vector<const uint8_t *> rgb;  // host copies of the two tables
    std::vector<int64_t> pitch;
    std::vector<LaunchMap> phase_map;    // batch: [level * 9 + cls]
    std::vector<LaunchMap> descend_map;  // batch: [level]
    LaunchMap init_map;                  // batch
    int log_groups = 1, log_cap = 1;  // move-log shape of the per-phase launches
    PersistentGeom geom{};            // single image only
    int mode = SEEDS_LAUNCH_GRAPH;    // seeds_launch_mode
    PhaseTuning tune;                 // mapping of the per-phase launches
    hipStream_t capture = nullptr;    // private stream used only to capture graphs
    CachedGraph graphs[kGraphSlots];
    int next_slot = 0;
    // Schedule cursor on the batch's levels. sched.level is the level whose
    // unit grids hold the labels; an image of fewer levels is at its top
    // level until sched.level comes down to it.
    Sched sched{};
    bool cold = true;       // the first, hierarchical schedule is still running
    bool poisoned = false;  // a device error happened: only destroy is allowed
    hipStream_t last_stream = nullptr;
};

namespace {

seeds_status device_error(seeds_ctx *ctx, hipError_t e, const char *what) {
    if (ctx) ctx->poisoned = true;
    return fail(SEEDS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Superpixel grid (Sec. 5.1): gx = round(sqrt(K W / H)) with halves rounding
// up, i.e. the largest g >= 1 with (2g - 1)^2 H <= 4 K W; gy = round(K / gx).
void grid_of(int64_t H, int64_t W, int64_t K, int *gx_out, int *gy_out) {
    const int64_t rhs = 4 * K * W;
    int64_t g = (int64_t)std::floor(std::sqrt((double)K * (double)W / (double)H) + 0.5);
    if (g < 1) g = 1;
    while ((2 * g + 1) * (2 * g + 1) * H <= rhs) ++g;
    while (g > 1 && (2 * g - 1) * (2 * g - 1) * H > rhs) --g;
    int64_t gy = K / g + (2 * (K % g) >= g ? 1 : 0);
    if (gy < 1) gy = 1;
    *gx_out = (int)g;
    *gy_out = (int)gy;
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
size_t round64(size_t v) { return (v + 63) & ~(size_t)63; }

BatchArgs batch_args(const seeds_ctx *ctx) {
    BatchArgs b;
    b.imgs = ctx->d_imgs;
    b.nimg = ctx->nimg;
    b.ar = ctx->ar;
    b.log_cap = ctx->log_cap;
    b.log_groups = ctx->log_groups;
    return b;
}

LaunchMap phase_launch(const seeds_ctx *ctx, int level, int cls) {
    if (ctx->nimg == 1) return {nullptr, phase_groups(ctx->imgs[0].d, level, cls)};
    return ctx->phase_map[level * 9 + cls];
}
LaunchMap descend_launch(const seeds_ctx *ctx, int level) {
    if (ctx->nimg == 1) return {nullptr, descend_groups(ctx->imgs[0].d, level)};
    return ctx->descend_map[level];
}
LaunchMap init_launch(const seeds_ctx *ctx) {
    if (ctx->nimg == 1) return {nullptr, init_groups(ctx->imgs[0].d)};
    return ctx->init_map;
}

// Level of image i's labels, and the unit grid holding them.
int image_level(const seeds_ctx *ctx, int i) {
    return std::min(ctx->sched.level, ctx->imgs[i].d.L - 1);
}
const int32_t *image_units(const seeds_ctx *ctx, int i) {
    const ImageDesc &g = ctx->imgs[i];
    const int l = image_level(ctx, i);
    return l == 0 ? ctx->ar.lab + g.lab : ctx->ar.bl + g.bl[l & 1];
}

seeds_status start_schedule(seeds_ctx *ctx, hipStream_t s) {
    const LaunchMap m = init_launch(ctx);
    // both state copies (histograms, then sizes, of every image) are contiguous
    hipError_t e = launch_fill(ctx->ar.state[0], 0, 2 * ctx->state_elems, s);
    if (e == hipSuccess)
        e = launch_init(batch_args(ctx), ctx->imgs[0], ctx->rgb[0], ctx->pitch[0], m.map,
                        ctx->d_rgb, ctx->d_pitch, m.groups, s);
    if (e != hipSuccess) return device_error(ctx, e, "init launch");
    ctx->sched.level = ctx->top.L - 1;
    ctx->sched.cur_level = ctx->top.L - 1;
    ctx->sched.cur_sweep = 0;
    ctx->sched.cur_class = 0;
    ctx->cold = true;
    ctx->last_stream = s;
    return SEEDS_OK;
}

// Enqueue the schedule from the current cursor as per-phase launches (at
// most max_phases phases; < 0: all), ending with the replay that makes both
// state copies equal again.
seeds_status enqueue_phases(seeds_ctx *ctx, int32_t max_phases, int32_t *done_out, hipStream_t s) {
    const Dims &top = ctx->top;
    const bool exact = top.rule == SEEDS_BLOCK_EXACT;
    const BatchArgs b = batch_args(ctx);
    const ImageDesc &one = ctx->imgs[0];
    int32_t done = 0;
    int par = 0, prev_groups = 0;
    uint32_t stamp = 0;
    hipError_t e = hipSuccess;
    if (exact) e = launch_fill(ctx->ar.src, 0, ctx->src_elems, s);
    for (;;) {
        if (e != hipSuccess) return device_error(ctx, e, "phase launch");
        int cls = 0;
        const SchedOp op = sched_next(top, ctx->sched, max_phases < 0 ? -1 : max_phases - done, &cls);
        if (op == OP_END) break;
        if (op == OP_DESCEND) {
            const LaunchMap m = descend_launch(ctx, ctx->sched.level);
            if (m.groups > 0) e = launch_descend(b, one, m.map, ctx->sched.level, m.groups, s);
        } else {
            const int level = ctx->sched.level;
            const LaunchMap m = phase_launch(ctx, level, cls);
            ++stamp;
            if (m.groups == 0) {
                // no unit of this class in any image: nothing moves; the
                // previous phase's deltas go to the copy it read, and the
                // next phase starts from equal copies
                if (prev_groups > 0) e = launch_final_replay(b, par ^ 1, prev_groups, s);
                prev_groups = 0;
                par = 0;
            } else {
                if (level > 0 && exact) {
                    e = launch_phase(b, one, m.map, top.L - 1, level, cls, par, 1, stamp, m.groups,
                                     prev_groups, ctx->tune, s);
                    if (e == hipSuccess)
                        e = launch_phase(b, one, m.map, top.L - 1, level, cls, par, 2, stamp,
                                         m.groups, 0, ctx->tune, s);
                } else {
                    e = launch_phase(b, one, m.map, top.L - 1, level, cls, par, 0, stamp, m.groups,
                                     prev_groups, ctx->tune, s);
                }
                prev_groups = m.groups;
                par ^= 1;
            }
            ++done;
        }
        sched_done(ctx->sched, op);
    }
    if (e == hipSuccess && prev_groups > 0) e = launch_final_replay(b, par ^ 1, prev_groups, s);
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
        if (g.valid && same_sched(g.start, ctx->sched)) {
            hipError_t e = hipGraphLaunch(g.exec, s);
            if (e != hipSuccess) return device_error(ctx, e, "hipGraphLaunch");
            ctx->sched = g.end;
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
    g.phases = done;
    g.valid = true;
    e = hipGraphLaunch(g.exec, s);
    if (e != hipSuccess) return device_error(ctx, e, "hipGraphLaunch");
    if (done_out) *done_out = done;
    return SEEDS_OK;
}

seeds_status run_schedule(seeds_ctx *ctx, int32_t max_phases, int32_t *done_out, hipStream_t s) {
    const Dims &top = ctx->top;
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
        int ops = 0;
        for (;;) {
            int cls = 0;
            const SchedOp op = sched_next(top, ctx->sched, max_phases < 0 ? -1 : max_phases - done, &cls);
            if (op == OP_END) break;
            if (op == OP_PHASE) ++done;
            sched_done(ctx->sched, op);
            ++ops;
        }
        if (ops) {
            hipError_t e = hipSuccess;
            if (top.rule == SEEDS_BLOCK_EXACT) e = launch_fill(ctx->ar.src, 0, ctx->src_elems, s);
            if (e == hipSuccess)
                e = launch_refine(batch_args(ctx), ctx->imgs[0], ctx->geom, start, max_phases, 0, s);
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

// Device-side failure flag of the kernels (a grid barrier that timed out, a
// full move log); read after the stream has drained.
seeds_status check_device_flag(seeds_ctx *ctx, hipStream_t s) {
    uint32_t flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, ctx->ar.sync + 2, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "synchronise");
    if (flag) {
        ctx->poisoned = true;
        return fail(SEEDS_E_DEVICE, flag == 2 ? "move log overflow"
                                              : "persistent kernel: grid barrier timed out");
    }
    return SEEDS_OK;
}

// Drop every captured refinement (after a change of the launch mapping).
void clear_graphs(seeds_ctx *ctx) {
    for (auto &g : ctx->graphs)
        if (g.valid) {
            (void)hipGraphExecDestroy(g.exec);
            g.valid = false;
        }
}

void destroy_ctx(seeds_ctx *ctx) {
    for (auto &g : ctx->graphs)
        if (g.valid) (void)hipGraphExecDestroy(g.exec);
    if (ctx->slab) (void)hipFree(ctx->slab);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    delete ctx;
}

struct ImageIn {
    const uint8_t *rgb;
    int64_t pitch;
    Dims d;
};

// Workgroup map of one launch over the images taking part: for each image in
// order, its workgroups ranked 0 .. n-1.
template <typename GroupsOf>
std::pair<size_t, int> append_map(std::vector<int2> &maps, const std::vector<ImageDesc> &imgs,
                                  int min_top_level, GroupsOf groups_of) {
    const size_t at = maps.size();
    for (size_t i = 0; i < imgs.size(); ++i) {
        if (imgs[i].d.L - 1 < min_top_level) continue;
        const int n = groups_of(imgs[i].d);
        for (int r = 0; r < n; ++r) maps.push_back(make_int2((int)i, r));
    }
    return {at, (int)(maps.size() - at)};
}

// Create a context for validated images that share B, I, gamma and the rule.
seeds_status create_ctx(seeds_ctx **out, const std::vector<ImageIn> &in, hipStream_t s) {
    seeds_ctx *ctx = new (std::nothrow) seeds_ctx();
    if (!ctx) return fail(SEEDS_E_NOMEM, "host allocation failed");
    ctx->nimg = (int)in.size();
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) {
        delete ctx;
        return fail(SEEDS_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    ctx->top = in[0].d;
    for (const auto &im : in) ctx->top.L = std::max(ctx->top.L, im.d.L);
    const int Lmax = ctx->top.L;
    // offsets of every image in the arenas; image 0 starts every arena at
    // offset 0, which the single-image kernels rely on
    size_t bins = 0, lab = 0, bl = 0, state = 0, src = 0, pend = 0;
    for (const auto &im : in) {
        const Dims &d = im.d;
        ImageDesc g;
        g.d = d;
        const size_t N = (size_t)d.H * d.W;
        const size_t blk = d.L > 1 ? (size_t)units_w(d, 1) * units_h(d, 1) : 0;
        g.bins = (int64_t)bins;
        bins += round64(N);
        g.lab = (int64_t)lab;
        lab += round64(N);
        g.bl[0] = (int64_t)bl;
        bl += round64(blk);
        g.bl[1] = (int64_t)bl;
        bl += round64(blk);
        g.state = (int64_t)state;
        state += round64((size_t)d.K * d.hs + d.K);
        g.src = (int64_t)src;
        src += round64(d.K);
        g.pend = (int64_t)pend;
        pend += d.L > 1 ? round64(class_units(d, 1, 0)) : 0;  // class 0 is the largest
        ctx->imgs.push_back(g);
        ctx->rgb.push_back(im.rgb);
        ctx->pitch.push_back(im.pitch);
    }
    // log entries and the kernels' state indices are int32
    if (state >= ((size_t)1 << 31)) {
        delete ctx;
        return fail(SEEDS_E_INVAL, "state of the batch (%zu cells) exceeds 2^31", state);
    }
    ctx->state_elems = (int64_t)state;
    ctx->src_elems = (int64_t)src;
    // workgroup maps of a batch
    std::vector<int2> maps;
    std::vector<std::pair<size_t, int>> phase_pos(Lmax * 9), descend_pos(Lmax);
    std::pair<size_t, int> init_pos{0, 0};
    if (ctx->nimg > 1) {
        for (int l = 0; l < Lmax; ++l)
            for (int c = 0; c < 9; ++c)
                phase_pos[l * 9 + c] = append_map(
                    maps, ctx->imgs, l, [&](const Dims &d) { return phase_groups(d, l, c); });
        for (int l = 1; l < Lmax; ++l)
            descend_pos[l] =
                append_map(maps, ctx->imgs, l, [&](const Dims &d) { return descend_groups(d, l); });
        init_pos = append_map(maps, ctx->imgs, 0, [](const Dims &d) { return init_groups(d); });
    }
    // move-log shape: as many slots as the largest phase launch, each as long
    // as the most deltas one workgroup of any image can produce in a phase
    ctx->log_groups = 1;
    ctx->log_cap = 1;
    for (int l = 0; l < Lmax; ++l)
        for (int c = 0; c < 9; ++c) {
            int n = 0;
            for (const auto &g : ctx->imgs)
                if (g.d.L - 1 >= l) n += phase_groups(g.d, l, c);
            ctx->log_groups = std::max(ctx->log_groups, n);
        }
    for (const auto &g : ctx->imgs)
        for (int l = 0; l < g.d.L; ++l) ctx->log_cap = std::max(ctx->log_cap, deltas_per_round(g.d, l));
    if (ctx->nimg == 1) ctx->geom = persistent_geometry(in[0].d, ctx->device, 2);
    const size_t log_entries = std::max((size_t)ctx->geom.groups * ctx->geom.log_cap,
                                        (size_t)ctx->log_groups * ctx->log_cap);
    const size_t log_slots = (size_t)std::max(ctx->geom.groups, ctx->log_groups);
    // one slab
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t o_bins = take(bins), o_lab = take(lab * 4), o_bl = take(bl * 4);
    const size_t o_state = take(2 * state * 4), o_src = take(src * 4), o_pend = take(pend * 4);
    const size_t o_log = take(2 * log_entries * 8), o_logn = take(2 * log_slots * 4);
    const size_t o_sync = take(16);
    const size_t o_imgs = take(ctx->imgs.size() * sizeof(ImageDesc));
    const size_t o_rgb = take(ctx->imgs.size() * sizeof(void *));
    const size_t o_pitch = take(ctx->imgs.size() * sizeof(int64_t));
    const size_t o_maps = take(maps.size() * sizeof(int2));
    e = hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        ctx->capture = nullptr;
        destroy_ctx(ctx);
        return fail(SEEDS_E_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    e = hipMalloc(&ctx->slab, off);
    if (e != hipSuccess) {
        ctx->slab = nullptr;
        (void)hipGetLastError();
        destroy_ctx(ctx);
        return fail(e == hipErrorOutOfMemory ? SEEDS_E_NOMEM : SEEDS_E_DEVICE,
                    "hipMalloc(%zu): %s", off, hipGetErrorString(e));
    }
    char *base = (char *)ctx->slab;
    ctx->ar.bins = (uint8_t *)(base + o_bins);
    ctx->ar.lab = (int32_t *)(base + o_lab);
    ctx->ar.bl = (int32_t *)(base + o_bl);
    ctx->ar.state[0] = (int32_t *)(base + o_state);
    ctx->ar.state[1] = ctx->ar.state[0] + state;
    ctx->ar.src = (int32_t *)(base + o_src);
    ctx->ar.pend = (int32_t *)(base + o_pend);
    ctx->ar.log = (int2 *)(base + o_log);
    ctx->ar.log_n = (int32_t *)(base + o_logn);
    ctx->ar.sync = (uint32_t *)(base + o_sync);
    ctx->d_imgs = (ImageDesc *)(base + o_imgs);
    ctx->d_rgb = (const uint8_t **)(base + o_rgb);
    ctx->d_pitch = (int64_t *)(base + o_pitch);
    const int2 *d_maps = (const int2 *)(base + o_maps);
    if (ctx->nimg > 1) {
        ctx->phase_map.resize(Lmax * 9);
        ctx->descend_map.resize(Lmax);
        for (int i = 0; i < Lmax * 9; ++i)
            ctx->phase_map[i] = {d_maps + phase_pos[i].first, phase_pos[i].second};
        for (int l = 1; l < Lmax; ++l)
            ctx->descend_map[l] = {d_maps + descend_pos[l].first, descend_pos[l].second};
        ctx->init_map = {d_maps + init_pos.first, init_pos.second};
    }
    // tables, in stream order; `maps` is local, so wait for the copies
    e = hipMemcpyAsync(ctx->d_imgs, ctx->imgs.data(), ctx->imgs.size() * sizeof(ImageDesc),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync((void *)ctx->d_rgb, ctx->rgb.data(), ctx->rgb.size() * sizeof(void *),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->d_pitch, ctx->pitch.data(), ctx->pitch.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !maps.empty())
        e = hipMemcpyAsync((void *)d_maps, maps.data(), maps.size() * sizeof(int2),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fill(ctx->ar.src, 0, ctx->src_elems, s);
    if (e == hipSuccess) e = launch_fill((int32_t *)ctx->ar.sync, 0, 4, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        destroy_ctx(ctx);
        return fail(SEEDS_E_DEVICE, "context set-up: %s", hipGetErrorString(e));
    }
    seeds_status st = start_schedule(ctx, s);
    if (st != SEEDS_OK) {
        (void)hipStreamSynchronize(s);
        destroy_ctx(ctx);
        return st;
    }
    *out = ctx;
    return SEEDS_OK;
}

seeds_status check_usable(const seeds_ctx *ctx) {
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (ctx->poisoned) return fail(SEEDS_E_STATE, "context is poisoned by an earlier device error");
    return SEEDS_OK;
}

seeds_status check_image(const seeds_ctx *ctx, int32_t image) {
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (image < 0 || image >= ctx->nimg)
        return fail(SEEDS_E_INVAL, "image %d outside [0,%d)", image, ctx->nimg);
    return check_usable(ctx);
}

seeds_status labels_of(seeds_ctx *ctx, int32_t image, int32_t *out, int32_t out_is_host,
                       hipStream_t s) {
    const ImageDesc &g = ctx->imgs[image];
    const Dims &d = g.d;
    const size_t bytes = (size_t)d.H * d.W * 4;
    int32_t *dst = out;
    void *stage = nullptr;
    hipError_t e;
    if (out_is_host) {
        e = hipMallocAsync(&stage, bytes, s);
        if (e != hipSuccess) return device_error(nullptr, e, "hipMallocAsync");
        dst = (int32_t *)stage;
    }
    const int level = image_level(ctx, image);
    if (level == 0)
        e = launch_copy(dst, ctx->ar.lab + g.lab, (int64_t)d.H * d.W, s);
    else
        e = launch_expand(d, image_units(ctx, image), level, dst, s);
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

seeds_status histograms_of(seeds_ctx *ctx, int32_t image, int32_t *hist, int32_t *size,
                           int32_t out_is_host, hipStream_t s) {
    const ImageDesc &g = ctx->imgs[image];
    const Dims &d = g.d;
    int32_t *st0 = ctx->ar.state[0] + g.state, *st1 = ctx->ar.state[1] + g.state;
    const hipMemcpyKind kind = out_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    // pixel phases do not maintain the sizes: derive them from the histograms
    hipError_t e = launch_sizes(d, st0, st1, s);
    if (e == hipSuccess && hist)
        e = hipMemcpy2DAsync(hist, (size_t)d.nb * 4, st0, (size_t)d.hs * 4, (size_t)d.nb * 4, d.K,
                             kind, s);
    if (e == hipSuccess && size)
        e = hipMemcpyAsync(size, st0 + (size_t)d.K * d.hs, (size_t)d.K * 4, kind, s);
    if (e == hipSuccess && out_is_host) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "histogram copy");
    if (out_is_host) return check_device_flag(ctx, s);
    return SEEDS_OK;
}

// H' and G' of one image's current state (G' on the pixel labels that
// labels_of returns); host outputs, waits for the stream.
seeds_status energy_of(seeds_ctx *ctx, int32_t image, int64_t *h_energy, int64_t *g_energy,
                       hipStream_t s) {
    const ImageDesc &g = ctx->imgs[image];
    const Dims &d = g.d;
    const int level = image_level(ctx, image);
    const size_t lab_bytes = level == 0 ? 0 : (size_t)d.H * d.W * 4;
    void *buf = nullptr;
    hipError_t e = hipMallocAsync(&buf, 16 + lab_bytes, s);
    if (e != hipSuccess) return device_error(nullptr, e, "hipMallocAsync");
    unsigned long long *cnt = (unsigned long long *)buf;
    const int32_t *lab = ctx->ar.lab + g.lab;
    if (level > 0) {
        int32_t *pix = (int32_t *)((char *)buf + 16);
        e = launch_expand(d, image_units(ctx, image), level, pix, s);
        lab = pix;
    }
    unsigned long long host[2] = {0, 0};
    if (e == hipSuccess) e = launch_energy(ctx->ar.state[0] + g.state, d, lab, cnt, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host, cnt, 16, hipMemcpyDeviceToHost, s);
    hipError_t e2 = hipFreeAsync(buf, s);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "energy");
    *h_energy = (int64_t)host[0];
    *g_energy = (int64_t)host[1];
    return check_device_flag(ctx, s);
}

// Take new image pointers and pitches (checked) for the next init or warm
// start. A batch keeps them in device tables, re-uploaded only on change.
seeds_status set_images(seeds_ctx *ctx, const uint8_t *const *rgb, const int64_t *row_pitch_bytes,
                        hipStream_t s) {
    if (!rgb || !row_pitch_bytes) return fail(SEEDS_E_INVAL, "image tables are NULL");
    bool changed = false;
    for (int i = 0; i < ctx->nimg; ++i) {
        if (!rgb[i]) return fail(SEEDS_E_INVAL, "image %d: rgb is NULL", i);
        if (row_pitch_bytes[i] < 3 * (int64_t)ctx->imgs[i].d.W)
            return fail(SEEDS_E_INVAL, "image %d: row pitch %lld < 3 W", i,
                        (long long)row_pitch_bytes[i]);
        changed |= rgb[i] != ctx->rgb[i] || row_pitch_bytes[i] != ctx->pitch[i];
    }
    if (changed && ctx->nimg > 1) {
        // the device tables are read by earlier init launches and copied from
        // the host vectors in stream order: let both finish first
        hipError_t e = hipStreamSynchronize(ctx->last_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return device_error(ctx, e, "synchronise");
        for (int i = 0; i < ctx->nimg; ++i) {
            ctx->rgb[i] = rgb[i];
            ctx->pitch[i] = row_pitch_bytes[i];
        }
        e = hipMemcpyAsync((void *)ctx->d_rgb, ctx->rgb.data(), ctx->rgb.size() * sizeof(void *),
                           hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->d_pitch, ctx->pitch.data(), ctx->pitch.size() * sizeof(int64_t),
                               hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return device_error(ctx, e, "image table upload");
    } else if (changed) {
        ctx->rgb[0] = rgb[0];
        ctx->pitch[0] = row_pitch_bytes[0];
    }
    return SEEDS_OK;
}

// Warm start (a new frame of every image of the context): bins from the new
// pixels, histograms and sizes recounted from the current pixel labels, and
// the schedule marked finished so that the next refine runs I pixel sweeps.
seeds_status warm_start(seeds_ctx *ctx, const uint8_t *const *rgb, const int64_t *pitch,
                        hipStream_t s) {
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    if (ctx->sched.level != 0)
        return fail(SEEDS_E_STATE, "warm start needs pixel labels: the context is at level %d "
                                   "(refine the first frame to the end)", ctx->sched.level);
    st = set_images(ctx, rgb, pitch, s);
    if (st != SEEDS_OK) return st;
    const LaunchMap m = init_launch(ctx);
    hipError_t e = launch_fill(ctx->ar.state[0], 0, 2 * ctx->state_elems, s);
    if (e == hipSuccess)
        e = launch_rehist(batch_args(ctx), ctx->imgs[0], ctx->rgb[0], ctx->pitch[0], m.map,
                          ctx->d_rgb, ctx->d_pitch, m.groups, s);
    if (e != hipSuccess) return device_error(ctx, e, "warm start launch");
    ctx->sched.cur_level = -1;
    ctx->sched.cur_sweep = 0;
    ctx->sched.cur_class = 0;
    ctx->cold = false;
    ctx->last_stream = s;
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
    ImageIn im;
    seeds_status st = check_params(H, W, num_superpixels, p, &im.d);
    if (st != SEEDS_OK) return st;
    if (row_pitch_bytes < 3 * (int64_t)W)
        return fail(SEEDS_E_INVAL, "row pitch %lld < 3 W", (long long)row_pitch_bytes);
    im.rgb = rgb;
    im.pitch = row_pitch_bytes;
    return create_ctx(out, {im}, (hipStream_t)hip_stream);
}

seeds_status seeds_batch_init(seeds_ctx **out, const seeds_image *images, int32_t count,
                              const seeds_params *p, void *hip_stream) {
    if (!out) return fail(SEEDS_E_INVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > SEEDS_MAX_BATCH)
        return fail(SEEDS_E_INVAL, "batch of %d images outside [1,%d]", count, SEEDS_MAX_BATCH);
    if (!images) return fail(SEEDS_E_INVAL, "images is NULL");
    if (!p) return fail(SEEDS_E_INVAL, "params is NULL");
    std::vector<ImageIn> in;
    in.reserve(count);
    for (int i = 0; i < count; ++i) {
        const seeds_image &x = images[i];
        if (!x.rgb) return fail(SEEDS_E_INVAL, "image %d: rgb is NULL", i);
        seeds_params q = *p;
        q.levels = x.levels;
        ImageIn im;
        seeds_status st = check_params(x.height, x.width, x.num_superpixels, &q, &im.d);
        if (st != SEEDS_OK) {
            char msg[512];
            snprintf(msg, sizeof(msg), "%s", g_err);
            return fail(st, "image %d: %s", i, msg);
        }
        if (x.row_pitch_bytes < 3 * (int64_t)x.width)
            return fail(SEEDS_E_INVAL, "image %d: row pitch %lld < 3 W", i,
                        (long long)x.row_pitch_bytes);
        im.rgb = x.rgb;
        im.pitch = x.row_pitch_bytes;
        in.push_back(im);
    }
    return create_ctx(out, in, (hipStream_t)hip_stream);
}

int32_t seeds_batch_count(const seeds_ctx *ctx) { return ctx ? ctx->nimg : -1; }

seeds_status seeds_reinit(seeds_ctx *ctx, const uint8_t *rgb, int64_t row_pitch_bytes,
                          void *hip_stream) {
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (ctx->nimg != 1)
        return fail(SEEDS_E_INVAL, "context holds %d images: use seeds_batch_reinit", ctx->nimg);
    return seeds_batch_reinit(ctx, &rgb, &row_pitch_bytes, hip_stream);
}

seeds_status seeds_batch_reinit(seeds_ctx *ctx, const uint8_t *const *rgb,
                                const int64_t *row_pitch_bytes, void *hip_stream) {
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    st = set_images(ctx, rgb, row_pitch_bytes, (hipStream_t)hip_stream);
    if (st != SEEDS_OK) return st;
    return start_schedule(ctx, (hipStream_t)hip_stream);
}

seeds_status seeds_warm_start(seeds_ctx *ctx, const uint8_t *rgb, int64_t row_pitch_bytes,
                              void *hip_stream) {
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (ctx->nimg != 1)
        return fail(SEEDS_E_INVAL, "context holds %d images: use seeds_batch_warm_start",
                    ctx->nimg);
    return warm_start(ctx, &rgb, &row_pitch_bytes, (hipStream_t)hip_stream);
}

seeds_status seeds_batch_warm_start(seeds_ctx *ctx, const uint8_t *const *rgb,
                                    const int64_t *row_pitch_bytes, void *hip_stream) {
    return warm_start(ctx, rgb, row_pitch_bytes, (hipStream_t)hip_stream);
}

seeds_status seeds_refine_phases(seeds_ctx *ctx, int32_t max_phases, int32_t *phases_done,
                                 void *hip_stream) {
    if (phases_done) *phases_done = 0;
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    return run_schedule(ctx, max_phases, phases_done, (hipStream_t)hip_stream);
}

seeds_status seeds_refine(seeds_ctx *ctx, void *hip_stream) {
    return seeds_refine_phases(ctx, -1, nullptr, hip_stream);
}

seeds_status seeds_labels(const seeds_ctx *ctx, int32_t *out, int32_t out_is_host,
                          void *hip_stream) {
    return seeds_batch_labels(ctx, 0, out, out_is_host, hip_stream);
}

seeds_status seeds_batch_labels(const seeds_ctx *cctx, int32_t image, int32_t *out,
                                int32_t out_is_host, void *hip_stream) {
    seeds_ctx *ctx = const_cast<seeds_ctx *>(cctx);
    seeds_status st = check_image(ctx, image);
    if (st != SEEDS_OK) return st;
    if (!out) return fail(SEEDS_E_INVAL, "out is NULL");
    return labels_of(ctx, image, out, out_is_host, (hipStream_t)hip_stream);
}

int32_t seeds_num_superpixels(const seeds_ctx *ctx) { return seeds_batch_num_superpixels(ctx, 0); }

int32_t seeds_batch_num_superpixels(const seeds_ctx *ctx, int32_t image) {
    if (!ctx || image < 0 || image >= ctx->nimg) return -1;
    return ctx->imgs[image].d.K;
}

int32_t seeds_level(const seeds_ctx *ctx) { return ctx ? ctx->sched.level : -1; }

seeds_status seeds_histograms(const seeds_ctx *ctx, int32_t *hist, int32_t *size,
                              int32_t out_is_host, void *hip_stream) {
    return seeds_batch_histograms(ctx, 0, hist, size, out_is_host, hip_stream);
}

seeds_status seeds_batch_histograms(const seeds_ctx *cctx, int32_t image, int32_t *hist,
                                    int32_t *size, int32_t out_is_host, void *hip_stream) {
    seeds_ctx *ctx = const_cast<seeds_ctx *>(cctx);
    seeds_status st = check_image(ctx, image);
    if (st != SEEDS_OK) return st;
    return histograms_of(ctx, image, hist, size, out_is_host, (hipStream_t)hip_stream);
}

seeds_status seeds_energy(const seeds_ctx *ctx, int64_t *h_energy, int64_t *g_energy,
                          void *hip_stream) {
    return seeds_batch_energy(ctx, 0, h_energy, g_energy, hip_stream);
}

seeds_status seeds_batch_energy(const seeds_ctx *cctx, int32_t image, int64_t *h_energy,
                                int64_t *g_energy, void *hip_stream) {
    seeds_ctx *ctx = const_cast<seeds_ctx *>(cctx);
    seeds_status st = check_image(ctx, image);
    if (st != SEEDS_OK) return st;
    if (!h_energy || !g_energy) return fail(SEEDS_E_INVAL, "energy outputs are NULL");
    return energy_of(ctx, image, h_energy, g_energy, (hipStream_t)hip_stream);
}

seeds_status seeds_set_launch_mode(seeds_ctx *ctx, int32_t mode) {
    if (!ctx) return fail(SEEDS_E_INVAL, "ctx is NULL");
    if (mode != SEEDS_LAUNCH_GRAPH && mode != SEEDS_LAUNCH_PERSISTENT && mode != SEEDS_LAUNCH_STEPS)
        return fail(SEEDS_E_INVAL, "unknown launch mode %d", mode);
    if (mode == SEEDS_LAUNCH_PERSISTENT && ctx->nimg != 1)
        return fail(SEEDS_E_INVAL, "the persistent launch serves single-image contexts only");
    ctx->mode = mode;
    return SEEDS_OK;
}

seeds_status seeds_sync(seeds_ctx *ctx, void *hip_stream) {
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    return check_device_flag(ctx, (hipStream_t)hip_stream);
}

seeds_status seeds_destroy(seeds_ctx *ctx) {
    if (!ctx) return SEEDS_OK;
    // the stream must drain before the memory goes (also after a device error)
    hipError_t e = hipStreamSynchronize(ctx->last_stream);
    destroy_ctx(ctx);
    if (e != hipSuccess) return fail(SEEDS_E_DEVICE, "destroy: %s", hipGetErrorString(e));
    return SEEDS_OK;
}

seeds_status seeds_quality_metrics(const int32_t *labels, const int32_t *truth, int32_t H,
                                   int32_t W, int32_t num_labels, int32_t num_truth, int32_t eps,
                                   seeds_quality *out, void *hip_stream) {
    if (!labels || !truth || !out) return fail(SEEDS_E_INVAL, "NULL pointer");
    if (H < 1 || W < 1 || (int64_t)H * W >= ((int64_t)1 << 31))
        return fail(SEEDS_E_INVAL, "image size %d x %d outside [1, 2^31) pixels", W, H);
    if (num_labels < 1 || num_truth < 1 ||
        (int64_t)num_labels * num_truth > ((int64_t)1 << 28))
        return fail(SEEDS_E_INVAL, "%d labels x %d segments: need both >= 1 and product <= 2^28",
                    num_labels, num_truth);
    if (eps < 1 || eps > 64) return fail(SEEDS_E_INVAL, "eps %d outside [1,64]", eps);
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t table_bytes = align_up((size_t)num_labels * num_truth * 4);
    void *mem = nullptr;
    hipError_t e = hipMallocAsync(&mem, table_bytes + 64, s);
    if (e != hipSuccess) return fail(SEEDS_E_NOMEM, "hipMallocAsync: %s", hipGetErrorString(e));
    unsigned long long cnt[6] = {0, 0, 0, 0, 0, 0};
    auto *d_cnt = (unsigned long long *)((char *)mem + table_bytes);
    e = launch_quality(labels, truth, H, W, num_labels, num_truth, eps, (int32_t *)mem, d_cnt, s);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt, d_cnt, sizeof(cnt), hipMemcpyDeviceToHost, s);
    hipError_t e2 = hipFreeAsync(mem, s);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(SEEDS_E_DEVICE, "quality metrics: %s", hipGetErrorString(e));
    if (cnt[5]) return fail(SEEDS_E_INVAL, "%llu label or segment values out of range", cnt[5]);
    out->pixels = (int64_t)H * W;
    out->ue = (int64_t)cnt[0];
    out->asa = (int64_t)cnt[1];
    out->cue = (int64_t)cnt[2];
    out->br_hits = (int64_t)cnt[3];
    out->br_total = (int64_t)cnt[4];
    return SEEDS_OK;
}

seeds_status seeds_get_tuning(const seeds_ctx *ctx, seeds_tuning *out) {
    if (!ctx || !out) return fail(SEEDS_E_INVAL, "NULL argument");
    out->pixel_compaction = ctx->tune.pixel_compact ? 1 : 0;
    out->xcd_remap = ctx->tune.xcd_remap ? 1 : 0;
    return SEEDS_OK;
}

seeds_status seeds_set_tuning(seeds_ctx *ctx, const seeds_tuning *t) {
    if (!ctx || !t) return fail(SEEDS_E_INVAL, "NULL argument");
    if ((t->pixel_compaction != 0 && t->pixel_compaction != 1) ||
        (t->xcd_remap != 0 && t->xcd_remap != 1))
        return fail(SEEDS_E_INVAL, "tuning fields are 0 or 1");
    ctx->tune.pixel_compact = t->pixel_compaction != 0;
    ctx->tune.xcd_remap = t->xcd_remap != 0;
    clear_graphs(ctx);
    return SEEDS_OK;
}

seeds_status seeds_autotune(seeds_ctx *ctx, int32_t reps, seeds_tuning *chosen,
                            float *ms_per_variant, void *hip_stream) {
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    if (ctx->mode == SEEDS_LAUNCH_PERSISTENT)
        return fail(SEEDS_E_INVAL, "autotuning applies to the per-phase launch modes");
    if (reps < 1 || reps > 50) return fail(SEEDS_E_INVAL, "reps %d outside [1,50]", reps);
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best_ms = 0;
    int best = 0;
    for (int v = 0; v < 4 && e == hipSuccess; ++v) {
        ctx->tune.pixel_compact = (v & 1) == 0;
        ctx->tune.xcd_remap = (v & 2) == 0;
        clear_graphs(ctx);
        std::vector<float> t;
        for (int r = 0; r <= reps && e == hipSuccess; ++r) {  // r = 0 warms up (capture)
            st = start_schedule(ctx, s);
            if (st != SEEDS_OK) break;
            e = hipEventRecord(e0, s);
            if (e != hipSuccess) break;
            st = run_schedule(ctx, -1, nullptr, s);
            if (st != SEEDS_OK) break;
            e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) t.push_back(ms);
        }
        if (st != SEEDS_OK || e != hipSuccess) break;
        std::sort(t.begin(), t.end());
        const float med = t[t.size() / 2];
        if (ms_per_variant) ms_per_variant[v] = med;
        if (v == 0 || med < best_ms) {
            best_ms = med;
            best = v;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != SEEDS_OK) return st;
    if (e != hipSuccess) return device_error(ctx, e, "autotune timing");
    ctx->tune.pixel_compact = (best & 1) == 0;
    ctx->tune.xcd_remap = (best & 2) == 0;
    clear_graphs(ctx);
    if (chosen) {
        chosen->pixel_compaction = ctx->tune.pixel_compact ? 1 : 0;
        chosen->xcd_remap = ctx->tune.xcd_remap ? 1 : 0;
    }
    return start_schedule(ctx, s);
}

const char *seeds_last_error(void) { return g_err; }

}  // extern "C"
