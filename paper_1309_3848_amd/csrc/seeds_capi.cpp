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
#include <atomic>
#include <new>
#include <utility>
#include <vector>

#include "seeds.h"
#include "seeds_internal.h"
#include "seeds_readback.h"
#include "seeds_trace.h"

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

// Operations of each kind still allowed before an injected failure (< 0: none
// armed). Decremented by every operation of that kind while armed.
std::atomic<int> g_fault_after[2] = {{-1}, {-1}};

bool inject_fault(int kind) {
    if (kind < 0 || kind > 1) return false;
    int left = g_fault_after[kind].load(std::memory_order_relaxed);
    while (left >= 0) {
        if (g_fault_after[kind].compare_exchange_weak(left, left - 1, std::memory_order_relaxed))
            return left == 0;
    }
    return false;
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
    unsigned long long *hook = nullptr;  // test-hook counters: 2 per image
    int32_t *stage = nullptr;  // int32 pixel labels of one image (readback, hooks)
    const uint8_t **d_rgb = nullptr;  // batch: device table of image pointers
    int64_t *d_pitch = nullptr;       // batch: device table of row pitches
    std::vector<const uint8_t *> rgb;  // host copies of the two tables
    std::vector<int64_t> pitch;
    // batch maps, one set per tuning choice of items per workgroup and block
    // pixels per lane / of init rows
    std::vector<LaunchMap> phase_map[3][2];  // batch: [item choice][ppl choice][level * 9 + cls]
    std::vector<LaunchMap> descend_map;      // batch: [level]
    LaunchMap init_map[3];                   // batch: [row choice]
    // move-log shape of the per-phase launches for each choice of items per
    // workgroup and block pixels per lane (the slab holds the largest)
    int log_groups_of[3][2] = {{1, 1}, {1, 1}, {1, 1}}, log_cap_of[3][2] = {{1, 1}, {1, 1}, {1, 1}};
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

}  // namespace

namespace seeds {

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

}  // namespace seeds

namespace {

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }
size_t round64(size_t v) { return (v + 63) & ~(size_t)63; }

BatchArgs batch_args(const seeds_ctx *ctx) {
    BatchArgs b;
    b.imgs = ctx->d_imgs;
    b.nimg = ctx->nimg;
    b.ar = ctx->ar;
    const int it = item_index(ctx->tune.items), pp = ppl_index(ctx->tune.block_ppl);
    b.log_cap = ctx->log_cap_of[it][pp];
    b.log_groups = ctx->log_groups_of[it][pp];
    b.items = ctx->tune.items;
    b.bppl = ctx->tune.block_ppl;
    return b;
}


LaunchMap descend_launch(const seeds_ctx *ctx, int level) {
    if (ctx->nimg == 1) return {nullptr, descend_groups(ctx->imgs[0].d, level)};
    return ctx->descend_map[level];
}
// Tiles of `rows` rows over every image (initialisation and warm start).
LaunchMap tile_launch(const seeds_ctx *ctx, int rows) {
    if (ctx->nimg == 1) return {nullptr, init_groups(ctx->imgs[0].d, rows)};
    return ctx->init_map[row_index(rows)];
}
LaunchMap init_launch(const seeds_ctx *ctx) { return tile_launch(ctx, ctx->tune.init_rows); }

// Level of image i's labels, and the unit grid holding them.
int image_level(const seeds_ctx *ctx, int i) {
    return std::min(ctx->sched.level, ctx->imgs[i].d.L - 1);
}
// The int32 block grid holding image i's labels (level >= 1).
const int32_t *image_grid(const seeds_ctx *ctx, int i) {
    const ImageDesc &g = ctx->imgs[i];
    return ctx->ar.bl + g.bl[image_level(ctx, i) & 1];
}

seeds_status start_schedule(seeds_ctx *ctx, hipStream_t s) {
    TraceRange tr("seeds init");
    const LaunchMap m = init_launch(ctx);
    // both state copies (histograms, then sizes, of every image) are contiguous
    hipError_t e = inject_fault(SEEDS_FAULT_LAUNCH)
                       ? hipErrorLaunchFailure
                       : launch_fill(ctx->ar.state[0], 0, 2 * ctx->state_elems, s);
    if (e == hipSuccess)
        e = launch_init(batch_args(ctx), ctx->imgs[0], ctx->rgb[0], ctx->pitch[0], m.map,
                        ctx->d_rgb, ctx->d_pitch, m.groups, ctx->tune.init_rows, s);
    if (e != hipSuccess) return device_error(ctx, e, "init launch");
    ctx->sched.level = ctx->top.L - 1;
    ctx->sched.cur_level = ctx->top.L - 1;
    ctx->sched.cur_sweep = 0;
    ctx->sched.cur_class = 0;
    ctx->cold = true;
    ctx->last_stream = s;
    return SEEDS_OK;
}

}  // namespace

namespace seeds {

// Enqueue the schedule from the cursor as per-phase launches (at most
// max_phases phases; < 0: all), ending with the replay that makes both state
// copies equal again.
hipError_t enqueue_schedule(const ScheduleArgs &a, Sched &sched, int32_t max_phases,
                            int32_t *done_out, hipStream_t s) {
    const Dims &top = a.top;
    const bool exact = top.rule == SEEDS_BLOCK_EXACT;
    const BatchArgs &b = a.b;
    const ImageDesc &one = a.one;
    int32_t done = 0;
    int par = 0, prev_groups = 0;
    uint32_t stamp = 0;
    hipError_t e = hipSuccess;
    if (exact) e = launch_fill(b.ar.src, 0, a.src_elems, s);
    // one range per level (opened at the level's first operation)
    int traced_level = -1;
    bool range_open = false;
    for (;;) {
        if (e != hipSuccess) break;
        int cls = 0;
        const SchedOp op = sched_next(top, sched, max_phases < 0 ? -1 : max_phases - done, &cls);
        if (op == OP_END) break;
        if (inject_fault(SEEDS_FAULT_LAUNCH)) {
            e = hipErrorLaunchFailure;
            break;
        }
        const int lv = op == OP_DESCEND ? sched.level - 1 : sched.level;
        if (a.trace && lv != traced_level) {
            if (range_open) roctxRangePop();
            char name[48];
            snprintf(name, sizeof(name), "seeds level %d (unit side %d)", lv, 1 << lv);
            roctxRangePushA(name);
            range_open = true;
            traced_level = lv;
        }
        if (op == OP_DESCEND) {
            const LaunchMap m = a.phase_map ? a.descend_map[sched.level]
                                            : LaunchMap{nullptr, descend_groups(one.d, sched.level)};
            if (m.groups > 0) e = launch_descend(b, one, m.map, sched.level, m.groups, s);
        } else {
            const int level = sched.level;
            const LaunchMap m =
                a.phase_map ? a.phase_map[level * 9 + cls]
                            : LaunchMap{nullptr, phase_launch_groups(one.d, level, cls, a.tune.items,
                                                                     a.tune.block_ppl)};
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
                                     prev_groups, a.tune, s);
                    if (e == hipSuccess)
                        e = launch_phase(b, one, m.map, top.L - 1, level, cls, par, 2, stamp,
                                         m.groups, 0, a.tune, s);
                } else {
                    e = launch_phase(b, one, m.map, top.L - 1, level, cls, par, 0, stamp, m.groups,
                                     prev_groups, a.tune, s);
                }
                prev_groups = m.groups;
                par ^= 1;
            }
            ++done;
        }
        sched_done(sched, op);
    }
    if (range_open) roctxRangePop();
    if (e == hipSuccess && prev_groups > 0) e = launch_final_replay(b, par ^ 1, prev_groups, s);
    if (e == hipSuccess && done_out) *done_out = done;
    return e;
}

}  // namespace seeds

namespace {

seeds_status enqueue_phases(seeds_ctx *ctx, int32_t max_phases, int32_t *done_out, hipStream_t s) {
    ScheduleArgs a;
    a.b = batch_args(ctx);
    a.one = ctx->imgs[0];
    a.top = ctx->top;
    a.phase_map = ctx->nimg > 1
                      ? ctx->phase_map[item_index(ctx->tune.items)][ppl_index(ctx->tune.block_ppl)].data()
                      : nullptr;
    a.descend_map = ctx->nimg > 1 ? ctx->descend_map.data() : nullptr;
    a.src_elems = ctx->src_elems;
    a.tune = ctx->tune;
    const hipError_t e = enqueue_schedule(a, ctx->sched, max_phases, done_out, s);
    if (e != hipSuccess) return device_error(ctx, e, "phase launch");
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
    TraceRange tr("seeds refine");
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
            hipError_t e = inject_fault(SEEDS_FAULT_LAUNCH) ? hipErrorLaunchFailure : hipSuccess;
            if (e == hipSuccess && top.rule == SEEDS_BLOCK_EXACT)
                e = launch_fill(ctx->ar.src, 0, ctx->src_elems, s);
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
    bool lab16 = true;
    size_t max_n = 0;
    for (const auto &im : in) {
        ctx->top.L = std::max(ctx->top.L, im.d.L);
        lab16 &= im.d.K <= kLab16MaxK;
        max_n = std::max(max_n, (size_t)im.d.H * im.d.W);
    }
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
    std::vector<std::pair<size_t, int>> phase_pos[3][2], descend_pos(Lmax);
    std::pair<size_t, int> init_pos[3];
    if (ctx->nimg > 1) {
        for (int v = 0; v < 3; ++v)
            for (int p = 0; p < 2; ++p) {
                phase_pos[v][p].resize(Lmax * 9);
                for (int l = 0; l < Lmax; ++l)
                    for (int c = 0; c < 9; ++c) {
                        if (p == 1 && (l == 0 || l > 3)) {  // the same as one pixel per lane
                            phase_pos[v][p][l * 9 + c] = phase_pos[v][0][l * 9 + c];
                            continue;
                        }
                        phase_pos[v][p][l * 9 + c] =
                            append_map(maps, ctx->imgs, l, [&](const Dims &d) {
                                return phase_launch_groups(d, l, c, kItemChoices[v], kPplChoices[p]);
                            });
                    }
            }
        for (int l = 1; l < Lmax; ++l)
            descend_pos[l] =
                append_map(maps, ctx->imgs, l, [&](const Dims &d) { return descend_groups(d, l); });
        for (int v = 0; v < 3; ++v)
            init_pos[v] = append_map(maps, ctx->imgs, 0,
                                     [&](const Dims &d) { return init_groups(d, kRowChoices[v]); });
    }
    // move-log shape: as many slots as the largest phase launch, each as long
    // as the most deltas one workgroup of any image can produce in a phase
    // (per choice of work items per workgroup: a workgroup's log holds the
    // deltas of all its items)
    size_t log_entries = 0, log_slots = 0;
    for (int p = 0; p < 2; ++p) {
        int round_cap = 1;
        for (const auto &g : ctx->imgs)
            for (int l = 0; l < g.d.L; ++l)
                round_cap = std::max(round_cap, deltas_per_round(g.d, l, kPplChoices[p]));
        for (int v = 0; v < 3; ++v) {
            int groups = 1;
            for (int l = 0; l < Lmax; ++l)
                for (int c = 0; c < 9; ++c) {
                    int n = 0;
                    for (const auto &g : ctx->imgs)
                        if (g.d.L - 1 >= l)
                            n += phase_launch_groups(g.d, l, c, kItemChoices[v], kPplChoices[p]);
                    groups = std::max(groups, n);
                }
            ctx->log_groups_of[v][p] = groups;
            ctx->log_cap_of[v][p] = round_cap * kItemChoices[v];
            log_entries = std::max(log_entries, (size_t)groups * ctx->log_cap_of[v][p]);
            log_slots = std::max(log_slots, (size_t)groups);
        }
    }
    if (ctx->nimg == 1) ctx->geom = persistent_geometry(in[0].d, ctx->device, 2);
    log_entries = std::max(log_entries, (size_t)ctx->geom.groups * ctx->geom.log_cap);
    log_slots = std::max(log_slots, (size_t)ctx->geom.groups);
    // one slab
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t o_bins = take(bins), o_lab = take(lab * (lab16 ? 2 : 4)), o_bl = take(bl * 4);
    const size_t o_state = take(2 * state * 4), o_src = take(src * 4), o_pend = take(pend * 4);
    const size_t o_log = take(2 * log_entries * 8), o_logn = take(2 * log_slots * 4);
    const size_t o_sync = take(16);
    const size_t o_hook = take(16 * std::max<size_t>(2, ctx->imgs.size()));
    const size_t o_stage = take(max_n * 4);
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
    e = inject_fault(SEEDS_FAULT_ALLOC) ? hipErrorOutOfMemory : hipMalloc(&ctx->slab, off);
    if (e != hipSuccess) {
        ctx->slab = nullptr;
        (void)hipGetLastError();
        destroy_ctx(ctx);
        return fail(e == hipErrorOutOfMemory ? SEEDS_E_NOMEM : SEEDS_E_DEVICE,
                    "hipMalloc(%zu): %s", off, hipGetErrorString(e));
    }
    char *base = (char *)ctx->slab;
    ctx->ar.bins = (uint8_t *)(base + o_bins);
    ctx->ar.lab = lab16 ? nullptr : (int32_t *)(base + o_lab);
    ctx->ar.lab16 = lab16 ? (uint16_t *)(base + o_lab) : nullptr;
    ctx->ar.bl = (int32_t *)(base + o_bl);
    ctx->ar.state[0] = (int32_t *)(base + o_state);
    ctx->ar.state[1] = ctx->ar.state[0] + state;
    ctx->ar.src = (int32_t *)(base + o_src);
    ctx->ar.pend = (int32_t *)(base + o_pend);
    ctx->ar.log = (int2 *)(base + o_log);
    ctx->ar.log_n = (int32_t *)(base + o_logn);
    ctx->ar.sync = (uint32_t *)(base + o_sync);
    ctx->hook = (unsigned long long *)(base + o_hook);
    ctx->stage = (int32_t *)(base + o_stage);
    ctx->d_imgs = (ImageDesc *)(base + o_imgs);
    ctx->d_rgb = (const uint8_t **)(base + o_rgb);
    ctx->d_pitch = (int64_t *)(base + o_pitch);
    const int2 *d_maps = (const int2 *)(base + o_maps);
    if (ctx->nimg > 1) {
        for (int v = 0; v < 3; ++v) {
            for (int p = 0; p < 2; ++p) {
                ctx->phase_map[v][p].resize(Lmax * 9);
                for (int i = 0; i < Lmax * 9; ++i)
                    ctx->phase_map[v][p][i] = {d_maps + phase_pos[v][p][i].first,
                                               phase_pos[v][p][i].second};
            }
            ctx->init_map[v] = {d_maps + init_pos[v].first, init_pos[v].second};
        }
        ctx->descend_map.resize(Lmax);
        for (int l = 1; l < Lmax; ++l)
            ctx->descend_map[l] = {d_maps + descend_pos[l].first, descend_pos[l].second};
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

// Image i's pixel labels as int32 in device memory: the int32 pixel plane
// itself, or the staging buffer holding the 16-bit plane widened or a block
// grid expanded (stream-ordered: valid until the next use of the buffer).
const int32_t *pixel_labels32(seeds_ctx *ctx, int32_t image, hipError_t *e, hipStream_t s) {
    const ImageDesc &g = ctx->imgs[image];
    const int level = image_level(ctx, image);
    if (level > 0) {
        *e = launch_expand(g.d, image_grid(ctx, image), level, ctx->stage, s);
        return ctx->stage;
    }
    if (ctx->ar.lab) {
        *e = hipSuccess;
        return ctx->ar.lab + g.lab;
    }
    *e = launch_copy_labels(ctx->stage, ctx->ar, g.lab, (int64_t)g.d.H * g.d.W, s);
    return ctx->stage;
}

// Image i's labels on the unit grid of its current level, as int32.
const int32_t *units32(seeds_ctx *ctx, int32_t image, hipError_t *e, hipStream_t s) {
    if (image_level(ctx, image) > 0) {
        *e = hipSuccess;
        return image_grid(ctx, image);
    }
    return pixel_labels32(ctx, image, e, s);
}

seeds_status labels_of(seeds_ctx *ctx, int32_t image, int32_t *out, int32_t out_is_host,
                       hipStream_t s) {
    const ImageDesc &g = ctx->imgs[image];
    const Dims &d = g.d;
    const int level = image_level(ctx, image);
    hipError_t e;
    if (!out_is_host) {
        e = level == 0 ? launch_copy_labels(out, ctx->ar, g.lab, (int64_t)d.H * d.W, s)
                       : launch_expand(d, image_grid(ctx, image), level, out, s);
        if (e != hipSuccess) return device_error(ctx, e, "labels copy");
        return SEEDS_OK;
    }
    const int32_t *lab = pixel_labels32(ctx, image, &e, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, lab, (size_t)d.H * d.W * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "labels copy");
    return check_device_flag(ctx, s);
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
    hipError_t e;
    const int32_t *lab = pixel_labels32(ctx, image, &e, s);
    unsigned long long host[2] = {0, 0};
    if (e == hipSuccess) e = launch_energy(ctx->ar.state[0] + g.state, g.d, lab, ctx->hook, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host, ctx->hook, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "energy");
    *h_energy = (int64_t)host[0];
    *g_energy = (int64_t)host[1];
    return check_device_flag(ctx, s);
}

// Boundary units of class cls (< 0: all) of every image on the unit grid of
// `level` (< 0: the image's current level; otherwise min(level, L - 1) of the
// image, which the caller keeps at or below its current level), and the
// pixels they cover; host outputs, waits for the stream.
seeds_status boundary_of(seeds_ctx *ctx, int32_t level, int32_t cls, int64_t *units,
                         int64_t *pixels, hipStream_t s) {
    const int n = ctx->nimg;
    hipError_t e = launch_fill((int32_t *)ctx->hook, 0, 4 * (int64_t)n, s);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        const int cur = image_level(ctx, i);
        const int l = level < 0 ? cur : std::min(level, ctx->imgs[i].d.L - 1);
        const int32_t *units = units32(ctx, i, &e, s);
        if (e == hipSuccess)
            e = launch_boundary(units, ctx->imgs[i].d, cur, l, cls, ctx->hook + 2 * i, s);
    }
    std::vector<unsigned long long> host(2 * (size_t)n);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host.data(), ctx->hook, 16 * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "boundary count");
    for (int i = 0; i < n; ++i) {
        if (units) units[i] = (int64_t)host[2 * i];
        if (pixels) pixels[i] = (int64_t)host[2 * i + 1];
    }
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
    TraceRange tr("seeds warm start");
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    if (ctx->sched.level != 0)
        return fail(SEEDS_E_STATE, "warm start needs pixel labels: the context is at level %d "
                                   "(refine the first frame to the end)", ctx->sched.level);
    st = set_images(ctx, rgb, pitch, s);
    if (st != SEEDS_OK) return st;
    const LaunchMap m = tile_launch(ctx, ctx->tune.warm_rows);
    hipError_t e = inject_fault(SEEDS_FAULT_LAUNCH)
                       ? hipErrorLaunchFailure
                       : launch_fill(ctx->ar.state[0], 0, 2 * ctx->state_elems, s);
    if (e == hipSuccess)
        e = launch_rehist(batch_args(ctx), ctx->imgs[0], ctx->rgb[0], ctx->pitch[0], m.map,
                          ctx->d_rgb, ctx->d_pitch, m.groups, ctx->tune.warm_rows, s);
    if (e != hipSuccess) return device_error(ctx, e, "warm start launch");
    ctx->sched.cur_level = -1;
    ctx->sched.cur_sweep = 0;
    ctx->sched.cur_class = 0;
    ctx->cold = false;
    ctx->last_stream = s;
    return SEEDS_OK;
}

// ---- Snapshots -----------------------------------------------------------
// Layout of a snapshot (host memory, native byte order): a SnapHeader, one
// SnapImage per image, then per image its bins (H W bytes), its labels on the
// unit grid of its current level (4 B per unit) and its colour histograms and
// sizes (K hs + K int32, the context's row stride), each part starting at a
// multiple of 8 bytes.
constexpr uint64_t kSnapMagic = 0x31504e5344454553ull;  // "SEEDSNP1"

struct SnapHeader {
    uint64_t magic;
    int32_t nimg;
    int32_t B, I, gamma, rule;
    int32_t level, cur_level, cur_sweep, cur_class, cold;
    int64_t bytes;
};

struct SnapImage {
    int32_t H, W, K, L;
};

size_t up8(size_t v) { return (v + 7) & ~(size_t)7; }

int64_t unit_count(const Dims &d, int level) { return (int64_t)units_w(d, level) * units_h(d, level); }

// Bytes of a snapshot of ctx with its cursor at `level` (the images' unit
// grids depend on it).
int64_t snapshot_bytes(const seeds_ctx *ctx, int level) {
    size_t b = up8(sizeof(SnapHeader)) + up8(sizeof(SnapImage) * ctx->nimg);
    for (const auto &g : ctx->imgs) {
        const Dims &d = g.d;
        const int l = std::min(level, d.L - 1);
        b += up8((size_t)d.H * d.W) + up8((size_t)unit_count(d, l) * 4) +
             up8(((size_t)d.K * d.hs + d.K) * 4);
    }
    return (int64_t)b;
}

seeds_status snapshot(seeds_ctx *ctx, void *host, int64_t bytes, hipStream_t s) {
    const int64_t need = snapshot_bytes(ctx, ctx->sched.level);
    if (bytes < need)
        return fail(SEEDS_E_INVAL, "snapshot buffer of %lld bytes < %lld", (long long)bytes,
                    (long long)need);
    char *p = (char *)host;
    SnapHeader h{};
    h.magic = kSnapMagic;
    h.nimg = ctx->nimg;
    h.B = ctx->top.B;
    h.I = ctx->top.I;
    h.gamma = ctx->top.gamma;
    h.rule = ctx->top.rule;
    h.level = ctx->sched.level;
    h.cur_level = ctx->sched.cur_level;
    h.cur_sweep = ctx->sched.cur_sweep;
    h.cur_class = ctx->sched.cur_class;
    h.cold = ctx->cold ? 1 : 0;
    h.bytes = need;
    std::memcpy(p, &h, sizeof(h));
    size_t off = up8(sizeof(SnapHeader));
    for (int i = 0; i < ctx->nimg; ++i) {
        const Dims &d = ctx->imgs[i].d;
        const SnapImage im{d.H, d.W, d.K, d.L};
        std::memcpy(p + off + i * sizeof(SnapImage), &im, sizeof(im));
    }
    off += up8(sizeof(SnapImage) * ctx->nimg);
    hipError_t e = hipSuccess;
    for (int i = 0; i < ctx->nimg && e == hipSuccess; ++i) {
        const ImageDesc &g = ctx->imgs[i];
        const Dims &d = g.d;
        const size_t nbins = (size_t)d.H * d.W;
        const size_t nunits = (size_t)unit_count(d, image_level(ctx, i)) * 4;
        const size_t nstate = ((size_t)d.K * d.hs + d.K) * 4;
        int32_t *st0 = ctx->ar.state[0] + g.state, *st1 = ctx->ar.state[1] + g.state;
        // pixel phases do not maintain the sizes: derive them first
        e = launch_sizes(d, st0, st1, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p + off, ctx->ar.bins + g.bins, nbins, hipMemcpyDeviceToHost, s);
        off += up8(nbins);
        const int32_t *units = nullptr;
        if (e == hipSuccess) units = units32(ctx, i, &e, s);
        if (e == hipSuccess) e = hipMemcpyAsync(p + off, units, nunits, hipMemcpyDeviceToHost, s);
        off += up8(nunits);
        if (e == hipSuccess) e = hipMemcpyAsync(p + off, st0, nstate, hipMemcpyDeviceToHost, s);
        off += up8(nstate);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "snapshot copy");
    return check_device_flag(ctx, s);
}

seeds_status restore(seeds_ctx *ctx, const void *host, int64_t bytes, hipStream_t s) {
    const char *p = (const char *)host;
    if (bytes < (int64_t)sizeof(SnapHeader)) return fail(SEEDS_E_INVAL, "snapshot too short");
    SnapHeader h;
    std::memcpy(&h, p, sizeof(h));
    if (h.magic != kSnapMagic) return fail(SEEDS_E_INVAL, "not a snapshot (bad magic)");
    if (h.nimg != ctx->nimg)
        return fail(SEEDS_E_INVAL, "snapshot holds %d images, the context %d", h.nimg, ctx->nimg);
    if (h.B != ctx->top.B || h.I != ctx->top.I || h.gamma != ctx->top.gamma ||
        h.rule != ctx->top.rule)
        return fail(SEEDS_E_INVAL, "snapshot parameters (B, I, gamma, rule) differ");
    if (bytes < (int64_t)(up8(sizeof(SnapHeader)) + up8(sizeof(SnapImage) * h.nimg)))
        return fail(SEEDS_E_INVAL, "snapshot too short");
    size_t off = up8(sizeof(SnapHeader));
    for (int i = 0; i < ctx->nimg; ++i) {
        SnapImage im;
        std::memcpy(&im, p + off + i * sizeof(SnapImage), sizeof(im));
        const Dims &d = ctx->imgs[i].d;
        if (im.H != d.H || im.W != d.W || im.K != d.K || im.L != d.L)
            return fail(SEEDS_E_INVAL, "image %d: snapshot %d x %d, K %d, L %d differs from the "
                                       "context", i, im.W, im.H, im.K, im.L);
    }
    Sched sc;
    sc.level = h.level;
    sc.cur_level = h.cur_level;
    sc.cur_sweep = h.cur_sweep;
    sc.cur_class = h.cur_class;
    if (sc.level < 0 || sc.level > ctx->top.L - 1 || sc.cur_level < -1 ||
        sc.cur_level > sc.level || sc.cur_sweep < 0 || sc.cur_sweep > ctx->top.I ||
        sc.cur_class < 0 || sc.cur_class > 8 || (h.cold != 0 && h.cold != 1))
        return fail(SEEDS_E_INVAL, "snapshot cursor (%d, %d, %d, %d) is not a schedule position",
                    sc.level, sc.cur_level, sc.cur_sweep, sc.cur_class);
    const int64_t need = snapshot_bytes(ctx, sc.level);
    if (h.bytes != need || bytes < need)
        return fail(SEEDS_E_INVAL, "snapshot of %lld bytes, expected %lld", (long long)bytes,
                    (long long)need);
    off += up8(sizeof(SnapImage) * ctx->nimg);
    // bins and labels index the histograms: every value is checked before
    // anything reaches the device
    {
        size_t at = off;
        for (int i = 0; i < ctx->nimg; ++i) {
            const Dims &d = ctx->imgs[i].d;
            const size_t nbins = (size_t)d.H * d.W;
            const int l = std::min(sc.level, d.L - 1);
            const size_t nunits = (size_t)unit_count(d, l);
            const uint8_t *bp = (const uint8_t *)(p + at);
            for (size_t q = 0; q < nbins; ++q)
                if (bp[q] >= d.nb) return fail(SEEDS_E_INVAL, "image %d: colour bin out of range", i);
            at += up8(nbins);
            const int32_t *lp = (const int32_t *)(p + at);
            for (size_t q = 0; q < nunits; ++q)
                if (lp[q] < 0 || lp[q] >= d.K) return fail(SEEDS_E_INVAL, "image %d: label out of range", i);
            at += up8(nunits * 4) + up8(((size_t)d.K * d.hs + d.K) * 4);
        }
    }
    ctx->sched = sc;
    ctx->cold = h.cold != 0;
    hipError_t e = hipSuccess;
    for (int i = 0; i < ctx->nimg && e == hipSuccess; ++i) {
        const ImageDesc &g = ctx->imgs[i];
        const Dims &d = g.d;
        const size_t nbins = (size_t)d.H * d.W;
        const size_t nunits = (size_t)unit_count(d, image_level(ctx, i)) * 4;
        const size_t nstate = ((size_t)d.K * d.hs + d.K) * 4;
        e = hipMemcpyAsync(ctx->ar.bins + g.bins, p + off, nbins, hipMemcpyHostToDevice, s);
        off += up8(nbins);
        if (e == hipSuccess) {
            if (image_level(ctx, i) > 0)
                e = hipMemcpyAsync(const_cast<int32_t *>(image_grid(ctx, i)), p + off, nunits,
                                   hipMemcpyHostToDevice, s);
            else if (ctx->ar.lab)
                e = hipMemcpyAsync(ctx->ar.lab + g.lab, p + off, nunits, hipMemcpyHostToDevice, s);
            else {
                // through the staging buffer into the 16-bit plane (values
                // checked below the superpixel count on the host)
                e = hipMemcpyAsync(ctx->stage, p + off, nunits, hipMemcpyHostToDevice, s);
                if (e == hipSuccess)
                    e = launch_narrow_labels(ctx->ar, g.lab, ctx->stage, (int64_t)d.H * d.W, s);
            }
        }
        off += up8(nunits);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->ar.state[0] + g.state, p + off, nstate, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->ar.state[1] + g.state, p + off, nstate, hipMemcpyHostToDevice, s);
        off += up8(nstate);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_error(ctx, e, "restore copy");
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

seeds_status seeds_batch_labels_all(const seeds_ctx *cctx, int32_t *const *outs,
                                    void *hip_stream) {
    seeds_ctx *ctx = const_cast<seeds_ctx *>(cctx);
    seeds_status st = check_image(ctx, 0);
    if (st != SEEDS_OK) return st;
    if (!outs) return fail(SEEDS_E_INVAL, "outs is NULL");
    for (int i = 0; i < ctx->nimg; ++i)
        if (!outs[i]) return fail(SEEDS_E_INVAL, "outs[%d] is NULL", i);
    hipStream_t s = (hipStream_t)hip_stream;
    // images at pixel level with a 16-bit plane: widened together, up to
    // kReadbackMax per launch; any other image through its own copy
    ReadbackList l;
    l.count = 0;
    hipError_t e = hipSuccess;
    for (int i = 0; i < ctx->nimg && e == hipSuccess; ++i) {
        const ImageDesc &g = ctx->imgs[i];
        if (!ctx->ar.lab16 || image_level(ctx, i) > 0) {
            st = labels_of(ctx, i, outs[i], 0, s);
            if (st != SEEDS_OK) return st;
            continue;
        }
        l.src[l.count] = ctx->ar.lab16 + g.lab;
        l.dst[l.count] = outs[i];
        l.n[l.count] = (int64_t)g.d.H * g.d.W;
        if (++l.count == kReadbackMax) {
            e = launch_widen_list(l, s);
            l.count = 0;
        }
    }
    if (e == hipSuccess) e = launch_widen_list(l, s);
    if (e != hipSuccess) return device_error(ctx, e, "labels copy");
    return SEEDS_OK;
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
    out->items_per_group = ctx->tune.items;
    out->init_rows = ctx->tune.init_rows;
    out->warm_rows = ctx->tune.warm_rows;
    out->block_ppl = ctx->tune.block_ppl;
    return SEEDS_OK;
}

seeds_status seeds_set_tuning(seeds_ctx *ctx, const seeds_tuning *t) {
    if (!ctx || !t) return fail(SEEDS_E_INVAL, "NULL argument");
    if ((t->pixel_compaction != 0 && t->pixel_compaction != 1) ||
        (t->xcd_remap != 0 && t->xcd_remap != 1))
        return fail(SEEDS_E_INVAL, "pixel_compaction and xcd_remap are 0 or 1");
    if (t->items_per_group != 1 && t->items_per_group != 2 && t->items_per_group != 4)
        return fail(SEEDS_E_INVAL, "items_per_group %d is not 1, 2 or 4", t->items_per_group);
    if (t->init_rows != 8 && t->init_rows != 16 && t->init_rows != 32)
        return fail(SEEDS_E_INVAL, "init_rows %d is not 8, 16 or 32", t->init_rows);
    if (t->warm_rows != 8 && t->warm_rows != 16 && t->warm_rows != 32)
        return fail(SEEDS_E_INVAL, "warm_rows %d is not 8, 16 or 32", t->warm_rows);
    if (t->block_ppl != 1 && t->block_ppl != 4)
        return fail(SEEDS_E_INVAL, "block_ppl %d is not 1 or 4", t->block_ppl);
    ctx->tune.pixel_compact = t->pixel_compaction != 0;
    ctx->tune.xcd_remap = t->xcd_remap != 0;
    ctx->tune.items = t->items_per_group;
    ctx->tune.init_rows = t->init_rows;
    ctx->tune.warm_rows = t->warm_rows;
    ctx->tune.block_ppl = t->block_ppl;
    clear_graphs(ctx);
    return SEEDS_OK;
}

}  // extern "C"

namespace {

// What time_runs times.
enum TimedOp { TIME_REFINE, TIME_INIT, TIME_WARM };

// Median over reps timed runs (after one untimed warm-up, which also captures
// the refinement graph) of the whole refinement that follows an
// initialisation, of a fresh initialisation, or of a warm start on the
// context's own images (the context must be at pixel level).
seeds_status time_runs(seeds_ctx *ctx, int reps, TimedOp op, hipEvent_t e0, hipEvent_t e1,
                       hipStream_t s, float *median) {
    std::vector<float> t;
    hipError_t e = hipSuccess;
    for (int r = 0; r <= reps; ++r) {
        if (op == TIME_REFINE) {
            seeds_status st = start_schedule(ctx, s);
            if (st != SEEDS_OK) return st;
        }
        e = hipEventRecord(e0, s);
        if (e != hipSuccess) break;
        seeds_status st = op == TIME_REFINE ? run_schedule(ctx, -1, nullptr, s)
                          : op == TIME_INIT ? start_schedule(ctx, s)
                                            : warm_start(ctx, ctx->rgb.data(), ctx->pitch.data(), s);
        if (st != SEEDS_OK) return st;
        e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        if (r > 0) t.push_back(ms);
    }
    if (e != hipSuccess) return device_error(ctx, e, "autotune timing");
    std::sort(t.begin(), t.end());
    *median = t[t.size() / 2];
    return SEEDS_OK;
}

}  // namespace

extern "C" {

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
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return device_error(ctx, e, "hipEventCreate");
    }
    // the phase mapping (compaction x remap x items per workgroup, one pixel
    // per lane in block phases), timed on whole refinements; then four pixels
    // per lane with each choice of items and the chosen compaction and remap;
    // then the rows of the initialisation tiles, timed on initialisations
    // with the chosen mapping
    float best_ms = 0;
    int best = 0;
    ctx->tune.block_ppl = 1;
    for (int v = 0; v < 12 && st == SEEDS_OK; ++v) {
        ctx->tune.pixel_compact = (v & 1) == 0;
        ctx->tune.xcd_remap = (v & 2) == 0;
        ctx->tune.items = kItemChoices[v / 4];
        clear_graphs(ctx);
        float med = 0;
        st = time_runs(ctx, reps, TIME_REFINE, e0, e1, s, &med);
        if (st != SEEDS_OK) break;
        if (ms_per_variant) ms_per_variant[v] = med;
        if (v == 0 || med < best_ms) {
            best_ms = med;
            best = v;
        }
    }
    if (st == SEEDS_OK) {
        ctx->tune.pixel_compact = (best & 1) == 0;
        ctx->tune.xcd_remap = (best & 2) == 0;
    }
    int best_items = best / 4, best_ppl = 0;
    for (int v = 0; v < 3 && st == SEEDS_OK; ++v) {
        ctx->tune.items = kItemChoices[v];
        ctx->tune.block_ppl = 4;
        clear_graphs(ctx);
        float med = 0;
        st = time_runs(ctx, reps, TIME_REFINE, e0, e1, s, &med);
        if (st != SEEDS_OK) break;
        if (ms_per_variant) ms_per_variant[12 + v] = med;
        if (med < best_ms) {
            best_ms = med;
            best_items = v;
            best_ppl = 1;
        }
    }
    if (st == SEEDS_OK) {
        ctx->tune.items = kItemChoices[best_items];
        ctx->tune.block_ppl = kPplChoices[best_ppl];
        clear_graphs(ctx);
    }
    int best_rows = 1;
    for (int v = 0; v < 3 && st == SEEDS_OK; ++v) {
        ctx->tune.init_rows = kRowChoices[v];
        float med = 0;
        st = time_runs(ctx, reps, TIME_INIT, e0, e1, s, &med);
        if (st != SEEDS_OK) break;
        if (ms_per_variant) ms_per_variant[15 + v] = med;
        if (v == 0 || med < best_ms) {
            best_ms = med;
            best_rows = v;
        }
    }
    if (st == SEEDS_OK) ctx->tune.init_rows = kRowChoices[best_rows];
    // the warm start: refine to pixel level once, then warm starts on the
    // same images (each run restarts from the labels the last one left)
    int best_warm = 1;
    if (st == SEEDS_OK) st = start_schedule(ctx, s);
    if (st == SEEDS_OK) st = run_schedule(ctx, -1, nullptr, s);
    for (int v = 0; v < 3 && st == SEEDS_OK; ++v) {
        ctx->tune.warm_rows = kRowChoices[v];
        float med = 0;
        st = time_runs(ctx, reps, TIME_WARM, e0, e1, s, &med);
        if (st != SEEDS_OK) break;
        if (ms_per_variant) ms_per_variant[18 + v] = med;
        if (v == 0 || med < best_ms) {
            best_ms = med;
            best_warm = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != SEEDS_OK) return st;
    ctx->tune.warm_rows = kRowChoices[best_warm];
    if (chosen) (void)seeds_get_tuning(ctx, chosen);
    return start_schedule(ctx, s);
}

seeds_status seeds_boundary_units(const seeds_ctx *cctx, int32_t level, int32_t cls,
                                  int64_t *units, int64_t *pixels, void *hip_stream) {
    seeds_ctx *ctx = const_cast<seeds_ctx *>(cctx);
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    if (cls < -1 || cls > 8) return fail(SEEDS_E_INVAL, "class %d outside [-1,8]", cls);
    if (level > ctx->sched.level)
        return fail(SEEDS_E_INVAL, "level %d is above the context's level %d", level,
                    ctx->sched.level);
    if (!units && !pixels) return fail(SEEDS_E_INVAL, "both outputs are NULL");
    return boundary_of(ctx, level, cls, units, pixels, (hipStream_t)hip_stream);
}

seeds_status seeds_snapshot_size(const seeds_ctx *ctx, int64_t *bytes) {
    if (!bytes) return fail(SEEDS_E_INVAL, "bytes is NULL");
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    *bytes = snapshot_bytes(ctx, ctx->sched.level);
    return SEEDS_OK;
}

seeds_status seeds_snapshot(const seeds_ctx *cctx, void *host, int64_t bytes, void *hip_stream) {
    seeds_ctx *ctx = const_cast<seeds_ctx *>(cctx);
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    if (!host) return fail(SEEDS_E_INVAL, "snapshot buffer is NULL");
    return snapshot(ctx, host, bytes, (hipStream_t)hip_stream);
}

seeds_status seeds_restore(seeds_ctx *ctx, const void *host, int64_t bytes, void *hip_stream) {
    seeds_status st = check_usable(ctx);
    if (st != SEEDS_OK) return st;
    if (!host) return fail(SEEDS_E_INVAL, "snapshot buffer is NULL");
    return restore(ctx, host, bytes, (hipStream_t)hip_stream);
}

seeds_status seeds_debug_inject_fault(int32_t kind, int32_t after) {
    if (kind != SEEDS_FAULT_ALLOC && kind != SEEDS_FAULT_LAUNCH)
        return fail(SEEDS_E_INVAL, "unknown fault kind %d", kind);
    g_fault_after[kind].store(after < 0 ? -1 : after, std::memory_order_relaxed);
    return SEEDS_OK;
}

const char *seeds_last_error(void) { return g_err; }

}  // extern "C"
