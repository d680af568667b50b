// Serving engine: requests (images) arrive at any time and are refined
// together by continuous batching. Every tick is one launch per kind of work
// - zero and initialise the images admitted in this tick, split the blocks
// of images moving down a level, and one phase of every image in flight, each
// at its own level and class - so a new image starts at its top level while
// others are in the middle of their hierarchy. Images are admitted in arrival
// order as device memory (pixels, histograms, move logs) allows, and their
// memory returns to the pool two ticks after their last phase.
//
// Each image runs exactly its single-image schedule: one phase per tick, all
// of its decisions made from its own state at the start of the phase, so its
// labels equal those of a single-image context bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "seeds.h"
#include "seeds_internal.h"
#include "seeds_trace.h"

using namespace seeds;

namespace {

template <typename... A>
seeds_status sfail(seeds_status st, const char *fmt, A... a) {
    return set_error(st, fmt, a...);
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing of freed ranges.
class FreeList {
public:
    explicit FreeList(size_t size = 0) { if (size) free_[0] = size; }
    bool alloc(size_t n, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }

private:
    std::map<size_t, size_t> free_;
};

constexpr size_t kGran = 256;  // allocation granule (bytes / 4-byte elements x 64)
constexpr int kRing = 8;       // ticks the host may run ahead of the device
constexpr int kCoarseCap = 1 << 16;  // coarse index entries per tick (all lists)

struct Request {
    int64_t id;
    const uint8_t *rgb;
    int64_t pitch;
    Dims d;
    int32_t *out;
    bool out_host;
    int32_t *out_dev;      // pinned host output as the device sees it, else nullptr
    ImageDesc g;
    Sched sc;
    size_t px_off, px_len, st_off, st_len;
    int groups_max;        // most phase workgroups of any of its phases
    int64_t finish_tick;   // tick of its last phase, -1 while running
    hipEvent_t done;       // recorded after its labels are written
    bool reported;
};

// Device footprint of one image in the pixel arena: bins, labels, two block
// grids, each rounded to the granule.
size_t pixel_bytes(const Dims &d) {
    const size_t N = (size_t)d.H * d.W;
    const size_t blk = d.L > 1 ? (size_t)units_w(d, 1) * units_h(d, 1) : 0;
    return round_up(N, kGran) + round_up(N * 4, kGran) + 2 * round_up(blk * 4, kGran);
}
size_t state_elems(const Dims &d) { return round_up((size_t)d.K * d.hs + d.K, 64); }
int max_phase_groups(const Dims &d, int items) {
    int g = 0;
    for (int l = 0; l < d.L; ++l)
        for (int c = 0; c < 9; ++c) g = std::max(g, phase_launch_groups(d, l, c, items));
    return g;
}

}  // namespace

struct seeds_server {
    seeds_server_params p;
    PhaseTuning tune;
    int device = 0;
    hipStream_t s = nullptr;
    hipStream_t copy = nullptr;    // label outputs, overlapped with the ticks
    hipEvent_t gate[kRing] = {};   // end of a tick's kernels, for the copy stream
    void *slab = nullptr;
    uint8_t *px_base = nullptr;
    size_t px_size = 0, st_size = 0;
    Arenas ar{};
    int log_cap = 1, g_cap = 1, g_used = 0;
    FreeList px, st;
    size_t ring_bytes = 0, items_bytes = 0;
    uint8_t *ring_host = nullptr;  // pinned, kRing slots
    uint8_t *ring_dev = nullptr;   // device, kRing slots
    uint32_t *flag_host = nullptr; // pinned copy of the device error flag
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    std::deque<Request *> queue;
    std::vector<Request *> running, finishing, unreported;
    int64_t next_id = 1, tick = 0;
    int par = 0, prev_groups = 0;
    bool poisoned = false;
    seeds_server_stats stats{};
};

namespace {

seeds_status srv_device_error(seeds_server *sv, hipError_t e, const char *what) {
    sv->poisoned = true;
    return sfail(SEEDS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void destroy_request(Request *r) {
    if (r->done) (void)hipEventDestroy(r->done);
    delete r;
}

hipError_t release_request(seeds_server *sv, Request *r) {
    // the labels copy reads the pixel region on the copy stream: later ticks
    // on the main stream, which may reuse it, wait for that copy
    hipError_t e = hipStreamWaitEvent(sv->s, r->done, 0);
    sv->px.release(r->px_off, r->px_len);
    sv->st.release(r->st_off, r->st_len);
    sv->g_used -= r->groups_max;
    sv->stats.bytes_in_use -= (int64_t)(r->px_len + r->st_len * 8);
    return e;
}

bool try_admit(seeds_server *sv, Request *r) {
    if ((int)sv->running.size() >= sv->p.max_inflight) return false;
    if (sv->g_used + r->groups_max > sv->g_cap) return false;
    size_t po, so;
    if (!sv->px.alloc(r->px_len, &po)) return false;
    if (!sv->st.alloc(r->st_len, &so)) {
        sv->px.release(po, r->px_len);
        return false;
    }
    r->px_off = po;
    r->st_off = so;
    sv->g_used += r->groups_max;
    const Dims &d = r->d;
    const size_t N = (size_t)d.H * d.W;
    const size_t blk = d.L > 1 ? (size_t)units_w(d, 1) * units_h(d, 1) : 0;
    ImageDesc &g = r->g;
    g.d = d;
    g.bins = (int64_t)po;
    g.lab = (int64_t)(po + round_up(N, kGran)) / 4;
    g.bl[0] = g.lab + (int64_t)round_up(N * 4, kGran) / 4;
    g.bl[1] = g.bl[0] + (int64_t)round_up(blk * 4, kGran) / 4;
    g.state = (int64_t)so;
    g.src = 0;
    g.pend = 0;
    r->sc.level = d.L - 1;
    r->sc.cur_level = d.L - 1;
    r->sc.cur_sweep = 0;
    r->sc.cur_class = 0;
    sv->stats.bytes_in_use += (int64_t)(r->px_len + r->st_len * 8);
    sv->stats.peak_bytes_in_use = std::max(sv->stats.peak_bytes_in_use, sv->stats.bytes_in_use);
    return true;
}

BatchArgs server_args(const seeds_server *sv) {
    BatchArgs b;
    b.imgs = nullptr;
    b.nimg = 2;  // mixed launches take their images from their items
    b.ar = sv->ar;
    b.log_cap = sv->log_cap;
    b.log_groups = sv->g_cap;
    return b;
}

}  // namespace

extern "C" {

seeds_status seeds_server_default_params(seeds_server_params *p) {
    if (!p) return sfail(SEEDS_E_INVAL, "params is NULL");
    p->bins_per_channel = 5;
    p->iters_per_level = 4;
    p->gamma = 1;
    p->max_levels = 4;
    p->hbm_budget_bytes = (int64_t)4 << 30;
    p->max_inflight = 512;
    p->pixel_compaction = 0;
    p->xcd_remap = 0;
    p->items_per_group = 2;
    return SEEDS_OK;
}

seeds_status seeds_server_create(seeds_server **out, const seeds_server_params *p,
                                 void *hip_stream) {
    if (!out) return sfail(SEEDS_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!p) return sfail(SEEDS_E_INVAL, "params is NULL");
    if (p->bins_per_channel < 1 || p->bins_per_channel > 6)
        return sfail(SEEDS_E_INVAL, "bins_per_channel %d outside [1,6]", p->bins_per_channel);
    if (p->iters_per_level < 1)
        return sfail(SEEDS_E_INVAL, "iters_per_level %d < 1", p->iters_per_level);
    if (p->gamma < 0 || p->gamma > 65536)
        return sfail(SEEDS_E_INVAL, "gamma %d outside [0,65536]", p->gamma);
    if (p->max_levels < 1 || p->max_levels > 8)
        return sfail(SEEDS_E_INVAL, "max_levels %d outside [1,8]", p->max_levels);
    if (p->max_inflight < 1 || p->max_inflight > 65536)
        return sfail(SEEDS_E_INVAL, "max_inflight %d outside [1,65536]", p->max_inflight);
    if (p->hbm_budget_bytes < ((int64_t)64 << 20) || p->hbm_budget_bytes > ((int64_t)128 << 30))
        return sfail(SEEDS_E_INVAL, "hbm_budget_bytes outside [64 MiB, 128 GiB]");
    if ((p->pixel_compaction != 0 && p->pixel_compaction != 1) ||
        (p->xcd_remap != 0 && p->xcd_remap != 1))
        return sfail(SEEDS_E_INVAL, "pixel_compaction and xcd_remap are 0 or 1");
    if (p->items_per_group != 1 && p->items_per_group != 2 && p->items_per_group != 4)
        return sfail(SEEDS_E_INVAL, "items_per_group %d is not 1, 2 or 4", p->items_per_group);
    seeds_server *sv = new (std::nothrow) seeds_server();
    if (!sv) return sfail(SEEDS_E_NOMEM, "host allocation failed");
    sv->p = *p;
    sv->tune.pixel_compact = p->pixel_compaction != 0;
    sv->tune.xcd_remap = p->xcd_remap != 0;
    sv->tune.items = p->items_per_group;
    sv->s = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&sv->device);
    // log entries per workgroup and phase: the most any level can produce
    Dims dd{};
    dd.B = p->bins_per_channel;
    dd.nb = dd.B * dd.B * dd.B;
    for (int l = 0; l < p->max_levels; ++l) sv->log_cap = std::max(sv->log_cap, deltas_per_round(dd, l));
    sv->log_cap *= p->items_per_group;  // a workgroup's log holds all its items
    // budget: 60% pixels, 8% histograms (two copies), 32% move logs
    const size_t budget = (size_t)p->hbm_budget_bytes;
    sv->px_size = round_up(budget / 100 * 60, kGran);
    sv->st_size = round_up(budget / 100 * 8 / 8, 64);  // elements per copy
    if (sv->st_size >= ((size_t)1 << 31)) sv->st_size = ((size_t)1 << 31) - 64;
    sv->g_cap = (int)std::min<size_t>(budget / 100 * 32 / (2 * (size_t)sv->log_cap * 8), 1 << 26);
    sv->px = FreeList(sv->px_size);
    sv->st = FreeList(sv->st_size);
    sv->items_bytes = round_up((size_t)4 * p->max_inflight * sizeof(TickItem), kGran);
    sv->ring_bytes = sv->items_bytes + kCoarseCap * sizeof(int32_t);
    size_t off = 0;
    auto take = [&](size_t n) { const size_t o = off; off += round_up(n, kGran); return o; };
    const size_t o_px = take(sv->px_size), o_st = take(2 * sv->st_size * 4);
    const size_t o_log = take(2 * (size_t)sv->g_cap * sv->log_cap * 8);
    const size_t o_logn = take(2 * (size_t)sv->g_cap * 4), o_sync = take(16), o_dummy = take(256);
    const size_t o_ring = take(kRing * sv->ring_bytes);
    if (e == hipSuccess)
        e = inject_fault(SEEDS_FAULT_ALLOC) ? hipErrorOutOfMemory : hipMalloc(&sv->slab, off);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sv->ring_host, kRing * sv->ring_bytes, 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sv->flag_host, 64, 0);
    if (e == hipSuccess) *sv->flag_host = 0;
    for (int i = 0; e == hipSuccess && i < kRing; ++i) {
        e = hipEventCreateWithFlags(&sv->ring_ev[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->gate[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->copy, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        seeds_server_destroy(sv);
        return sfail(e == hipErrorOutOfMemory ? SEEDS_E_NOMEM : SEEDS_E_DEVICE,
                     "server set-up (%zu device bytes): %s", off, hipGetErrorString(e));
    }
    char *base = (char *)sv->slab;
    sv->px_base = (uint8_t *)(base + o_px);
    sv->ar.bins = sv->px_base;
    sv->ar.lab = (int32_t *)sv->px_base;
    sv->ar.bl = (int32_t *)sv->px_base;
    sv->ar.state[0] = (int32_t *)(base + o_st);
    sv->ar.state[1] = sv->ar.state[0] + sv->st_size;
    sv->ar.src = (int32_t *)(base + o_dummy);   // block decisions of the exact rule only:
    sv->ar.pend = (int32_t *)(base + o_dummy);  // never touched under Prop. 1
    sv->ar.log = (int2 *)(base + o_log);
    sv->ar.log_n = (int32_t *)(base + o_logn);
    sv->ar.sync = (uint32_t *)(base + o_sync);
    sv->ring_dev = (uint8_t *)(base + o_ring);
    e = launch_fill((int32_t *)sv->ar.sync, 0, 4, sv->s);
    if (e == hipSuccess) e = hipStreamSynchronize(sv->s);
    if (e != hipSuccess) {
        seeds_server_destroy(sv);
        return sfail(SEEDS_E_DEVICE, "server set-up: %s", hipGetErrorString(e));
    }
    sv->stats.budget_bytes = p->hbm_budget_bytes;
    *out = sv;
    return SEEDS_OK;
}

seeds_status seeds_server_submit(seeds_server *sv, const uint8_t *rgb, int32_t H, int32_t W,
                                 int64_t row_pitch_bytes, int32_t num_superpixels, int32_t levels,
                                 int32_t *labels_out, int32_t out_is_host, int64_t *request_id) {
    if (!sv) return sfail(SEEDS_E_INVAL, "server is NULL");
    if (sv->poisoned) return sfail(SEEDS_E_STATE, "server is poisoned by an earlier device error");
    if (!rgb || !labels_out) return sfail(SEEDS_E_INVAL, "rgb or labels_out is NULL");
    if (levels > sv->p.max_levels)
        return sfail(SEEDS_E_INVAL, "levels %d above the server's max_levels %d", levels,
                     sv->p.max_levels);
    seeds_params q;
    q.levels = levels;
    q.bins_per_channel = sv->p.bins_per_channel;
    q.iters_per_level = sv->p.iters_per_level;
    q.gamma = sv->p.gamma;
    q.block_rule = SEEDS_BLOCK_INTERSECT;
    // reuse the single-image checks (grid, sizes) through a throw-away grid call
    int32_t gx, gy;
    seeds_status st = seeds_grid(H, W, num_superpixels, levels, &gx, &gy);
    if (st != SEEDS_OK) return st;  // seeds_grid has set the error text
    if (row_pitch_bytes < 3 * (int64_t)W)
        return sfail(SEEDS_E_INVAL, "row pitch %lld < 3 W", (long long)row_pitch_bytes);
    Request *r = new (std::nothrow) Request();
    if (!r) return sfail(SEEDS_E_NOMEM, "host allocation failed");
    Dims &d = r->d;
    d.H = H;
    d.W = W;
    d.B = q.bins_per_channel;
    d.nb = d.B * d.B * d.B;
    d.hs = hist_stride(d.nb);
    d.L = levels;
    d.I = q.iters_per_level;
    d.gamma = q.gamma;
    d.rule = SEEDS_BLOCK_INTERSECT;
    d.gx = gx;
    d.gy = gy;
    d.K = gx * gy;
    d.T = 1 << (levels - 1);
    r->px_len = pixel_bytes(d);
    r->st_len = state_elems(d);
    r->groups_max = max_phase_groups(d, sv->tune.items);
    if (r->px_len > sv->px_size || r->st_len > sv->st_size || r->groups_max > sv->g_cap) {
        delete r;
        return sfail(SEEDS_E_INVAL, "a %d x %d image does not fit the server's memory budget", W, H);
    }
    hipError_t e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete r;
        return sfail(SEEDS_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
    r->id = sv->next_id++;
    r->rgb = rgb;
    r->pitch = row_pitch_bytes;
    r->out = labels_out;
    r->out_host = out_is_host != 0;
    r->out_dev = nullptr;
    if (r->out_host) {
        // pinned, device-visible host memory takes a narrow copy kernel;
        // anything else (pageable memory) a plain asynchronous copy
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, labels_out) == hipSuccess &&
            attr.type == hipMemoryTypeHost && attr.devicePointer)
            r->out_dev = (int32_t *)attr.devicePointer;
        (void)hipGetLastError();  // a pageable pointer leaves an error behind
    }
    r->finish_tick = -1;
    r->reported = false;
    sv->queue.push_back(r);
    sv->stats.submitted++;
    if (request_id) *request_id = r->id;
    return SEEDS_OK;
}

seeds_status seeds_server_step(seeds_server *sv, int32_t *pending) {
    if (!sv) return sfail(SEEDS_E_INVAL, "server is NULL");
    TraceRange tr("seeds server tick %d", (int)sv->tick);
    if (sv->poisoned) return sfail(SEEDS_E_STATE, "server is poisoned by an earlier device error");
    hipStream_t s = sv->s;
    const int64_t t = sv->tick;
    // memory of images whose last phase ran two ticks ago (its deltas were
    // added in the tick after it) goes back to the pool
    for (auto it = sv->finishing.begin(); it != sv->finishing.end();) {
        Request *r = *it;
        if (r->finish_tick <= t - 2) {
            hipError_t e = release_request(sv, r);
            if (e != hipSuccess) return srv_device_error(sv, e, "stream wait");
            it = sv->finishing.erase(it);
            if (r->reported) destroy_request(r);
        } else {
            ++it;
        }
    }
    // admission in arrival order
    std::vector<Request *> admitted;
    while (!sv->queue.empty() && try_admit(sv, sv->queue.front())) {
        admitted.push_back(sv->queue.front());
        sv->running.push_back(sv->queue.front());
        sv->queue.pop_front();
    }
    sv->stats.admitted += (int64_t)admitted.size();
    // this tick's items
    const int slot = (int)(t % kRing);
    if (sv->ring_used[slot]) {
        hipError_t e = hipEventSynchronize(sv->ring_ev[slot]);
        if (e != hipSuccess) return srv_device_error(sv, e, "tick ring wait");
    }
    TickItem *items = (TickItem *)(sv->ring_host + slot * sv->ring_bytes);
    int n = 0;
    auto add = [&](const Request *r, int level, int cls, int first, int groups) {
        TickItem &it = items[n++];
        it.g = r->g;
        it.rgb = r->rgb;
        it.pitch = r->pitch;
        it.level = level;
        it.cls = cls;
        it.first = first;
        it.groups = groups;
    };
    const int zero0 = n;
    int zero_groups_total = 0;
    for (Request *r : admitted) {
        add(r, 0, 0, zero_groups_total, zero_groups(r->d));
        zero_groups_total += zero_groups(r->d);
    }
    const int init0 = n;
    int init_groups_total = 0;
    for (Request *r : admitted) {
        add(r, 0, 0, init_groups_total, init_groups(r->d));
        init_groups_total += init_groups(r->d);
    }
    const int desc0 = n;
    int desc_groups_total = 0;
    std::vector<std::pair<Request *, std::pair<int, int>>> phase_of;  // (level, cls)
    std::vector<Request *> finished_now;
    for (Request *r : sv->running) {
        int cls = 0;
        SchedOp op = sched_next(r->d, r->sc, -1, &cls);
        if (op == OP_DESCEND) {
            const int gr = descend_groups(r->d, r->sc.level);
            add(r, r->sc.level, 0, desc_groups_total, gr);
            desc_groups_total += gr;
            sched_done(r->sc, op);
            op = sched_next(r->d, r->sc, -1, &cls);
        }
        if (op == OP_PHASE) {
            phase_of.push_back({r, {r->sc.level, cls}});
            sched_done(r->sc, op);
        }
        Sched peek = r->sc;
        int c2;
        if (op != OP_PHASE || sched_next(r->d, peek, -1, &c2) == OP_END) finished_now.push_back(r);
    }
    // phase items: pixel-level ones, then block-level ones (two launches)
    const int phase0 = n;
    int pixel_groups = 0, block_groups = 0, max_level = 0;
    for (auto &pr : phase_of) {
        if (pr.second.first != 0) continue;
        const int gr = phase_launch_groups(pr.first->d, 0, pr.second.second, sv->tune.items);
        if (gr == 0) continue;
        add(pr.first, 0, pr.second.second, pixel_groups, gr);
        pixel_groups += gr;
    }
    const int block0 = n;
    for (auto &pr : phase_of) {
        if (pr.second.first == 0) continue;
        const int gr =
            phase_launch_groups(pr.first->d, pr.second.first, pr.second.second, sv->tune.items);
        if (gr == 0) continue;
        add(pr.first, pr.second.first, pr.second.second, block_groups, gr);
        block_groups += gr;
        max_level = std::max(max_level, pr.second.first);
    }
    const int phase_groups_total = pixel_groups + block_groups;
    // coarse indexes of the four lists, after the items in the same slot
    int32_t *coarse_host = (int32_t *)(sv->ring_host + slot * sv->ring_bytes + sv->items_bytes);
    int ncoarse_used = 0;
    const uint8_t *slot_dev = sv->ring_dev + slot * sv->ring_bytes;
    const TickItem *dev_items = (const TickItem *)slot_dev;
    const int32_t *dev_coarse = (const int32_t *)(slot_dev + sv->items_bytes);
    auto make_list = [&](int i0, int i1, int groups) {
        TickList l;
        l.items = dev_items + i0;
        l.n = i1 - i0;
        l.coarse = nullptr;
        l.ncoarse = 0;
        l.hs = hist_stride(sv->p.bins_per_channel * sv->p.bins_per_channel * sv->p.bins_per_channel);
        const int nc = (groups + kTickCoarse - 1) / kTickCoarse;
        if (l.n > 1 && ncoarse_used + nc <= kCoarseCap) {
            int it = i0;
            for (int c = 0; c < nc; ++c) {
                const int lg = c * kTickCoarse;
                while (it + 1 < i1 && items[it + 1].first <= lg) ++it;
                coarse_host[ncoarse_used + c] = it - i0;
            }
            l.coarse = dev_coarse + ncoarse_used;
            l.ncoarse = nc;
            ncoarse_used += nc;
        }
        return l;
    };
    const TickList zero_l = make_list(zero0, init0, zero_groups_total);
    const TickList init_l = make_list(init0, desc0, init_groups_total);
    const TickList desc_l = make_list(desc0, phase0, desc_groups_total);
    const TickList pixel_l = make_list(phase0, block0, pixel_groups);
    const TickList block_l = make_list(block0, n, block_groups);
    hipError_t e = hipSuccess;
    if (n > 0)
        e = hipMemcpyAsync((void *)dev_items, items, n * sizeof(TickItem), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && ncoarse_used > 0)
        e = hipMemcpyAsync((void *)dev_coarse, coarse_host, ncoarse_used * sizeof(int32_t),
                           hipMemcpyHostToDevice, s);
    const BatchArgs b = server_args(sv);
    if (e == hipSuccess && n > 0 && inject_fault(SEEDS_FAULT_LAUNCH)) e = hipErrorLaunchFailure;
    if (e == hipSuccess && zero_groups_total > 0)
        e = launch_zero_mixed(b, zero_l, zero_groups_total, s);
    if (e == hipSuccess && init_groups_total > 0)
        e = launch_init_mixed(b, init_l, init_groups_total, s);
    if (e == hipSuccess && desc_groups_total > 0)
        e = launch_descend_mixed(b, desc_l, desc_groups_total, s);
    if (e == hipSuccess) {
        if (phase_groups_total > 0) {
            // the first launch of the tick adds the previous tick's deltas
            int replay = sv->prev_groups;
            if (pixel_groups > 0) {
                e = launch_phase_mixed(b, pixel_l, true, 0, sv->par, pixel_groups, replay, 0,
                                       sv->tune, s);
                replay = 0;
            }
            if (e == hipSuccess && block_groups > 0)
                e = launch_phase_mixed(b, block_l, false, max_level, sv->par, block_groups, replay,
                                       pixel_groups, sv->tune, s);
            sv->prev_groups = phase_groups_total;
            sv->par ^= 1;
        } else if (sv->prev_groups > 0) {
            // nothing to decide: the previous phase's deltas go to the copy it read
            e = launch_final_replay(b, sv->par ^ 1, sv->prev_groups, s);
            sv->prev_groups = 0;
        }
    }
    // labels of the images whose schedule ended in this tick, copied on the
    // copy stream once this tick's kernels are done
    if (e == hipSuccess && !finished_now.empty()) {
        e = hipEventRecord(sv->gate[slot], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(sv->copy, sv->gate[slot], 0);
    }
    for (Request *r : finished_now) {
        if (e != hipSuccess) break;
        const size_t bytes = (size_t)r->d.H * r->d.W * 4;
        if (r->out_dev)
            e = launch_copy_out(r->out_dev, sv->ar.lab + r->g.lab, (int64_t)r->d.H * r->d.W,
                                sv->copy);
        else
            e = hipMemcpyAsync(r->out, sv->ar.lab + r->g.lab, bytes,
                               r->out_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                               sv->copy);
        if (e == hipSuccess) e = hipEventRecord(r->done, sv->copy);
        r->finish_tick = t;
        sv->finishing.push_back(r);
        sv->unreported.push_back(r);
        sv->running.erase(std::find(sv->running.begin(), sv->running.end(), r));
    }
    // with the labels, the kernels' error flag (a full move log) comes back
    if (e == hipSuccess && !finished_now.empty())
        e = hipMemcpyAsync(sv->flag_host, sv->ar.sync + 2, 4, hipMemcpyDeviceToHost, sv->copy);
    if (e == hipSuccess) e = hipEventRecord(sv->ring_ev[slot], s);
    if (e != hipSuccess) return srv_device_error(sv, e, "tick launch");
    sv->ring_used[slot] = true;
    sv->tick++;
    sv->stats.ticks++;
    sv->stats.peak_inflight = std::max<int64_t>(sv->stats.peak_inflight, (int64_t)sv->running.size());
    if (pending)
        *pending = (int32_t)(sv->queue.size() + sv->running.size() + sv->finishing.size());
    return SEEDS_OK;
}

seeds_status seeds_server_poll(seeds_server *sv, int64_t *done_ids, int32_t max_ids,
                               int32_t *n_done) {
    if (n_done) *n_done = 0;
    if (!sv || !n_done || (max_ids > 0 && !done_ids))
        return sfail(SEEDS_E_INVAL, "NULL argument");
    if (sv->poisoned) return sfail(SEEDS_E_STATE, "server is poisoned by an earlier device error");
    int k = 0;
    for (auto it = sv->unreported.begin(); it != sv->unreported.end() && k < max_ids;) {
        Request *r = *it;
        hipError_t q = hipEventQuery(r->done);
        if (q == hipErrorNotReady) {
            ++it;
            continue;
        }
        if (q != hipSuccess) return srv_device_error(sv, q, "request completion");
        done_ids[k++] = r->id;
        r->reported = true;
        sv->stats.completed++;
        it = sv->unreported.erase(it);
        if (std::find(sv->finishing.begin(), sv->finishing.end(), r) == sv->finishing.end())
            destroy_request(r);
    }
    *n_done = k;
    // the error flag as copied back with the last labels that are complete
    if (k > 0 && __atomic_load_n(sv->flag_host, __ATOMIC_ACQUIRE)) {
        sv->poisoned = true;
        return sfail(SEEDS_E_DEVICE, "move log overflow");
    }
    return SEEDS_OK;
}

seeds_status seeds_server_get_stats(const seeds_server *sv, seeds_server_stats *out) {
    if (!sv || !out) return sfail(SEEDS_E_INVAL, "NULL argument");
    *out = sv->stats;
    out->queued = (int64_t)sv->queue.size();
    out->inflight = (int64_t)sv->running.size();
    return SEEDS_OK;
}

seeds_status seeds_server_destroy(seeds_server *sv) {
    if (!sv) return SEEDS_OK;
    hipError_t e = hipStreamSynchronize(sv->s);
    if (sv->copy) {
        hipError_t e2 = hipStreamSynchronize(sv->copy);
        if (e == hipSuccess) e = e2;
    }
    std::vector<Request *> all(sv->queue.begin(), sv->queue.end());
    all.insert(all.end(), sv->running.begin(), sv->running.end());
    all.insert(all.end(), sv->finishing.begin(), sv->finishing.end());
    for (Request *r : sv->unreported)
        if (std::find(all.begin(), all.end(), r) == all.end()) all.push_back(r);
    for (Request *r : all) destroy_request(r);
    for (auto &ev : sv->ring_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &ev : sv->gate)
        if (ev) (void)hipEventDestroy(ev);
    if (sv->copy) (void)hipStreamDestroy(sv->copy);
    if (sv->ring_host) (void)hipHostFree(sv->ring_host);
    if (sv->flag_host) (void)hipHostFree(sv->flag_host);
    if (sv->slab) (void)hipFree(sv->slab);
    delete sv;
    if (e != hipSuccess) return sfail(SEEDS_E_DEVICE, "destroy: %s", hipGetErrorString(e));
    return SEEDS_OK;
}

}  // extern "C"
