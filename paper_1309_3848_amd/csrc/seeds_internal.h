// Internal declarations shared by the host side (seeds_capi.cpp) and the
// kernels of libseeds.
//
// Every context is a batch of one or more images. Their buffers live in
// pooled arenas; an ImageDesc gives each image's dimensions and offsets. One
// phase launch processes the same phase (level, class) of every image that
// takes part at that step of the schedule; a device array per launch maps
// each workgroup to its image and its rank among that image's workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "seeds.h"

namespace seeds {

// Record the text of a failure for seeds_last_error() on this thread and
// return st.
seeds_status set_error(seeds_status st, const char *fmt, ...);

// Fault injection (seeds_debug_inject_fault): true when the next operation of
// this kind must fail instead of running. kind: SEEDS_FAULT_ALLOC for device
// allocations, SEEDS_FAULT_LAUNCH for kernel launches of contexts and servers.
bool inject_fault(int kind);

// Histogram rows are padded so every row starts on a 32-byte boundary.
__host__ __device__ inline int hist_stride(int nbins) { return (nbins + 7) & ~7; }

struct Dims {
    int H, W;        // image
    int B, nb, hs;   // bins per channel, B^3, padded histogram row stride
    int L, I;        // levels, sweeps per level
    int gamma, rule;
    int gx, gy, K;   // superpixel grid, K = gx * gy
    int T;           // top block side 2^(L-1)
};

// Unit grid of level l: ceil(W / 2^l) x ceil(H / 2^l).
__host__ __device__ inline int units_w(const Dims &d, int level) { return (d.W + (1 << level) - 1) >> level; }
__host__ __device__ inline int units_h(const Dims &d, int level) { return (d.H + (1 << level) - 1) >> level; }

// Number of units of class c (3 (uy mod 3) + (ux mod 3)) on a uw x uh grid.
__host__ __device__ inline int class_cols(int uw, int cls) { return cls % 3 < uw ? (uw - cls % 3 + 2) / 3 : 0; }
__host__ __device__ inline int class_rows(int uh, int cls) { return cls / 3 < uh ? (uh - cls / 3 + 2) / 3 : 0; }
__host__ __device__ inline int class_units(const Dims &d, int level, int cls) {
    return class_cols(units_w(d, level), cls) * class_rows(units_h(d, level), cls);
}

// Schedule (Sec. 5.2): levels L-1 .. 0, I sweeps per level, nine classes
// per sweep. `level` is the level whose unit grid currently holds the labels;
// (cur_level, cur_sweep, cur_class) is the next phase; cur_level < 0 once the
// schedule is exhausted (the labels are then brought down to pixel level).
struct Sched {
    int level;
    int cur_level, cur_sweep, cur_class;
};

enum SchedOp { OP_END = 0, OP_DESCEND = 1, OP_PHASE = 2 };

// Next operation of the schedule; phases_left < 0 means no limit. Returns
// OP_PHASE with the phase's class in *cls. The caller executes the op and
// then calls sched_done(op).
__host__ __device__ inline SchedOp sched_next(const Dims &d, Sched &s, int phases_left, int *cls) {
    for (;;) {
        if (s.cur_level < 0) return s.level > 0 ? OP_DESCEND : OP_END;
        if (s.cur_sweep >= d.I) {
            --s.cur_level;
            s.cur_sweep = 0;
            s.cur_class = 0;
            continue;
        }
        if (phases_left == 0) return OP_END;
        if (s.level > s.cur_level) return OP_DESCEND;
        *cls = s.cur_class;
        return OP_PHASE;
    }
}

__host__ __device__ inline void sched_done(Sched &s, SchedOp op) {
    if (op == OP_DESCEND) {
        --s.level;
    } else if (op == OP_PHASE) {
        if (++s.cur_class == 9) {
            s.cur_class = 0;
            ++s.cur_sweep;
        }
    }
}

// One image of a context: its dimensions and its offsets into the arenas.
// The block grid of level l >= 1 lives in block-grid buffer l % 2.
struct ImageDesc {
    Dims d;
    int64_t bins;      // byte offset into the bins arena (H * W)
    int64_t lab;       // element offset into the label arena (H * W)
    int64_t bl[2];     // element offsets into the block-grid arena
    int64_t state;     // element offset into each state copy: K * hs cells, then K sizes
    int64_t src;       // element offset into the source-stamp arena (K)
    int64_t pend;      // element offset into the decision arena (largest class)
};

// Pixel labels are stored as 16-bit values when every image of a context has
// at most kLab16MaxK superpixels (labels 0 .. 65534), halving the bytes the
// pixel phases read; otherwise as int32. Block grids are always int32.
constexpr int kLab16MaxK = 65535;

// Arenas of a context.
struct Arenas {
    uint8_t *bins;
    int32_t *lab;       // pixel labels (int32), or nullptr when lab16 is used
    uint16_t *lab16;    // pixel labels (16-bit), or nullptr
    int32_t *bl;
    int32_t *state[2];  // two equal copies between launches; phases alternate them
    int32_t *src;       // phase stamps of move sources (exact rule's drop rule)
    int32_t *pend;      // exact rule: one decision per class unit
    int2 *log;          // per-workgroup delta logs: [2 parities][log_groups][log_cap]
    int32_t *log_n;     // entries in each log: [2][log_groups]
    uint32_t *sync;     // persistent kernel: barrier count, generation, error flag
};

// One image's share of a mixed launch (the serving engine): its descriptor,
// what it does in the launch and which logical workgroups do it. Items of a
// launch are sorted by `first` and none is empty.
struct TickItem {
    ImageDesc g;
    const uint8_t *rgb;  // init items: the image's pixels
    int64_t pitch;
    int level, cls;      // phase items: the phase; descend items: the level left
    int first, groups;   // logical workgroups [first, first + groups)
};

// The items of one mixed launch and a coarse index into them: coarse[c] is
// the item holding logical workgroup c * kTickCoarse (nullptr: none, the
// lookup searches all items).
constexpr int kTickCoarse = 32;
struct TickList {
    const TickItem *items;
    const int32_t *coarse;
    int n;       // items
    int ncoarse; // coarse entries
    int hs;      // histogram row stride (shared by every image of a server)
};

// Index of the item that holds logical workgroup lg: the last item whose
// first workgroup is <= lg, searched between the coarse bounds.
__host__ __device__ inline int find_tick_item(const TickList &l, int lg) {
    int lo = 0, hi = l.n - 1;
    if (l.coarse) {
        const int c = lg / kTickCoarse;
        lo = l.coarse[c];
        if (c + 1 < l.ncoarse) hi = l.coarse[c + 1];
    }
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (l.items[mid].first <= lg) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Device view of a whole context for one launch.
struct BatchArgs {
    const ImageDesc *imgs;  // device array, nimg entries
    int nimg;
    Arenas ar;
    int log_cap;
    int log_groups;
    int items = 1;  // phase work items per workgroup (batch maps count workgroups with it)
    int bppl = 1;   // pixels per lane of the block levels 1-3 (1 or 4; batch maps count with it)
};

constexpr int kPersistentThreads = 256;

// Segment shape of block level l (side s = 2^l): SEG lanes per block, PPL
// pixels per lane, SEG * PPL = s * s. bppl (a tuning choice) is the number
// of pixels per lane at levels 1-3: 1 gives one lane per pixel (at most one
// block per wavefront at side 8), 4 gives four times as many blocks per
// wavefront, whose loads are then in flight together. Larger blocks always
// take 64 lanes.
__host__ __device__ inline int seg_lanes(int level, int bppl = 1) {
    if (bppl == 4 && level <= 3) return 1 << (2 * level - 2);
    return level >= 3 ? 64 : 1 << (2 * level);
}
__host__ __device__ inline int seg_ppl(int level, int bppl = 1) {
    if (bppl == 4 && level <= 3) return 4;
    return level >= 3 ? 1 << (2 * level - 6) : 1;
}
// How a segment finds the count h_l(j) of each bin j of its block:
//   0 in registers (shuffles among at most 16 pixels),
//   1 in one LDS histogram row per segment (16 to 64 pixels),
//   2 from the block's bins staged in LDS (more than 64 pixels).
__host__ __device__ constexpr int bin_count_kind(int seg, int ppl) {
    if (seg == 64 && ppl > 1) return 2;
    return seg * ppl > 16 || seg >= 16 ? 1 : 0;
}

// Dynamic LDS of a block phase at `level` (hs: histogram row stride): the
// staged bins (one byte per pixel) or the histogram rows.
__host__ __device__ inline int phase_lds_bytes(int level, int hs, int bppl = 1) {
    if (level == 0) return 0;
    const int seg = seg_lanes(level, bppl), ppl = seg_ppl(level, bppl);
    switch (bin_count_kind(seg, ppl)) {
        case 2: return kPersistentThreads * ppl;
        case 1: return (kPersistentThreads / seg) * hs * 4;
        default: return 0;
    }
}
// The most any level up to max_level needs.
__host__ __device__ inline int phase_lds_bytes_upto(int max_level, int hs, int bppl = 1) {
    int b = 0;
    for (int l = 1; l <= max_level; ++l) {
        const int x = phase_lds_bytes(l, hs, bppl);
        b = b > x ? b : x;
    }
    return b;
}

// Pixel phases work on tiles of kPixTX x kPixTY class pixels, one wavefront
// per class row of the tile. A tile's pixels sit 3 apart, and their 5x5
// windows together cover kWinH x kWinW image cells, which the workgroup
// stages in LDS.
constexpr int kPixTX = 64, kPixTY = kPersistentThreads / kPixTX;
constexpr int kWinW = 3 * kPixTX + 2, kWinH = 3 * kPixTY + 2;
__host__ __device__ inline int pixel_tiles_x(const Dims &d, int cls) {
    return (class_cols(d.W, cls) + kPixTX - 1) / kPixTX;
}
__host__ __device__ inline int pixel_tiles(const Dims &d, int cls) {
    return pixel_tiles_x(d, cls) * ((class_rows(d.H, cls) + kPixTY - 1) / kPixTY);
}

// Work items of one phase of class cls for an image (pixel tiles, or rounds of
// kPersistentThreads / seg_lanes(level) blocks): one workgroup each in a
// phase launch.
__host__ __device__ inline int phase_groups(const Dims &d, int level, int cls, int bppl = 1) {
    if (level == 0) return pixel_tiles(d, cls);
    const int per = kPersistentThreads / seg_lanes(level, bppl);
    return (class_units(d, level, cls) + per - 1) / per;
}

// Workgroups of one image in a phase launch that gives each workgroup `items`
// work items (the last one may get fewer).
__host__ __device__ inline int phase_launch_groups(const Dims &d, int level, int cls, int items,
                                                   int bppl = 1) {
    return (phase_groups(d, level, cls, bppl) + items - 1) / items;
}

// Upper bound on the log entries (deltas) one workgroup produces in one work
// item of a phase at `level`.
__host__ __device__ inline int deltas_per_round(const Dims &d, int level, int bppl = 1) {
    if (level == 0) return 2 * kPersistentThreads;
    const int segs = kPersistentThreads / seg_lanes(level, bppl);
    const int bins = (1 << (2 * level)) < d.nb ? (1 << (2 * level)) : d.nb;
    return segs * (2 * bins + 2);
}

// Workgroups of one descend launch for an image and of one init launch.
// A descend workgroup copies one row chunk of up to 256 units of `level` to
// their children.
__host__ __device__ inline int descend_groups(const Dims &d, int level) {
    const int fw = units_w(d, level), fh = units_h(d, level);
    return fh * ((fw + kPersistentThreads - 1) / kPersistentThreads);
}
// Initialisation and warm-start tiles: kInitTW x rows pixels, rows in
// {8, 16, 32} (a tuning choice; kInitTH by default).
constexpr int kInitTW = 64, kInitTH = 16, kMaxInitTH = 32;
__host__ __device__ inline int init_groups(const Dims &d, int rows = kInitTH) {
    return ((d.W + kInitTW - 1) / kInitTW) * ((d.H + rows - 1) / rows);
}

// Persistent-kernel launch geometry, fixed per single-image context.
struct PersistentGeom {
    int groups;     // co-resident workgroups
    int log_cap;    // log entries per workgroup and phase parity
    int lds_bytes;  // dynamic LDS for staging block bins
};

// Launchers. They only enqueue work and return the launch status; shapes are
// checked by the caller. For a single image (b.nimg == 1) the launch uses
// `one` and needs no map; for a batch, map[logical workgroup] = (image, rank
// of the workgroup among that image's workgroups of the launch) and `groups`
// is the launch's total.
hipError_t launch_fill(int32_t *p, int32_t v, int64_t n, hipStream_t s);
// n int32 from src to dst, both in device memory, by the copy-out kernel
// spread over the whole device (a runtime copy when src is not 16-byte
// aligned).
hipError_t launch_copy(int32_t *dst, const int32_t *src, int64_t n, hipStream_t s);
// n pixel labels of an arena (int32 or 16-bit, at element offset `at`) to
// int32 device memory, over the whole device.
hipError_t launch_copy_labels(int32_t *dst, const Arenas &a, int64_t at, int64_t n, hipStream_t s);
// n int32 labels (values < 65536) into the 16-bit plane at element offset at.
hipError_t launch_narrow_labels(const Arenas &a, int64_t at, const int32_t *src, int64_t n,
                                hipStream_t s);
hipError_t launch_init(const BatchArgs &b, const ImageDesc &one, const uint8_t *rgb_one,
                       int64_t pitch_one, const int2 *map, const uint8_t *const *rgb_table,
                       const int64_t *pitch_table, int groups, int rows, hipStream_t s);
// One phase as one launch. pass: 0 decide and apply, 1 exact-rule decide
// only, 2 exact-rule apply. replay_groups: workgroups of the previous phase
// launch, whose logs (parity par ^ 1) this launch adds to its write copy.
// max_level: the largest level of any image (selects the kernel variant).
// Mapping choices of the per-phase launches (results never depend on them).
struct PhaseTuning {
    bool pixel_compact = false;  // pixel phases: pre-test and compaction
    bool xcd_remap = true;      // workgroups numbered in contiguous bands per XCD
    int items = 1;              // work items (pixel tiles, block rounds) per workgroup: 1, 2, 4
    int init_rows = kInitTH;    // rows of an initialisation tile: 8, 16, 32
    int warm_rows = kInitTH;    // rows of a warm-start tile: 8, 16, 32
    int block_ppl = 1;          // pixels per lane at block levels 1-3: 1, 4
};
constexpr int kItemChoices[3] = {1, 2, 4};
constexpr int kPplChoices[2] = {1, 4};
__host__ __device__ inline int ppl_index(int bppl) { return bppl == 4 ? 1 : 0; }
constexpr int kRowChoices[3] = {8, 16, 32};
__host__ __device__ inline int item_index(int items) { return items == 4 ? 2 : items == 2 ? 1 : 0; }
__host__ __device__ inline int row_index(int rows) { return rows == 32 ? 2 : rows == 8 ? 0 : 1; }
hipError_t launch_phase(const BatchArgs &b, const ImageDesc &one, const int2 *map, int max_level,
                        int level, int cls, int par, int pass, uint32_t stamp, int groups,
                        int replay_groups, const PhaseTuning &tune, hipStream_t s);
// Add the logs of the last phase launch (parity par, `groups` slots) to the
// copy that phase read.
hipError_t launch_final_replay(const BatchArgs &b, int par, int groups, hipStream_t s);
// Split every block of `level` into its 2x2 children (level 1: pixel labels).
hipError_t launch_descend(const BatchArgs &b, const ImageDesc &one, const int2 *map, int level,
                          int groups, hipStream_t s);
// Sizes from the histograms of one image (pixel phases do not maintain them).
hipError_t launch_sizes(const Dims &d, int32_t *state0, int32_t *state1, hipStream_t s);
// Pixel labels of one image from the unit grid of `level`.
// Warm start: bins from new frames and histograms and sizes recounted from
// the current pixel labels (both state copies must be zero). Same workgroup
// map and tables as launch_init.
hipError_t launch_rehist(const BatchArgs &b, const ImageDesc &one, const uint8_t *rgb_one,
                         int64_t pitch_one, const int2 *map, const uint8_t *const *rgb_table,
                         const int64_t *pitch_table, int groups, int rows, hipStream_t s);
hipError_t launch_expand(const Dims &d, const int32_t *units, int level, int32_t *out,
                         hipStream_t s);

// Quality metrics (overlap table of K x R int32 and six 64-bit counters,
// both zeroed here): UE, ASA and CUE numerators, BR hits, |B(g)|, and the
// number of out-of-range values.
hipError_t launch_quality(const int32_t *lab, const int32_t *gt, int H, int W, int K, int R,
                          int eps, int32_t *table, unsigned long long *cnt, hipStream_t s);

// Mixed launches of the serving engine: every item is one image. Phase items
// run their own (level, class) with the Prop. 1 rule, all of them at pixel
// level (pixel = true) or all at block levels up to max_level; replay as in
// launch_phase; the launch's log slots start at slot_base.
hipError_t launch_phase_mixed(const BatchArgs &b, const TickList &l, bool pixel, int max_level,
                              int par, int groups, int replay_groups, int slot_base,
                              const PhaseTuning &tune, hipStream_t s);
hipError_t launch_descend_mixed(const BatchArgs &b, const TickList &l, int groups, hipStream_t s);
// Zero both state copies of every item's image, then initialise it (quantise,
// grid, histograms) from item.rgb.
hipError_t launch_zero_mixed(const BatchArgs &b, const TickList &l, int groups, hipStream_t s);
hipError_t launch_init_mixed(const BatchArgs &b, const TickList &l, int groups, hipStream_t s);
// Workgroups of one image's state-zeroing share.
constexpr int kZeroPerGroup = 4096;
__host__ __device__ inline int zero_groups(const Dims &d) {
    const int64_t n = (int64_t)d.K * d.hs + d.K;
    return (int)((n + kZeroPerGroup - 1) / kZeroPerGroup);
}

// Test hook: out[0] = H' (sum of squared histogram cells of one image, row
// stride d.hs) and out[1] = G' (sum over pixels of the squared label counts of
// their clipped 3x3 patches) of H x W labels; out (two counters) is zeroed here.
hipError_t launch_energy(const int32_t *hist, const Dims &d, const int32_t *lab,
                         unsigned long long *out, hipStream_t s);

// Test hook: out[0] += the boundary units of class cls (< 0: all classes) on
// the unit grid of `level` of an image, out[1] += the pixels they cover (out
// is not cleared here). `units` is the image's grid of units_level >= level;
// finer units take their ancestor's label.
hipError_t launch_boundary(const int32_t *units, const Dims &d, int units_level, int level,
                           int cls, unsigned long long *out, hipStream_t s);

// Copy n int32 from 16-byte-aligned device memory to device-visible pinned
// host memory (dst is the device-side address) with a few workgroups.
hipError_t launch_copy_out(int32_t *dst, const int32_t *src, int64_t n, hipStream_t s);

// Workgroups of one launch: the map (device array of (image, rank) per
// logical workgroup; nullptr for a single image) and their number.
struct LaunchMap {
    const int2 *map = nullptr;
    int groups = 0;
};

// What the per-phase schedule needs of a context. phase_map ([level * 9 +
// cls]) and descend_map ([level]) are nullptr for a single image, whose
// launch shapes follow from `one`.
struct ScheduleArgs {
    BatchArgs b;
    ImageDesc one;
    Dims top;  // shared parameters; L = the most levels of any image
    const LaunchMap *phase_map = nullptr;
    const LaunchMap *descend_map = nullptr;
    int64_t src_elems = 0;
    PhaseTuning tune;
    bool trace = true;  // roctx ranges per level (host side)
};

// Enqueue the schedule from the cursor `sched` as per-phase launches (at most
// max_phases phases; < 0: all), ending with the replay that makes both state
// copies equal again; advances the cursor. *done (may be NULL) receives the
// phases enqueued.
hipError_t enqueue_schedule(const ScheduleArgs &a, Sched &sched, int32_t max_phases,
                            int32_t *done, hipStream_t s);

// Argument checks of seeds_init (every SEEDS_E_INVAL case) and the image's
// dimensions and grid.
seeds_status check_params(int32_t H, int32_t W, int32_t K, const seeds_params *p, Dims *d);

// Persistent cooperative refinement of a single image.
hipError_t launch_refine(const BatchArgs &b, const ImageDesc &one, const PersistentGeom &g,
                         const Sched &start, int max_phases, uint32_t stamp, hipStream_t s);
PersistentGeom persistent_geometry(const Dims &d, int device, int groups_per_cu);

}  // namespace seeds
