// Internal declarations shared by the host side (seeds_capi.cpp) and the
// kernels (seeds_kernels.hip) of libseeds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "seeds.h"

namespace seeds {

// Histogram rows are padded so every row starts on a 32-byte boundary.
inline int hist_stride(int nbins) { return (nbins + 7) & ~7; }

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

struct Buffers {
    uint8_t *bins;     // H*W colour bin of every pixel
    int32_t *lab;      // H*W pixel labels (valid at level 0)
    int32_t *bl[2];    // block-label grids, ping-pong (levels >= 1)
    int32_t *hist[2];  // state copy c: K*hs colour-histogram cells in pixel counts,
                       // immediately followed by the K superpixel sizes; the two
                       // copies are equal between launches and alternate in phases
    int32_t *size[2];  // = hist[c] + K*hs
    int32_t *src;      // K phase stamps of move sources (exact rule's drop rule)
    int32_t *pend;     // one decision per class unit: target label or -1
    int2 *log;         // per-workgroup delta logs, 2 parities x groups x cap (index, delta)
    int32_t *log_n;    // per-phase launches: entries in each log, 2 x groups
    uint32_t *sync;    // persistent kernel: barrier count, generation, error flag
};

// Persistent-kernel launch geometry, fixed per context.
struct PersistentGeom {
    int groups;     // co-resident workgroups
    int log_cap;    // log entries per workgroup and phase parity
    int lds_bytes;  // dynamic LDS for staging block bins
};

constexpr int kPersistentThreads = 256;

// Segment shape of block level l (side s = 2^l): SEG lanes per block, PPL
// pixels per lane, SEG * PPL = s * s.
__host__ __device__ inline int seg_lanes(int level) { return level >= 3 ? 64 : 1 << (2 * level); }
__host__ __device__ inline int seg_ppl(int level) { return level >= 3 ? 1 << (2 * level - 6) : 1; }

// Launchers (seeds_kernels.hip). They only enqueue work and return the launch
// status; shapes are checked by the caller.
hipError_t launch_fill(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_init(const Dims &d, const Buffers &b, const uint8_t *rgb, int64_t pitch,
                       int32_t *top_labels, hipStream_t s);
// One phase as one launch (level >= 0), or the final replay of the last
// phase's logs into the copy it read (level < 0). pass: 0 decide and apply,
// 1 exact-rule decide only, 2 exact-rule apply.
hipError_t launch_phase_kernel(const Dims &d, const Buffers &b, int log_groups, int log_cap,
                               int level, int cls, int par, int pass, uint32_t stamp, int cur_bl,
                               int replay_groups, hipStream_t s);
int phase_groups(const Dims &d, int level, int cls);
hipError_t launch_sizes(const Dims &d, const Buffers &b, hipStream_t s);
void phase_log_shape(const Dims &d, int *groups, int *cap);
hipError_t launch_refine(const Dims &d, const Buffers &b, const PersistentGeom &g,
                         const Sched &start, int cur_bl, int max_phases, uint32_t stamp,
                         hipStream_t s);
PersistentGeom persistent_geometry(const Dims &d, int device, int groups_per_cu);
hipError_t launch_upsample(const int32_t *from, int fw, int fh, int32_t *to, int tw, int th,
                           hipStream_t s);
hipError_t launch_expand(const Dims &d, const int32_t *blab, int level, int32_t *out,
                         hipStream_t s);

}  // namespace seeds
