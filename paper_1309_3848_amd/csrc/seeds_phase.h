// Phase machinery shared by the persistent kernel and the per-phase kernels:
// the pixel phase, the block phase (three passes) and the level transition,
// all with grid-stride loops, plus the move logs that keep the two histogram
// copies in step.
//
// Phase snapshot. Units of one class are at least three units apart, so a
// decision never reads a label that another decision of the same phase
// writes: labels are written in place as soon as a move is taken. The colour
// histograms and sizes exist twice. Phase t reads copy t % 2 (the state after
// phase t-1) and adds its deltas to the other copy, which holds the state
// after phase t-2; the deltas of phase t-1, kept in move logs, are added to
// that copy as well during phase t. Once phase t is complete the other copy
// holds the state after phase t.
#pragma once

#include "seeds_device.h"

namespace seeds {

constexpr int kPT = kPersistentThreads;

struct RefineArgs {
    Dims d;
    const uint8_t *bins;
    int32_t *lab;
    int32_t *bl[2];
    int32_t *hist[2];
    int32_t *size[2];
    int32_t *src;
    int32_t *pend;
    int4 *log;       // move logs: [2 parities][log_groups][log_cap] entries (k, n, j, cnt)
    int32_t *log_n;  // per-phase launches: entries in each log, [2][log_groups]
    int log_cap;
    int log_groups;
    uint32_t *sync;  // [0] arrivals, [1] generation, [2] error flag
    Sched start;
    int cur_bl;
    int max_phases;
    uint32_t stamp;  // stamp of the phase before the first one of this launch
};

// Pointer selection by a run-time index without indexing an array (which would
// put the array in scratch memory).
template <typename T>
__device__ __forceinline__ T *pick(T *const (&two)[2], int i) {
    return i ? two[1] : two[0];
}

__device__ __forceinline__ void log_move(const RefineArgs &a, int4 *mylog, int *s_logn, int k,
                                         int n, int j, int cnt) {
    const int slot = atomicAdd(s_logn, 1);
    if (slot < a.log_cap)
        mylog[slot] = make_int4(k, n, j, cnt);
    else
        __hip_atomic_store(&a.sync[2], 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Move cnt pixels of bin j from superpixel k to n in one histogram copy.
__device__ __forceinline__ void move_counts(int32_t *hist, int32_t *size, int hs, int k, int n,
                                            int j, int cnt) {
    atomicAdd(&hist[(int64_t)n * hs + j], cnt);
    atomicSub(&hist[(int64_t)k * hs + j], cnt);
    atomicAdd(&size[n], cnt);
    atomicSub(&size[k], cnt);
}

__device__ inline void replay(const RefineArgs &a, const int4 *entries, int n, int32_t *hist,
                       int32_t *size) {
    for (int e = threadIdx.x; e < n; e += kPT) {
        const int4 v = entries[e];
        move_counts(hist, size, a.d.hs, v.x, v.y, v.z, v.w);
    }
}

// ---------------------------------------------------------------------------
// Pixel phase: one thread per pixel of the class, grid-stride.
__device__ inline void pixel_phase(const RefineArgs &a, int cls, int par, int4 *mylog, int *s_logn) {
    const Dims &d = a.d;
    const int ncx = class_cols(d.W, cls), ncy = class_rows(d.H, cls);
    const int n = ncx * ncy;
    const int32_t *hR = pick(a.hist, par);
    int32_t *hW = pick(a.hist, par ^ 1);
    int32_t *sW = pick(a.size, par ^ 1);
    for (int i = blockIdx.x * kPT + threadIdx.x; i < n; i += gridDim.x * kPT) {
        const int x = cls % 3 + 3 * (i % ncx), y = cls / 3 + 3 * (i / ncx);
        const PixelMove mv = pixel_decision(d, a.lab, a.bins, hR, x, y);
        if (mv.n < 0) continue;
        a.lab[(int64_t)y * d.W + x] = mv.n;
        move_counts(hW, sW, d.hs, mv.k, mv.n, mv.j, 1);
        log_move(a, mylog, s_logn, mv.k, mv.n, mv.j, 1);
    }
}

// ---------------------------------------------------------------------------
// Block phase. Segments of SEG lanes handle one block each; SEGS = kPT / SEG
// blocks per round, rounds stride over the grid.
//   pass 0: decide and apply at once (Prop. 1 rule; no drop rule)
//   pass 1: exact rule, decide only: record the target and stamp the source
//   pass 2: exact rule, apply the recorded moves whose target is no source
template <int SEG, int PPL>
__device__ inline void block_phase(const RefineArgs &a, int level, int cls, int par, int pass,
                            uint32_t stamp, int32_t *units, uint8_t *sbin, int4 *mylog,
                            int *s_logn) {
    constexpr int SEGS = kPT / SEG;
    constexpr int NPX = SEG * PPL;
    const Dims &d = a.d;
    const int s = 1 << level;
    const int uw = units_w(d, level), uh = units_h(d, level);
    const int ncx = class_cols(uw, cls), ncy = class_rows(uh, cls);
    const int nunits = ncx * ncy;
    const int per_round = gridDim.x * SEGS;
    const int rounds = (nunits + per_round - 1) / per_round;
    const int seg = threadIdx.x / SEG, lane = threadIdx.x % SEG;
    const int32_t *hR = pick(a.hist, par);
    const int32_t *sR = pick(a.size, par);
    int32_t *hW = pick(a.hist, par ^ 1);
    int32_t *sW = pick(a.size, par ^ 1);
    const bool exact = d.rule == SEEDS_BLOCK_EXACT;
    uint8_t *mine = sbin + seg * NPX;
    for (int r = 0; r < rounds; ++r) {
        const int unit = (r * gridDim.x + blockIdx.x) * SEGS + seg;
        const bool in_range = unit < nunits;
        int ux = 0, uy = 0;
        Neighbourhood nb;
        nb.movable = false;
        nb.k = -1;
        nb.nc = 0;
        int target = -1;
        if (in_range) {
            ux = cls % 3 + 3 * (unit % ncx);
            uy = cls / 3 + 3 * (unit / ncx);
            if (pass == 2) {
                target = a.pend[unit];
                if (target >= 0 && a.src[target] == (int32_t)stamp) target = -1;
                nb.movable = target >= 0;
                nb.k = units[(int64_t)uy * uw + ux];
            } else {
                nb = neighbourhood(units, uw, uh, ux, uy);
            }
        }
#pragma unroll 4
        for (int t = 0; t < PPL; ++t) {
            const int q = lane + t * SEG;
            const int x = ux * s + (q & (s - 1)), y = uy * s + (q >> level);
            mine[q] = (nb.movable && x < d.W && y < d.H) ? a.bins[(int64_t)y * d.W + x] : 0xFF;
        }
        __syncthreads();
        if (nb.movable) {
            const int k = nb.k;
            const int64_t m = (int64_t)min(s, d.W - ux * s) * min(s, d.H - uy * s);
            if (pass != 2) {
                // evaluate the candidates
                const int64_t Ak = sR[k];
                int64_t An[4] = {0, 0, 0, 0};
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (c < nb.nc) An[c] = sR[nb.cand[c]];
                int64_t acc[4] = {0, 0, 0, 0}, acc_kl = 0;
#pragma unroll 4
                for (int t = 0; t < PPL; ++t) {
                    const int q = lane + t * SEG;
                    const int j = mine[q];
                    if (j == 0xFF) continue;
                    int cnt = 0;
                    bool first = true;
                    for (int q2 = 0; q2 < NPX; ++q2) {
                        const bool same = mine[q2] == j;
                        cnt += same;
                        first &= !(same && q2 < q);
                    }
                    if (!first) continue;
                    const int64_t hl = cnt;
                    const int64_t hk = hR[(int64_t)k * d.hs + j];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (c >= nb.nc) break;
                        const int64_t hn = hR[(int64_t)nb.cand[c] * d.hs + j];
                        if (exact) {
                            acc[c] += hl * (hn - hk + hl);
                        } else {
                            const int64_t x1 = hn * m, x2 = hl * An[c];
                            acc[c] += x1 < x2 ? x1 : x2;
                        }
                    }
                    if (!exact) {
                        const int64_t x1 = (hk - hl) * m, x2 = hl * (Ak - m);
                        acc_kl += x1 < x2 ? x1 : x2;
                    }
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = segment_sum<SEG>(acc[c]);
                acc_kl = segment_sum<SEG>(acc_kl);
                // every lane holds the sums: every lane takes the same decision
                int64_t bS = acc[0], bA = An[0];
                int bn = nb.cand[0];
#pragma unroll
                for (int c = 1; c < 4; ++c) {
                    if (c >= nb.nc) break;
                    const bool better = exact ? acc[c] > bS : acc[c] * bA > bS * An[c];
                    if (better) {
                        bS = acc[c];
                        bA = An[c];
                        bn = nb.cand[c];
                    }
                }
                const bool accept = exact ? bS > 0 : bS * (Ak - m) > acc_kl * bA;
                target = accept ? bn : -1;
                if (pass == 1) {
                    if (lane == 0) {
                        a.pend[unit] = target;
                        if (target >= 0)
                            __hip_atomic_store(&a.src[k], (int32_t)stamp, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                    target = -1;
                }
            }
            if (target >= 0) {
                // apply: move the block's pixels bin by bin
                if (lane == 0) units[(int64_t)uy * uw + ux] = target;
#pragma unroll 4
                for (int t = 0; t < PPL; ++t) {
                    const int q = lane + t * SEG;
                    const int j = mine[q];
                    if (j == 0xFF) continue;
                    int cnt = 0;
                    bool first = true;
                    for (int q2 = 0; q2 < NPX; ++q2) {
                        const bool same = mine[q2] == j;
                        cnt += same;
                        first &= !(same && q2 < q);
                    }
                    if (!first) continue;
                    move_counts(hW, sW, d.hs, k, target, j, cnt);
                    log_move(a, mylog, s_logn, k, target, j, cnt);
                }
            }
        } else if (in_range && pass == 1 && lane == 0) {
            a.pend[unit] = -1;
        }
        __syncthreads();
    }
}

// BIG = false instantiates block sides up to 8 only (levels <= 4): fewer
// registers and no scratch for the common hierarchies.
template <bool BIG>
__device__ inline void block_phase_any(const RefineArgs &a, int level, int cls, int par, int pass,
                                uint32_t stamp, int32_t *units, uint8_t *sbin, int4 *mylog,
                                int *s_logn) {
    if (!BIG) {
        switch (level) {
            case 1: block_phase<4, 1>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
            case 2: block_phase<16, 1>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
            default: block_phase<64, 1>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
        }
        return;
    }
    switch (level) {
        case 1: block_phase<4, 1>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
        case 2: block_phase<16, 1>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
        case 3: block_phase<64, 1>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
        case 4: block_phase<64, 4>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
        case 5: block_phase<64, 16>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
        case 6: block_phase<64, 64>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
        default: block_phase<64, 256>(a, level, cls, par, pass, stamp, units, sbin, mylog, s_logn); break;
    }
}

// Level transition: every block of `level` splits into its 2x2 children.
__device__ inline void descend(const RefineArgs &a, int level, int cur_bl) {
    const Dims &d = a.d;
    const int fw = units_w(d, level);
    const int32_t *from = pick(a.bl, cur_bl);
    int32_t *to = level == 1 ? a.lab : pick(a.bl, cur_bl ^ 1);
    const int tw = units_w(d, level - 1), th = units_h(d, level - 1);
    const int64_t n = (int64_t)tw * th;
    for (int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPT) {
        const int x = (int)(i % tw), y = (int)(i / tw);
        to[i] = from[(int64_t)(y >> 1) * fw + (x >> 1)];
    }
}


}  // namespace seeds
