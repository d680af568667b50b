// Phase machinery shared by the per-phase kernels and the persistent kernel:
// the pixel phase, the block phase (three passes) and the level transition,
// all with grid-stride loops, and the bookkeeping that keeps the two copies
// of the colour histograms and sizes in step.
//
// Phase snapshot. Units of one class are at least three units apart, so a
// decision never reads a label that another decision of the same phase
// writes: labels are written in place as soon as a move is taken. The colour
// histograms and sizes ("state") exist twice. Phase t reads copy t % 2 (the
// state after phase t-1) and adds its deltas to the other copy, which holds
// the state after phase t-2; the deltas of phase t-1, kept in move logs, are
// added to that copy during phase t as well. Once phase t is complete the
// other copy holds the state after phase t.
//
// Deltas. Each workgroup sums the deltas of its moves in an LDS hash table
// keyed by state index (histogram cell k * hs + j, or size K * hs + k), then
// adds every non-zero sum to the write copy with one global atomic and logs
// it as (index, delta). Neighbouring moves mostly share cells, so this cuts
// the global atomics and the log. Pixel phases leave the sizes alone: only
// the Prop. 1 block rule reads them, and pixel phases come last.
//
// Batches. Each workgroup serves one image: ImageView holds that image's
// dimensions, buffers and state, and the rank of the workgroup among the
// image's workgroups of the launch. Log entries hold global state indices
// (the image's state offset plus the local index), so any workgroup of the
// next launch can add them.
#pragma once

#include <type_traits>

#include "seeds_device.h"

namespace seeds {

constexpr int kPT = kPersistentThreads;

struct ImageView {
    Dims d;
    const uint8_t *bins;
    int32_t *lab;        // pixel labels: int32 plane, or
    uint16_t *lab16;     // the 16-bit plane (exactly one is non-null)
    int32_t *bl;         // block grid buffer 0 of this image; level l is in
    int64_t bl_step;     // buffer l % 2, at bl + (l % 2) * bl_step
    int64_t base;        // global index of this image's state in a state copy
    int32_t *src;
    int32_t *pend;
    int grp;             // rank of this workgroup among the image's workgroups
    int ngroups;         // the image's workgroups in this launch
};

// Selected by arithmetic, not by choosing between two struct fields, which
// the compiler may turn into an indexed load from a stack copy (scratch).
__device__ __forceinline__ int32_t *level_grid(const ImageView &v, int level) {
    return v.bl + (level & 1) * v.bl_step;
}

__device__ __forceinline__ ImageView make_view(const BatchArgs &b, const ImageDesc &g, int grp,
                                               int ngroups) {
    ImageView v;
    v.d = g.d;
    v.bins = b.ar.bins + g.bins;
    v.lab = b.ar.lab ? b.ar.lab + g.lab : nullptr;
    v.lab16 = b.ar.lab16 ? b.ar.lab16 + g.lab : nullptr;
    v.bl = b.ar.bl + g.bl[0];
    v.bl_step = g.bl[1] - g.bl[0];
    v.base = g.state;
    v.src = b.ar.src + g.src;
    v.pend = b.ar.pend + g.pend;
    v.grp = grp;
    v.ngroups = ngroups;
    return v;
}

// View of the only image of a single-image context: its offsets into the
// arenas are all zero (the context lays it out first), so the view needs no
// offset arithmetic and its state base is the constant 0.
__device__ __forceinline__ ImageView single_view(const BatchArgs &b, const ImageDesc &g, int grp,
                                                 int ngroups) {
    ImageView v;
    v.d = g.d;
    v.bins = b.ar.bins;
    v.lab = b.ar.lab;
    v.lab16 = b.ar.lab16;
    v.bl = b.ar.bl;
    v.bl_step = g.bl[1];
    v.base = 0;
    v.src = b.ar.src;
    v.pend = b.ar.pend;
    v.grp = grp;
    v.ngroups = ngroups;
    return v;
}

// The pixel-label plane of a view as the type the kernel variant was built
// for.
template <typename LabT>
__device__ __forceinline__ LabT *label_plane(const ImageView &v);
template <>
__device__ __forceinline__ int32_t *label_plane<int32_t>(const ImageView &v) { return v.lab; }
template <>
__device__ __forceinline__ uint16_t *label_plane<uint16_t>(const ImageView &v) { return v.lab16; }

// Pointer selection by a run-time index without indexing an array (which would
// put the array in scratch memory).
template <typename T>
__device__ __forceinline__ T *pick(T *const (&two)[2], int i) {
    return i ? two[1] : two[0];
}

// ---------------------------------------------------------------------------
// Per-workgroup delta table in LDS (open addressing, linear probing). A
// workgroup's work item produces at most 512-640 deltas and usually far fewer
// distinct keys; a 256-entry table sends the rare overflow straight to the
// write copy and the log, and costs far less to clear and scan than a table
// sized for the worst case (measured: 2048 entries took 11% longer per
// refine of one 1080p image, 16% per batch). The block phases of a batch
// with four pixels per lane and several work items per workgroup use 1024
// entries: their 512 to 1024 blocks per workgroup overflow the small table.
constexpr int kTableBits = 8, kTableBitsMulti = 10;
constexpr int kTableProbes = 64;
constexpr int32_t kEmptyKey = -1;

template <int BITS = kTableBits>
struct DeltaTable {
    static constexpr int kBits = BITS, kSize = 1 << BITS;
    int32_t key[kSize];
    int32_t val[kSize];
    int n;  // log entries written by this workgroup in this phase
};

template <typename Table>
__device__ __forceinline__ void table_clear(Table &t) {
    for (int i = threadIdx.x; i < Table::kSize; i += kPT) {
        t.key[i] = kEmptyKey;
        t.val[i] = 0;
    }
    if (threadIdx.x == 0) t.n = 0;
}

template <typename Table>
__device__ __forceinline__ void log_append(const BatchArgs &b, Table &t, int2 *mylog,
                                           int32_t idx, int32_t delta) {
    const int slot = atomicAdd(&t.n, 1);
    if (slot < b.log_cap)
        mylog[slot] = make_int2(idx, delta);
    else
        __hip_atomic_store(&b.ar.sync[2], 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Add delta to global state index idx. A full neighbourhood in the table sends
// the delta straight to the write copy W and the log.
template <typename Table>
__device__ __forceinline__ void table_add(const BatchArgs &b, Table &t, int32_t *W,
                                          int2 *mylog, int32_t idx, int32_t delta) {
    uint32_t h = ((uint32_t)idx * 2654435761u) >> (32 - Table::kBits);
#pragma nounroll
    for (int p = 0; p < kTableProbes; ++p, h = (h + 1) & (Table::kSize - 1)) {
        const int32_t prev = atomicCAS(&t.key[h], kEmptyKey, idx);
        if (prev == kEmptyKey || prev == idx) {
            atomicAdd(&t.val[h], delta);
            return;
        }
    }
    atomicAdd(&W[idx], delta);
    log_append(b, t, mylog, idx, delta);
}

// After the phase's moves (and a workgroup barrier): one global atomic and one
// log entry per non-zero sum.
template <typename Table>
__device__ __forceinline__ void table_flush(const BatchArgs &b, Table &t, int32_t *W,
                                            int2 *mylog) {
    for (int i = threadIdx.x; i < Table::kSize; i += kPT) {
        const int32_t k = t.key[i], v = t.val[i];
        if (k == kEmptyKey || v == 0) continue;
        atomicAdd(&W[k], v);
        log_append(b, t, mylog, k, v);
    }
}

__device__ __forceinline__ void replay(const int2 *entries, int n, int32_t *W) {
    for (int e = threadIdx.x; e < n; e += kPT) {
        const int2 v = entries[e];
        atomicAdd(&W[v.x], v.y);
    }
}

// ---------------------------------------------------------------------------
// Pixel phase, one tile of kPixTX x kPixTY class pixels per work item. The
// pixels of a class sit 3 apart, so the 5x5 windows of a wavefront's pixels
// overlap and a per-lane gather of each window cell would fetch every cache
// line several times: the workgroup instead loads the tile's whole window
// (kWinH x kWinW labels, -1 outside the image) into LDS with coalesced loads,
// together with its pixels' bins, and reads every window from there.
//
// COMPACT: every thread first makes the cheap 3x3 test, the movable pixels
// (~15%) are packed into a list (ballot + one LDS atomic per wavefront), and
// dense wavefronts then evaluate the gains. Otherwise every thread decides its
// own pixel. Both give the same moves.
struct PixelTile {
    int32_t lab[kWinH * kWinW];
    int n;
    int unit[kPT];  // packed list: thread | bin << 8
};

__device__ __forceinline__ void wave_append(PixelTile &pt, bool take, int value) {
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == __ffsll((unsigned long long)m) - 1) base = atomicAdd(&pt.n, __popcll(m));
    base = __shfl(base, __ffsll((unsigned long long)m) - 1);
    if (take) pt.unit[base + __popcll(m & ((1ull << lane) - 1))] = value;
}

template <bool COMPACT = true, typename LabT = int32_t, typename Table>
__device__ inline void pixel_phase(const BatchArgs &b, const ImageView &v, int cls, int par,
                                   Table &t, int2 *mylog, PixelTile &pt) {
    const Dims &d = v.d;
    LabT *const lab = label_plane<LabT>(v);
    const int cx = cls % 3, cy = cls / 3;
    const int ncx = class_cols(d.W, cls), ncy = class_rows(d.H, cls);
    const int ntx = (ncx + kPixTX - 1) / kPixTX;
    const int ntiles = ntx * ((ncy + kPixTY - 1) / kPixTY);
    const int32_t *hR = pick(b.ar.state, par) + v.base;
    int32_t *W = pick(b.ar.state, par ^ 1);
    const int ci = threadIdx.x % kPixTX, cj = threadIdx.x / kPixTX;
    static_assert(kWinW == 3 * kPixTX + 2 && 2 * kWinH <= 64 && kPT == 4 * kPixTX,
                  "the window load covers 3 kPixTX + 2 columns with four wavefronts");
    // one pixel's move: its label in place, its count from k to n
    auto apply = [&](int x, int y, int j, const PixelMove &mv) {
        lab[(int64_t)y * d.W + x] = (LabT)mv.n;
        table_add(b, t, W, mylog, (int32_t)(v.base + mv.n * d.hs + j), 1);
        table_add(b, t, W, mylog, (int32_t)(v.base + mv.k * d.hs + j), -1);
    };
    for (int tile = v.grp; tile < ntiles; tile += v.ngroups) {
        const int tx = tile % ntx, ty = tile / ntx;
        const int x0 = cx + 3 * kPixTX * tx, y0 = cy + 3 * kPixTY * ty;  // first pixel
        const int gi = tx * kPixTX + ci, gj = ty * kPixTY + cj;
        const bool valid = gi < ncx && gj < ncy;
        const int x = x0 + 3 * ci, y = y0 + 3 * cj;
        // The bin and the window cells: independent loads, all in flight at
        // once. Threads 0 .. 3 kPixTX - 1 load columns 0 .. 3 kPixTX - 1 of every
        // window row, the last wavefront the two right-most columns (no
        // division, so nothing per thread outlives the loads).
        int cell[kWinH];
        int j;
        const bool wide = (int)threadIdx.x < 3 * kPixTX;
        const int wl = (int)threadIdx.x - 3 * kPixTX;
        const int wc = wide ? (int)threadIdx.x : 3 * kPixTX + (wl & 1);
        const int wr = wide ? 0 : wl >> 1;
        const int xx = x0 - 2 + wc;
        const bool in_x = xx >= 0 && xx < d.W;
        if constexpr (!COMPACT) {
            // Unconditional loads from addresses clamped into the image, with
            // out-of-image cells replaced afterwards: a load behind a branch,
            // or into a register preset to a default, is waited for (with every
            // load before it) at the end of its branch. (The compacting variant
            // keeps the branches: it has no registers to spare for this form.)
            j = v.bins[(int64_t)min(y, d.H - 1) * d.W + min(x, d.W - 1)];
            const int xc = min(max(xx, 0), d.W - 1);
            if (wide) {
                if (y0 >= 2 && y0 - 2 + kWinH <= d.H) {
                    // every window row lies in the image: rows from one base
                    const LabT *base = lab + (int64_t)(y0 - 2) * d.W + xc;
#pragma unroll
                    for (int r = 0; r < kWinH; ++r) cell[r] = base[(int64_t)r * d.W];
#pragma unroll
                    for (int r = 0; r < kWinH; ++r)
                        if (!in_x) cell[r] = -1;
                } else {
#pragma unroll
                    for (int r = 0; r < kWinH; ++r)
                        cell[r] = lab[(int64_t)min(max(y0 - 2 + r, 0), d.H - 1) * d.W + xc];
#pragma unroll
                    for (int r = 0; r < kWinH; ++r) {
                        const int yy = y0 - 2 + r;
                        if (!(in_x && yy >= 0 && yy < d.H)) cell[r] = -1;
                    }
                }
            } else {
                const int yy = y0 - 2 + min(wr, kWinH - 1);
                cell[0] = lab[(int64_t)min(max(yy, 0), d.H - 1) * d.W + xc];
                if (!(in_x && yy >= 0 && yy < d.H)) cell[0] = -1;
            }
        } else {
            j = valid ? v.bins[(int64_t)y * d.W + x] : 0xFF;
            if (wide) {
#pragma unroll
                for (int r = 0; r < kWinH; ++r) {
                    const int yy = y0 - 2 + r;
                    cell[r] = (in_x && yy >= 0 && yy < d.H) ? (int)lab[(int64_t)yy * d.W + xx] : -1;
                }
            } else {
                const int yy = y0 - 2 + wr;
                cell[0] = (wr < kWinH && in_x && yy >= 0 && yy < d.H)
                              ? (int)lab[(int64_t)yy * d.W + xx]
                              : -1;
            }
        }
        __syncthreads();  // the previous tile's window and list are no longer read
        if (wide) {
#pragma unroll
            for (int r = 0; r < kWinH; ++r) pt.lab[r * kWinW + wc] = cell[r];
        } else if (wr < kWinH) {
            pt.lab[wr * kWinW + wc] = cell[0];
        }
        if (threadIdx.x == 0) pt.n = 0;
        __syncthreads();
        if constexpr (!COMPACT) {
            if (valid) {
                const PixelMove mv =
                    pixel_decision(d, pt.lab + 3 * cj * kWinW + 3 * ci, j, hR, x, y);
                if (mv.n >= 0) apply(x, y, j, mv);
            }
        } else {
            const bool take = valid && pixel_movable(pt.lab + 3 * cj * kWinW + 3 * ci);
            wave_append(pt, take, (int)threadIdx.x | j << 8);
            __syncthreads();
            if ((int)threadIdx.x < pt.n) {
                const int u = pt.unit[threadIdx.x];
                const int ui = (u & 0xFF) % kPixTX, uj = (u & 0xFF) / kPixTX, uj_bin = u >> 8;
                const int px = x0 + 3 * ui, py = y0 + 3 * uj;
                const PixelMove mv = pixel_decision<false>(d, pt.lab + 3 * uj * kWinW + 3 * ui,
                                                           uj_bin, hR, px, py);
                if (mv.n >= 0) apply(px, py, uj_bin, mv);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Sparse block histogram for blocks of at most 16 pixels held in registers
// (segments of SEG lanes inside one wavefront, PPL pixels per lane; pixel tt
// of lane i is pixel tt * SEG + i of the block): for each of the lane's bins
// j[tt] (0xFF = no pixel), cnt = h_l(j) of its segment's block and first = no
// lower pixel of the block has that bin. No LDS, no barrier.
template <int SEG, int PPL>
__device__ __forceinline__ void shuffle_bins(const int (&j)[PPL], int (&cnt)[PPL],
                                             bool (&first)[PPL]) {
    static_assert(SEG * PPL <= 16, "larger blocks count their bins in LDS (lds_bins)");
    const int me = (threadIdx.x & 63) & (SEG - 1);
#pragma unroll
    for (int tt = 0; tt < PPL; ++tt) {
        cnt[tt] = 0;
        first[tt] = j[tt] != 0xFF;
    }
#pragma unroll
    for (int t2 = 0; t2 < PPL; ++t2) {
#pragma unroll
        for (int q = 0; q < SEG; ++q) {
            const int v = SEG == 1 ? j[t2] : __shfl(j[t2], q, SEG);
#pragma unroll
            for (int tt = 0; tt < PPL; ++tt) {
                const bool same = v == j[tt] && j[tt] != 0xFF;
                cnt[tt] += same;
                first[tt] = first[tt] && !(same && t2 * SEG + q < tt * SEG + me);
            }
        }
    }
}

// The same in one zeroed LDS histogram row h per segment, for blocks of 16 to
// 64 pixels: a lane first merges its own repeated bins, then adds each of its
// distinct bins with its multiplicity; the lane whose addition found h[j] at 0
// leads the bin, reads h_l(j) and clears the entry again. Any one lead lane
// per bin gives the same integer sums. A wavefront's LDS operations complete
// in issue order, and the fence keeps the compiler from moving a read above
// an addition, so every read follows every addition of the segment.
template <int PPL>
__device__ __forceinline__ void lds_bins(const int (&j)[PPL], int32_t *h, int (&cnt)[PPL],
                                         bool (&first)[PPL]) {
    int mult[PPL];
#pragma unroll
    for (int tt = 0; tt < PPL; ++tt) {
        cnt[tt] = 0;
        first[tt] = false;
        bool repeat = false;
        mult[tt] = 1;
#pragma unroll
        for (int t2 = 0; t2 < PPL; ++t2) {
            if (t2 < tt) repeat = repeat || j[t2] == j[tt];
            if (t2 > tt) mult[tt] += j[t2] == j[tt];
        }
        if (j[tt] != 0xFF && !repeat) first[tt] = atomicAdd(&h[j[tt]], mult[tt]) == 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
    for (int tt = 0; tt < PPL; ++tt) {
        if (first[tt]) {
            cnt[tt] = __hip_atomic_load(&h[j[tt]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            __hip_atomic_store(&h[j[tt]], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
    }
}

// ---------------------------------------------------------------------------
// Block phase. Segments of SEG lanes handle one block each; SEGS = kPT / SEG
// blocks per round, rounds stride over the grid.
//   pass 0: decide and apply at once (Prop. 1 rule; no drop rule)
//   pass 1: exact rule, decide only: record the target and stamp the source
//   pass 2: exact rule, apply the recorded moves whose target is no source
template <int SEG, int PPL, typename Table>
__device__ inline void block_phase(const BatchArgs &b, const ImageView &v, int level, int cls,
                                   int par, int pass, uint32_t stamp, uint8_t *sbin,
                                   Table &t, int2 *mylog) {
    constexpr int SEGS = kPT / SEG;
    constexpr int NPX = SEG * PPL;
    // where the bins are counted (bin_count_kind): registers, an LDS row per
    // segment, or the block's bins staged in LDS
    constexpr int KIND = bin_count_kind(SEG, PPL);
    constexpr int RP = KIND == 2 ? 1 : PPL;  // pixels per lane held in registers
    const Dims &d = v.d;
    int32_t *units = level_grid(v, level);
    const int s = 1 << level;
    const int uw = units_w(d, level), uh = units_h(d, level);
    const int ncx = class_cols(uw, cls), ncy = class_rows(uh, cls);
    const int nunits = ncx * ncy;
    const int per_round = v.ngroups * SEGS;
    const int rounds = (nunits + per_round - 1) / per_round;
    const int seg = threadIdx.x / SEG, lane = threadIdx.x % SEG;
    const int64_t khs = (int64_t)d.K * d.hs;
    const int32_t *hR = pick(b.ar.state, par) + v.base;
    const int32_t *sR = hR + khs;
    int32_t *W = pick(b.ar.state, par ^ 1);
    const bool exact = d.rule == SEEDS_BLOCK_EXACT;
    uint8_t *mine = sbin + seg * NPX;
    (void)mine;
    int32_t *seg_hist = reinterpret_cast<int32_t *>(sbin) + seg * d.hs;
    if constexpr (KIND == 1) {
        for (int i = lane; i < d.hs; i += SEG) seg_hist[i] = 0;
    }
    const int grp = v.grp;
    for (int r = 0; r < rounds; ++r) {
        const int unit = (r * v.ngroups + grp) * SEGS + seg;
        const bool in_range = unit < nunits;
        int ux = 0, uy = 0;
        if (in_range) {
            ux = cls % 3 + 3 * (unit % ncx);
            uy = cls / 3 + 3 * (unit / ncx);
        }
        // The block's bins and the labels around it are independent: both
        // loads are issued before either is waited for, and blocks of up to 64
        // pixels count their bins while the labels are still in flight.
        int jr[RP], cr[RP];
        bool fr[RP];
        if constexpr (KIND != 2) {
#pragma unroll
            for (int tt = 0; tt < PPL; ++tt) {
                const int q = lane + tt * SEG;
                const int x = ux * s + (q & (s - 1)), y = uy * s + (q >> level);
                jr[tt] = (in_range && x < d.W && y < d.H) ? v.bins[(int64_t)y * d.W + x] : 0xFF;
            }
        }
        Neighbourhood nb;
        nb.movable = false;
        nb.k = -1;
        nb.nc = 0;
        Ring ring;
        int target = -1;
        if (in_range) {
            if (pass == 2) {
                // the recorded target and the block's label together, then the
                // target's stamp (at a stand-in index when there is none: a
                // load behind a branch would be waited for on its own)
                target = v.pend[unit];
                nb.k = units[(int64_t)uy * uw + ux];
                const int32_t tstamp = v.src[target >= 0 ? target : 0];
                if (target >= 0 && tstamp == (int32_t)stamp) target = -1;
                nb.movable = target >= 0;
            } else {
                ring = load_ring(units, uw, uh, ux, uy);
            }
        }
        // Blocks of up to 64 pixels keep their bins in registers and count
        // them with shuffles (up to 16 pixels) or in an LDS row; larger blocks
        // are staged in LDS.
        if constexpr (KIND == 0) {
            shuffle_bins<SEG, PPL>(jr, cr, fr);
        } else if constexpr (KIND == 1) {
            lds_bins<PPL>(jr, seg_hist, cr, fr);
        } else {
#pragma unroll 4
            for (int tt = 0; tt < PPL; ++tt) {
                const int q = lane + tt * SEG;
                const int x = ux * s + (q & (s - 1)), y = uy * s + (q >> level);
                mine[q] = (in_range && x < d.W && y < d.H) ? v.bins[(int64_t)y * d.W + x] : 0xFF;
            }
            __syncthreads();
        }
        if (in_range && pass != 2) nb = neighbourhood(ring);
        // pixel tt of this lane: its bin j and, if it is the first of its bin in
        // the block, the bin's count (0 otherwise)
        auto leader_bin = [&](int tt, int &j, int &cnt) {
            if constexpr (KIND != 2) {
                j = jr[tt];
                cnt = fr[tt] ? cr[tt] : 0;
            } else {
                const int q = lane + tt * SEG;
                j = mine[q];
                cnt = 0;
                if (j == 0xFF) return;
                bool first = true;
                for (int q2 = 0; q2 < NPX; ++q2) {
                    const bool same = mine[q2] == j;
                    cnt += same;
                    first &= !(same && q2 < q);
                }
                if (!first) cnt = 0;
            }
        };
        if (nb.movable) {
            const int k = nb.k;
            const int64_t m = (int64_t)min(s, d.W - ux * s) * min(s, d.H - uy * s);
            if (pass != 2) {
                // evaluate the candidates: every pixel that is the first of its
                // bin in the block contributes for its bin j with count h_l(j).
                // Every lane loads the sizes and its cells, unused candidates
                // and non-leading lanes at valid stand-in indices: a load behind
                // a branch is waited for at the end of that branch, which would
                // make each candidate's loads a memory round trip of their own.
                int cs[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) cs[c] = c < nb.nc ? nb.cand[c] : k;
                // Blocks of at most 64 pixels in images of fewer than 2^23:
                // every term below is under 2^29 in magnitude and every sum
                // (of one lane or of the segment) under 2^30, so they are
                // formed in 32 bits; larger blocks use 64 bits. Only the
                // comparisons below cross-multiply two sums.
                using Acc = typename std::conditional<NPX <= 64, int32_t, int64_t>::type;
                const Acc Ak = sR[k];
                Acc An[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) An[c] = sR[cs[c]];
                const Acc mm = (Acc)m;
                Acc acc[4] = {0, 0, 0, 0}, acc_kl = 0;
#pragma unroll 4
                for (int tt = 0; tt < PPL; ++tt) {
                    int j, cnt;
                    leader_bin(tt, j, cnt);
                    const int js = j == 0xFF ? 0 : j;
                    const Acc hk = hR[(int64_t)k * d.hs + js];
                    Acc hn[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) hn[c] = hR[(int64_t)cs[c] * d.hs + js];
                    if (!cnt) continue;
                    const Acc hl = cnt;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (c >= nb.nc) break;
                        if (exact) {
                            // EXACT: h_l(j) (h_n(j) - h_k(j) + h_l(j))
                            acc[c] += hl * (hn[c] - hk + hl);
                        } else {
                            // Prop. 1: min(h_n(j) m, h_l(j) A_n)
                            const Acc x1 = hn[c] * mm, x2 = hl * An[c];
                            acc[c] += x1 < x2 ? x1 : x2;
                        }
                    }
                    if (!exact) {
                        // Prop. 1, k without the block: min((h_k - h_l) m, h_l (A_k - m))
                        const Acc x1 = (hk - hl) * mm, x2 = hl * (Ak - mm);
                        acc_kl += x1 < x2 ? x1 : x2;
                    }
                }
                if constexpr (NPX <= 64) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] = segment_sum32<SEG>(acc[c]);
                    acc_kl = segment_sum32<SEG>(acc_kl);
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] = segment_sum<SEG>(acc[c]);
                    acc_kl = segment_sum<SEG>(acc_kl);
                }
                // every lane holds the sums: every lane takes the same decision;
                // candidates are ascending, so ">" keeps the smaller label on ties
                int64_t bS = acc[0], bA = An[0];
                int bn = nb.cand[0];
#pragma unroll
                for (int c = 1; c < 4; ++c) {
                    if (c >= nb.nc) break;
                    const bool better =
                        exact ? acc[c] > bS : (int64_t)acc[c] * bA > bS * (int64_t)An[c];
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
                        v.pend[unit] = target;
                        if (target >= 0)
                            __hip_atomic_store(&v.src[k], (int32_t)stamp, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                    target = -1;
                }
            }
            if (target >= 0) {
                // apply (Sec. 5.3.3): the block's counts leave k and join target
                if (lane == 0) {
                    units[(int64_t)uy * uw + ux] = target;
                    table_add(b, t, W, mylog, (int32_t)(v.base + khs + target), (int32_t)m);
                    table_add(b, t, W, mylog, (int32_t)(v.base + khs + k), -(int32_t)m);
                }
#pragma unroll 4
                for (int tt = 0; tt < PPL; ++tt) {
                    int j, cnt;
                    leader_bin(tt, j, cnt);
                    if (!cnt) continue;
                    table_add(b, t, W, mylog, (int32_t)(v.base + target * d.hs + j), cnt);
                    table_add(b, t, W, mylog, (int32_t)(v.base + k * d.hs + j), -cnt);
                }
            }
        } else if (in_range && pass == 1 && lane == 0) {
            v.pend[unit] = -1;
        }
        if constexpr (KIND == 2) __syncthreads();  // LDS staging is reused next round
    }
}

// BIG = false instantiates block sides up to 8 only (levels <= 4): fewer
// registers and no scratch for the common hierarchies. BPPL: pixels per lane
// at levels 1-3 (seg_lanes, seg_ppl).
template <bool BIG, int BPPL = 1, typename Table>
__device__ inline void block_phase_any(const BatchArgs &b, const ImageView &v, int level, int cls,
                                       int par, int pass, uint32_t stamp, uint8_t *sbin,
                                       Table &t, int2 *mylog) {
#define SEEDS_BLOCK(SEG, PPL) \
    block_phase<SEG, PPL>(b, v, level, cls, par, pass, stamp, sbin, t, mylog)
    if constexpr (BPPL == 4) {
        if (level <= 3) {
            switch (level) {
                case 1: SEEDS_BLOCK(1, 4); break;
                case 2: SEEDS_BLOCK(4, 4); break;
                default: SEEDS_BLOCK(16, 4); break;
            }
            return;
        }
    }
    if (!BIG) {
        switch (level) {
            case 1: SEEDS_BLOCK(4, 1); break;
            case 2: SEEDS_BLOCK(16, 1); break;
            default: SEEDS_BLOCK(64, 1); break;
        }
        return;
    }
    switch (level) {
        case 1: SEEDS_BLOCK(4, 1); break;
        case 2: SEEDS_BLOCK(16, 1); break;
        case 3: SEEDS_BLOCK(64, 1); break;
        case 4: SEEDS_BLOCK(64, 4); break;
        case 5: SEEDS_BLOCK(64, 16); break;
        case 6: SEEDS_BLOCK(64, 64); break;
        default: SEEDS_BLOCK(64, 256); break;
    }
#undef SEEDS_BLOCK
}

// Level transition: every block of `level` splits into its 2x2 children
// (into the pixel labels from level 1).
__device__ inline void descend(const ImageView &v, int level) {
    const Dims &d = v.d;
    const int fw = units_w(d, level), fh = units_h(d, level);
    const int32_t *from = level_grid(v, level);
    // into the pixel labels from level 1 (16-bit plane: to16)
    uint16_t *to16 = level == 1 ? v.lab16 : nullptr;
    int32_t *to = level == 1 ? v.lab : level_grid(v, level - 1);
    const int tw = units_w(d, level - 1), th = units_h(d, level - 1);
    // work item = (parent row, chunk of kPT parents): each thread copies one
    // parent label to its (up to) four children; no per-lane division
    const int chunks = (fw + kPT - 1) / kPT;
    const int items = fh * chunks;
    for (int it = v.grp; it < items; it += v.ngroups) {
        const int py = it / chunks, px = (it - py * chunks) * kPT + (int)threadIdx.x;
        if (px >= fw) continue;
        const int32_t l = from[(int64_t)py * fw + px];
        const int x = 2 * px, y = 2 * py;  // x < tw and y < th: the child grid is 2f-1 or 2f wide
        auto put = [&](auto *row) {
            using T = typename std::remove_pointer<decltype(row)>::type;
            row[0] = (T)l;
            if (x + 1 < tw) row[1] = (T)l;
            if (y + 1 < th) {
                row[tw] = (T)l;
                if (x + 1 < tw) row[tw + 1] = (T)l;
            }
        };
        if (to16)
            put(to16 + (int64_t)y * tw + x);
        else
            put(to + (int64_t)y * tw + x);
    }
}

}  // namespace seeds
