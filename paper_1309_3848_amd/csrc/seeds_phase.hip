// One launch per phase: the launch boundary is the phase barrier. A phase
// kernel first adds the previous phase's logged deltas to the state copy it
// writes, then decides and applies the moves of its class (see
// seeds_phase.h). The launches of a whole refinement are captured once into
// a HIP graph and replayed.
#include "seeds_phase.h"

namespace seeds {
namespace {

// Image and rank of this workgroup. A single image (BATCH = false) takes its
// view straight from the kernel arguments, so the compiler can reload any of
// its fields instead of keeping them all live; in a batch, map[logical
// group] = (image, rank among the image's workgroups).
template <bool BATCH>
__device__ __forceinline__ ImageView resolve(const BatchArgs &b, const ImageDesc &one,
                                             const int2 *map, int level, int cls, int remap) {
    const int lg = remap ? xcd_group() : (int)blockIdx.x;
    if constexpr (!BATCH) {
        return single_view(b, one, lg, gridDim.x);
    } else {
        const int2 e = map[lg];
        const ImageDesc g = b.imgs[e.x];
        return make_view(b, g, e.y, phase_launch_groups(g.d, level, cls, b.items, b.bppl));
    }
}

// Work of one workgroup in a phase launch: its image view and the phase.
struct PhaseWork {
    ImageView v;
    int level, cls;
};

// The body shared by every phase launch. `find` yields the workgroup's work;
// it runs after the replay prefetch is issued so that the two overlap.
// KINDS: 1 pixel phases only, 2 block phases only, 3 both (chosen per
// workgroup from its work).
template <bool BIG, int KINDS, bool COMPACT, typename LabT, int BPPL, int TBITS, typename Find>
__device__ __forceinline__ void phase_body(const BatchArgs &b, Find find, int par, int pass,
                                           uint32_t stamp, int replay_groups,
                                           int slot_base = 0) {
    extern __shared__ uint8_t sbin[];
    __shared__ DeltaTable<TBITS> t;
    __shared__ PixelTile pl;
    table_clear(t);
    __syncthreads();
    // The previous phase's deltas go to the copy this phase writes and nobody
    // reads, as this phase's own deltas do; additions commute, so they need no
    // ordering with the decisions. The first kPre entries of the log of slot
    // blockIdx.x are fetched now, together with its length, and added at the
    // end; a longer log (rare) is read once its length is known.
    int32_t *W = pick(b.ar.state, par ^ 1);
    constexpr int kPre = 64;
    // (unconditional loads: the slot exists whatever replay_groups is)
    const bool replay_own = (int)blockIdx.x < replay_groups;
    const int64_t own_slot = (int64_t)(par ^ 1) * b.log_groups + blockIdx.x;
    const int pre_n = replay_own ? b.ar.log_n[own_slot] : 0;
    const int2 pre = b.ar.log[own_slot * b.log_cap + (threadIdx.x & (kPre - 1))];
    const PhaseWork w = find();
    // this workgroup's log slot: a phase split over two launches gives the
    // second one the slots after the first one's
    const int64_t my_slot = (int64_t)par * b.log_groups + slot_base + blockIdx.x;
    int2 *mylog = b.ar.log + my_slot * b.log_cap;
    if constexpr (KINDS == 1) {
        pixel_phase<COMPACT, LabT>(b, w.v, w.cls, par, t, mylog, pl);
    } else if constexpr (KINDS == 2) {
        block_phase_any<BIG, BPPL>(b, w.v, w.level, w.cls, par, pass, stamp, sbin, t, mylog);
    } else {
        if (w.level == 0)
            pixel_phase<COMPACT, LabT>(b, w.v, w.cls, par, t, mylog, pl);
        else
            block_phase_any<BIG, BPPL>(b, w.v, w.level, w.cls, par, pass, stamp, sbin, t, mylog);
    }
    if (replay_own) {
        const int n = min(pre_n, b.log_cap);
        if ((int)threadIdx.x < min(n, kPre)) atomicAdd(&W[pre.x], pre.y);
        if (n > kPre) {
            const int2 *src_log = b.ar.log + own_slot * b.log_cap + kPre;
            for (int e = threadIdx.x; e < n - kPre; e += kPT) atomicAdd(&W[src_log[e].x], src_log[e].y);
        }
    }
    for (int g = blockIdx.x + gridDim.x; g < replay_groups; g += gridDim.x) {
        const int64_t slot = (int64_t)(par ^ 1) * b.log_groups + g;
        replay(b.ar.log + slot * b.log_cap, min(b.ar.log_n[slot], b.log_cap), W);
    }
    __syncthreads();
    if (pass == 1) return;
    table_flush(b, t, W, mylog);
    __syncthreads();
    if (threadIdx.x == 0) b.ar.log_n[my_slot] = min(t.n, b.log_cap);
}

// PIXEL selects the pixel-level or the block-level code: each variant holds
// only its own registers, and the block variant of the common hierarchies
// (BIG = false) fits six wavefronts per SIMD without spilling (five with
// four pixels per lane). L16: pixel labels stored as 16-bit values (pixel
// variants only). BPPL: pixels per lane at block levels 1-3 (block variants
// only). TBITS: delta-table size (the larger one for batch block phases with
// four pixels per lane and several work items per workgroup).
// Tuning (mapping only, never the moves): COMPACT for pixel phases, and
// `remap` = 1 numbers the workgroups so that each XCD works a contiguous band.
template <bool BIG, bool BATCH, bool PIXEL, bool COMPACT, bool L16 = false, int BPPL = 1,
          int TBITS = kTableBits>
__global__ __launch_bounds__(kPT, PIXEL ? 5 : BIG ? 1 : BPPL == 1 ? 6 : 5) void k_phase(
    BatchArgs b, ImageDesc one, const int2 *map, int level, int cls, int par, int pass,
    uint32_t stamp, int replay_groups, int remap) {
    phase_body<BIG, PIXEL ? 1 : 2, COMPACT, typename std::conditional<L16, uint16_t, int32_t>::type,
               BPPL, TBITS>(
        b,
        [&]() {
            return PhaseWork{resolve<BATCH>(b, one, map, level, cls, remap), level, cls};
        },
        par, pass, stamp, replay_groups);
}

// A mixed launch: every item is one image at its own phase (level, class).
// Only the Prop. 1 rule (one pass per phase) runs this way. A tick runs its
// pixel-level items and its block-level items as two launches of the two
// kernel variants; the second takes the log slots after the first's.
template <bool BIG, bool PIXEL, bool COMPACT>
__global__ __launch_bounds__(kPT, PIXEL ? 5 : !BIG ? 6 : 1) void k_phase_mixed(
    BatchArgs b, TickList l, int par, int replay_groups, int slot_base, int remap) {
    phase_body<BIG, PIXEL ? 1 : 2, COMPACT, int32_t, 1, kTableBits>(
        b,
        [&]() {
            const int lg = remap ? xcd_group() : (int)blockIdx.x;
            const TickItem &it = l.items[find_tick_item(l, lg)];
            return PhaseWork{make_view(b, it.g, lg - it.first, it.groups), it.level, it.cls};
        },
        par, 0, 0u, replay_groups, slot_base);
}

__global__ __launch_bounds__(kPT) void k_descend_mixed(BatchArgs b, TickList l) {
    const int lg = xcd_group();
    const TickItem &it = l.items[find_tick_item(l, lg)];
    descend(make_view(b, it.g, lg - it.first, it.groups), it.level);
}

// After the last phase: add its deltas to the copy it read, so that both
// copies hold the same state again.
__global__ __launch_bounds__(kPT) void k_replay(BatchArgs b, int par, int groups) {
    for (int g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t slot = (int64_t)par * b.log_groups + g;
        replay(b.ar.log + slot * b.log_cap, min(b.ar.log_n[slot], b.log_cap), pick(b.ar.state, par));
    }
}

// Sizes from the histograms of one image (pixel phases do not maintain them).
__global__ __launch_bounds__(kPT) void k_sizes(Dims d, int32_t *state0, int32_t *state1) {
    const int k = blockIdx.x * kPT + threadIdx.x;
    if (k >= d.K) return;
    int32_t sum = 0;
    for (int j = 0; j < d.nb; ++j) sum += state0[(int64_t)k * d.hs + j];
    const int64_t khs = (int64_t)d.K * d.hs;
    state0[khs + k] = sum;
    state1[khs + k] = sum;
}

__global__ __launch_bounds__(kPT) void k_descend(BatchArgs b, ImageDesc one, const int2 *map,
                                                 int level) {
    const int lg = xcd_group();
    if (b.nimg == 1) {
        descend(single_view(b, one, lg, gridDim.x), level);
        return;
    }
    const int2 e = map[lg];
    const ImageDesc g = b.imgs[e.x];
    descend(make_view(b, g, e.y, descend_groups(g.d, level)), level);
}

}  // namespace

hipError_t launch_phase(const BatchArgs &b, const ImageDesc &one, const int2 *map, int max_level,
                        int level, int cls, int par, int pass, uint32_t stamp, int groups,
                        int replay_groups, const PhaseTuning &tune, hipStream_t s) {
    const int lds = phase_lds_bytes(level, one.d.hs, tune.block_ppl);
    const bool batch = b.nimg > 1;
    const bool ppl4 = tune.block_ppl == 4;
    // block phases of a batch with four pixels per lane and several work items
    // per workgroup: the larger delta table (their blocks overflow the small one)
    const bool multi = batch && ppl4 && tune.items > 1;
    constexpr int M = kTableBitsMulti;
    decltype(&k_phase<false, false, true, true>) fn;
    if (level == 0 && b.ar.lab16) {
        if (tune.pixel_compact)
            fn = batch ? k_phase<false, true, true, true, true> : k_phase<false, false, true, true, true>;
        else
            fn = batch ? k_phase<false, true, true, false, true>
                       : k_phase<false, false, true, false, true>;
    } else if (level == 0) {
        if (tune.pixel_compact)
            fn = batch ? k_phase<false, true, true, true> : k_phase<false, false, true, true>;
        else
            fn = batch ? k_phase<false, true, true, false> : k_phase<false, false, true, false>;
    } else if (max_level >= 4) {
        if (ppl4)
            fn = !batch  ? k_phase<true, false, false, true, false, 4>
                 : multi ? k_phase<true, true, false, true, false, 4, M>
                         : k_phase<true, true, false, true, false, 4>;
        else
            fn = batch ? k_phase<true, true, false, true> : k_phase<true, false, false, true>;
    } else {
        if (ppl4)
            fn = !batch  ? k_phase<false, false, false, true, false, 4>
                 : multi ? k_phase<false, true, false, true, false, 4, M>
                         : k_phase<false, true, false, true, false, 4>;
        else
            fn = batch ? k_phase<false, true, false, true> : k_phase<false, false, false, true>;
    }
    hipLaunchKernelGGL(fn, dim3(groups), dim3(kPT), lds, s, b, one, map, level, cls, par, pass,
                       stamp, replay_groups, tune.xcd_remap ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_phase_mixed(const BatchArgs &b, const TickList &l, bool pixel, int max_level,
                              int par, int groups, int replay_groups, int slot_base,
                              const PhaseTuning &tune, hipStream_t s) {
    const int lds = pixel ? 0 : phase_lds_bytes_upto(max_level, l.hs);
    decltype(&k_phase_mixed<false, true, true>) fn;
    if (pixel)
        fn = tune.pixel_compact ? k_phase_mixed<false, true, true> : k_phase_mixed<false, true, false>;
    else
        fn = max_level >= 4 ? k_phase_mixed<true, false, true> : k_phase_mixed<false, false, true>;
    hipLaunchKernelGGL(fn, dim3(groups), dim3(kPT), lds, s, b, l, par, replay_groups, slot_base,
                       tune.xcd_remap ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_descend_mixed(const BatchArgs &b, const TickList &l, int groups, hipStream_t s) {
    hipLaunchKernelGGL(k_descend_mixed, dim3(groups), dim3(kPT), 0, s, b, l);
    return hipGetLastError();
}

hipError_t launch_final_replay(const BatchArgs &b, int par, int groups, hipStream_t s) {
    hipLaunchKernelGGL(k_replay, dim3(max(1, min(groups, 1024))), dim3(kPT), 0, s, b, par, groups);
    return hipGetLastError();
}

hipError_t launch_descend(const BatchArgs &b, const ImageDesc &one, const int2 *map, int level,
                          int groups, hipStream_t s) {
    hipLaunchKernelGGL(k_descend, dim3(groups), dim3(kPT), 0, s, b, one, map, level);
    return hipGetLastError();
}

hipError_t launch_sizes(const Dims &d, int32_t *state0, int32_t *state1, hipStream_t s) {
    hipLaunchKernelGGL(k_sizes, dim3((d.K + kPT - 1) / kPT), dim3(kPT), 0, s, d, state0, state1);
    return hipGetLastError();
}

}  // namespace seeds
