// Persistent refinement kernel: one cooperative launch runs the whole
// schedule (every phase of every level and the level transitions) with
// grid-wide barriers between phases.
//
// Phase snapshot without a second barrier. Units of one class are at least
// three units apart, so a decision never reads a label that another decision
// of the same phase writes: labels are written in place as soon as a move is
// taken. The colour histograms and sizes exist twice. Phase t reads copy
// t % 2 (the state after phase t-1) and adds its deltas to the other copy,
// which holds the state after phase t-2; each workgroup also re-applies the
// deltas it logged in phase t-1 to that copy. After the barrier the other
// copy holds the state after phase t. At the end of the launch the last
// phase's deltas are re-applied to the stale copy, so both copies are equal
// again between launches.
//
// Under the exact block rule a block phase needs the drop rule (a move k -> n
// is dropped when n is a source in the same phase), which is only known once
// every decision of the phase is made: those phases decide, synchronise,
// then filter and apply, and synchronise again.
#include "seeds_phase.h"

namespace seeds {
namespace {

constexpr int kSpinLimit = 1 << 22;  // about a second of waiting: then give up

// Grid-wide barrier. The last workgroup to arrive resets the arrival count
// and bumps the generation; the others wait for the generation to change.
// The arrival is acquire-release and the wait an acquire, both at device
// scope, so every write before the barrier is visible after it. A wait that
// exceeds kSpinLimit sets the error flag and makes every workgroup return.
__device__ bool grid_sync(uint32_t *sync, uint32_t &gen) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const uint32_t old =
            __hip_atomic_fetch_add(&sync[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gridDim.x - 1) {
            __hip_atomic_store(&sync[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&sync[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            int spins = 0;
            while (__hip_atomic_load(&sync[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kSpinLimit) {
                    ok = 0;
                    __hip_atomic_store(&sync[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        if (__hip_atomic_load(&sync[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
        ++gen;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok;
}

struct RefineLaunch {
    BatchArgs b;  // a single image: b.nimg == 1
    ImageDesc one;
    Sched start;
    int max_phases;
    uint32_t stamp;  // stamp of the phase before the first one of the launch
};

template <bool BIG, typename LabT>
__global__ __launch_bounds__(kPT) void k_refine(RefineLaunch a) {
    extern __shared__ uint8_t sbin[];
    __shared__ DeltaTable<> t;
    __shared__ PixelTile pl;
    __shared__ int s_prev_n;
    const BatchArgs &b = a.b;
    const Dims &d = a.one.d;
    const ImageView v = single_view(b, a.one, xcd_group(), gridDim.x);
    uint32_t *sync = b.ar.sync;
    uint32_t gen = __hip_atomic_load(&sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int2 *const log0 = b.ar.log + (int64_t)blockIdx.x * b.log_cap;
    int2 *const log1 = b.ar.log + ((int64_t)gridDim.x + blockIdx.x) * b.log_cap;
    if (threadIdx.x == 0) s_prev_n = 0;
    Sched sc = a.start;
    int par = 0;  // state copy holding the current state
    int phases = 0;
    uint32_t stamp = a.stamp;
    for (;;) {
        int cls = 0;
        const SchedOp op = sched_next(d, sc, a.max_phases < 0 ? -1 : a.max_phases - phases, &cls);
        if (op == OP_END) break;
        if (op == OP_DESCEND) {
            descend(v, sc.level);
            if (!grid_sync(sync, gen)) return;
        } else {
            int32_t *W = pick(b.ar.state, par ^ 1);
            int2 *cur_log = par ? log1 : log0;
            const int2 *prev_log = par ? log0 : log1;
            const int prev_n = s_prev_n;
            table_clear(t);
            __syncthreads();
            // the previous phase's deltas, logged by this workgroup
            if (phases > 0) replay(prev_log, min(prev_n, b.log_cap), W);
            ++stamp;
            if (sc.level == 0) {
                pixel_phase<true, LabT>(b, v, cls, par, t, cur_log, pl);
            } else if (d.rule == SEEDS_BLOCK_EXACT) {
                block_phase_any<BIG>(b, v, sc.level, cls, par, 1, stamp, sbin, t, cur_log);
                if (!grid_sync(sync, gen)) return;
                block_phase_any<BIG>(b, v, sc.level, cls, par, 2, stamp, sbin, t, cur_log);
            } else {
                block_phase_any<BIG>(b, v, sc.level, cls, par, 0, stamp, sbin, t, cur_log);
            }
            __syncthreads();
            table_flush(b, t, W, cur_log);
            __syncthreads();
            if (threadIdx.x == 0) s_prev_n = t.n;
            if (!grid_sync(sync, gen)) return;
            par ^= 1;
            ++phases;
        }
        sched_done(sc, op);
    }
    // the copy read by the last phase lacks that phase's deltas
    if (phases > 0) replay(par ? log0 : log1, min(s_prev_n, b.log_cap), pick(b.ar.state, par ^ 1));
}

}  // namespace

PersistentGeom persistent_geometry(const Dims &d, int device, int groups_per_cu) {
    PersistentGeom g;
    g.lds_bytes = max(1, phase_lds_bytes_upto(d.L - 1, d.hs));
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus < 1)
        cus = 1;
    int occ = 0;
    // (the 16-bit variants use no more resources than these)
    const void *fn = d.L > 4 ? (const void *)k_refine<true, int32_t>
                             : (const void *)k_refine<false, int32_t>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kPT, g.lds_bytes) != hipSuccess ||
        occ < 1)
        occ = 1;
    int groups = cus * min(occ, max(1, groups_per_cu));
    // no more groups than the busiest phase has work items (class 0 is the
    // largest class at every level)
    int useful = 1;
    for (int l = 0; l < d.L; ++l) useful = max(useful, phase_groups(d, l, 0));
    g.groups = max(1, min(groups, useful));
    int cap = 1;
    for (int l = 0; l < d.L; ++l) {
        const int items = (phase_groups(d, l, 0) + g.groups - 1) / g.groups;
        cap = max(cap, items * deltas_per_round(d, l));
    }
    g.log_cap = cap;
    return g;
}

hipError_t launch_refine(const BatchArgs &b, const ImageDesc &one, const PersistentGeom &g,
                         const Sched &start, int max_phases, uint32_t stamp, hipStream_t s) {
    RefineLaunch a;
    a.b = b;
    a.b.log_cap = g.log_cap;
    a.b.log_groups = g.groups;
    a.one = one;
    a.start = start;
    a.max_phases = max_phases;
    a.stamp = stamp;
    void *args[] = {&a};
    const void *fn;
    if (b.ar.lab16)
        fn = one.d.L > 4 ? (const void *)k_refine<true, uint16_t> : (const void *)k_refine<false, uint16_t>;
    else
        fn = one.d.L > 4 ? (const void *)k_refine<true, int32_t> : (const void *)k_refine<false, int32_t>;
    return hipLaunchCooperativeKernel(fn, dim3(g.groups), dim3(kPT), args, (unsigned)g.lds_bytes,
                                      s);
}

}  // namespace seeds
