// One launch per phase: the launch boundary is the phase barrier. A phase
// kernel first adds the previous phase's logged deltas to the histogram copy
// it writes, then decides and applies the moves of its class (see
// seeds_phase.h). The launches of a whole refinement are captured once into
// a HIP graph and replayed.
#include "seeds_phase.h"

namespace seeds {
namespace {

template <bool BIG>
__global__ __launch_bounds__(kPT) void k_phase(RefineArgs a, int level, int cls, int par, int pass,
                                               uint32_t stamp, int cur_bl, int replay_groups) {
    extern __shared__ uint8_t sbin[];
    __shared__ DeltaTable t;
    __shared__ PixelList pl;
    table_clear(t);
    __syncthreads();
    // The previous phase's deltas go to the copy this phase writes and nobody
    // reads, as this phase's own deltas do; additions commute, so they need no
    // ordering with the decisions. The first kPre entries of the log of slot
    // blockIdx.x are fetched now, together with its length, and added at the
    // end; a longer log (rare) is read once its length is known.
    int32_t *W = pick(a.state, par ^ 1);
    constexpr int kPre = 64;
    int2 pre = make_int2(0, 0);
    int pre_n = 0;
    const bool replay_own = (int)blockIdx.x < replay_groups;
    const int64_t own_slot = (int64_t)(par ^ 1) * a.log_groups + blockIdx.x;
    if (replay_own) {
        pre_n = a.log_n[own_slot];
        if (threadIdx.x < kPre) pre = a.log[own_slot * a.log_cap + threadIdx.x];
    }
    int2 *mylog = a.log + ((int64_t)par * a.log_groups + blockIdx.x) * a.log_cap;
    if (level == 0)
        pixel_phase(a, cls, par, t, mylog, pl);
    else
        block_phase_any<BIG>(a, level, cls, par, pass, stamp, pick(a.bl, cur_bl), sbin, t, mylog);
    if (replay_own) {
        const int n = min(pre_n, a.log_cap);
        if ((int)threadIdx.x < min(n, kPre)) atomicAdd(&W[pre.x], pre.y);
        if (n > kPre) {
            const int2 *src_log = a.log + own_slot * a.log_cap + kPre;
            for (int e = threadIdx.x; e < n - kPre; e += kPT) atomicAdd(&W[src_log[e].x], src_log[e].y);
        }
    }
    for (int g = blockIdx.x + gridDim.x; g < replay_groups; g += gridDim.x) {
        const int64_t slot = (int64_t)(par ^ 1) * a.log_groups + g;
        replay(a.log + slot * a.log_cap, min(a.log_n[slot], a.log_cap), W);
    }
    __syncthreads();
    if (pass == 1) return;
    table_flush(a, t, W, mylog);
    __syncthreads();
    if (threadIdx.x == 0) a.log_n[(int64_t)par * a.log_groups + blockIdx.x] = min(t.n, a.log_cap);
}

// After the last phase: add its deltas to the copy it read, so that both
// copies hold the same state again.
__global__ __launch_bounds__(kPT) void k_replay(RefineArgs a, int par, int groups) {
    for (int g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t slot = (int64_t)par * a.log_groups + g;
        replay(a.log + slot * a.log_cap, min(a.log_n[slot], a.log_cap), pick(a.state, par));
    }
}

// Sizes from the histograms (pixel phases do not maintain them).
__global__ __launch_bounds__(kPT) void k_sizes(Dims d, int32_t *state0, int32_t *state1) {
    const int k = blockIdx.x * kPT + threadIdx.x;
    if (k >= d.K) return;
    int32_t sum = 0;
    for (int j = 0; j < d.nb; ++j) sum += state0[(int64_t)k * d.hs + j];
    const int64_t khs = (int64_t)d.K * d.hs;
    state0[khs + k] = sum;
    state1[khs + k] = sum;
}

}  // namespace

int phase_groups(const Dims &d, int level, int cls) {
    const int n = class_cols(units_w(d, level), cls) * class_rows(units_h(d, level), cls);
    const int per_group = level == 0 ? kPT : kPT / seg_lanes(level);
    return max(1, (n + per_group - 1) / per_group);
}

void phase_log_shape(const Dims &d, int *groups, int *cap) {
    int g = 1, c = 1;
    for (int l = 0; l < d.L; ++l) {
        g = max(g, phase_groups(d, l, 0));
        c = max(c, deltas_per_round(d, l));
    }
    *groups = g;
    *cap = c;
}

hipError_t launch_sizes(const Dims &d, const Buffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_sizes, dim3((d.K + kPT - 1) / kPT), dim3(kPT), 0, s, d, b.hist[0],
                       b.hist[1]);
    return hipGetLastError();
}

hipError_t launch_phase_kernel(const Dims &d, const Buffers &b, int log_groups, int log_cap,
                               int level, int cls, int par, int pass, uint32_t stamp, int cur_bl,
                               int replay_groups, hipStream_t s) {
    RefineArgs a;
    a.d = d;
    a.bins = b.bins;
    a.lab = b.lab;
    a.bl[0] = b.bl[0];
    a.bl[1] = b.bl[1];
    a.state[0] = b.hist[0];
    a.state[1] = b.hist[1];
    a.src = b.src;
    a.pend = b.pend;
    a.log = b.log;
    a.log_n = b.log_n;
    a.log_cap = log_cap;
    a.log_groups = log_groups;
    a.sync = b.sync;
    const int groups = level < 0 ? max(1, min(replay_groups, 1024)) : phase_groups(d, level, cls);
    if (level < 0) {
        hipLaunchKernelGGL(k_replay, dim3(groups), dim3(kPT), 0, s, a, par, replay_groups);
        return hipGetLastError();
    }
    const int lds = level == 0 ? 0 : kPT * seg_ppl(level);
    if (d.L > 4)
        hipLaunchKernelGGL(k_phase<true>, dim3(groups), dim3(kPT), lds, s, a, level, cls, par, pass,
                           stamp, cur_bl, replay_groups);
    else
        hipLaunchKernelGGL(k_phase<false>, dim3(groups), dim3(kPT), lds, s, a, level, cls, par,
                           pass, stamp, cur_bl, replay_groups);
    return hipGetLastError();
}

}  // namespace seeds
