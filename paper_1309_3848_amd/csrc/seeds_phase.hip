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
    __shared__ int s_n;
    if (threadIdx.x == 0) s_n = 0;
    int32_t *hW = pick(a.hist, par ^ 1);
    int32_t *sW = pick(a.size, par ^ 1);
    for (int g = blockIdx.x; g < replay_groups; g += gridDim.x) {
        const int64_t slot = (int64_t)(par ^ 1) * a.log_groups + g;
        replay(a, a.log + slot * a.log_cap, min(a.log_n[slot], a.log_cap), hW, sW);
    }
    __syncthreads();
    int4 *mylog = a.log + ((int64_t)par * a.log_groups + blockIdx.x) * a.log_cap;
    if (level == 0)
        pixel_phase(a, cls, par, mylog, &s_n);
    else
        block_phase_any<BIG>(a, level, cls, par, pass, stamp, pick(a.bl, cur_bl), sbin, mylog,
                             &s_n);
    __syncthreads();
    if (threadIdx.x == 0 && pass != 1) a.log_n[(int64_t)par * a.log_groups + blockIdx.x] = s_n;
}

// After the last phase: add its deltas to the copy it read, so that both
// copies hold the same state again.
__global__ __launch_bounds__(kPT) void k_replay(RefineArgs a, int par, int groups) {
    for (int g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t slot = (int64_t)par * a.log_groups + g;
        replay(a, a.log + slot * a.log_cap, min(a.log_n[slot], a.log_cap), pick(a.hist, par),
               pick(a.size, par));
    }
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
        const int per_group = l == 0 ? kPT : kPT / seg_lanes(l);
        c = max(c, per_group * (l == 0 ? 1 : min(1 << (2 * l), d.nb)));
    }
    *groups = g;
    *cap = c;
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
    a.hist[0] = b.hist[0];
    a.hist[1] = b.hist[1];
    a.size[0] = b.size[0];
    a.size[1] = b.size[1];
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
