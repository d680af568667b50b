// Measurement hooks. The LDS-atomic throughput of the device, the secondary
// roof of the refinement kernels (their per-workgroup histograms and delta
// tables are LDS integer atomics). Every lane adds to its own LDS word, so a
// wavefront instruction touches 64 distinct words in distinct banks and
// nothing conflicts; the rate is wavefront instructions per second.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "seeds.h"
#include "seeds_internal.h"

namespace seeds {
namespace {

constexpr int kMbThreads = 256, kMbGroups = 4096, kMbIters = 1024;

__global__ __launch_bounds__(kMbThreads) void k_lds_atomics(int32_t *out) {
    __shared__ int32_t words[kMbThreads];
    words[threadIdx.x] = 0;
    __syncthreads();
    int32_t *w = &words[threadIdx.x];
#pragma unroll 16
    for (int i = 0; i < kMbIters; ++i) atomicAdd(w, 1);
    __syncthreads();
    // keep the result observable: one word per workgroup
    if (threadIdx.x == 0) out[blockIdx.x] = words[(blockIdx.x + 1) % kMbThreads];
}

// Launch floor of a phase: a chain of launches with the shape of one phase
// launch (`groups` workgroups of 256 lanes, one launch per phase, captured in
// a HIP graph), doing (0) nothing, (1) one round of coalesced loads like a
// pixel tile's window (fourteen 2-byte loads per lane from a plane of 7 KB per
// workgroup), or (2) that round, then five loads from a 512 KB table at
// addresses computed from its values (the histogram cells of a decision), then
// a few global atomics per workgroup (the delta flush). Every index is masked
// into its buffer. Every lane's loaded values feed a wavefront vote against a
// run-time value (`never`, which no sum reaches): a value used only on a rare
// path could have its loads moved into that path, and most lanes would then
// skip the round trip being measured.
constexpr int kFloorRows = 14, kFloorCells = 5, kFloorTable = 1 << 17;

__global__ __launch_bounds__(kMbThreads) void k_floor_empty(int32_t *) {}

__device__ __forceinline__ int floor_window(const uint16_t *plane) {
    const uint16_t *w = plane + (size_t)blockIdx.x * kFloorRows * kMbThreads + threadIdx.x;
    int sum = 0;
#pragma unroll
    for (int r = 0; r < kFloorRows; ++r) sum += w[r * kMbThreads];
    return sum;
}

__global__ __launch_bounds__(kMbThreads) void k_floor_one(const uint16_t *plane, int32_t *out,
                                                          int never) {
    const int sum = floor_window(plane);
    if (__any(sum == never) && threadIdx.x == 0) out[blockIdx.x & (kFloorTable - 1)] = sum;
}

__global__ __launch_bounds__(kMbThreads) void k_floor_two(const uint16_t *plane,
                                                          const int32_t *table, int32_t *out,
                                                          int never) {
    const int sum = floor_window(plane);
    int acc = 0;
#pragma unroll
    for (int q = 0; q < kFloorCells; ++q) acc += table[(sum * 131 + q * 7919) & (kFloorTable - 1)];
    if (__any(acc == never) && threadIdx.x == 0) out[blockIdx.x & (kFloorTable - 1)] = acc;
    if ((sum & 63) == 0) atomicAdd(&out[(sum + acc) & (kFloorTable - 1)], 1);
}

// Traffic probes: three kernels whose memory traffic is known exactly, for
// reading a profiler's byte counters on the access kinds of the refinement
// kernels. The buffer holds `lines` 128-byte lines of int32 (a power of two);
// every probe touches each line exactly once:
//   stream  reads the whole buffer with coalesced 16-byte loads;
//   scatter reads one 4-byte word per line, lines visited in a permuted
//           order (thread i takes line (i * odd) mod lines, a bijection), so
//           the 64 lanes of a wavefront hit 64 lines far apart;
//   atomic  adds 1 to one word per line in the same permuted order.
// Each workgroup sums what it read (the atomics: the old values) and stores
// the sum to its own word of `part` (plain stores to distinct words, so no
// same-address atomics queue up behind the probe); the host adds them up.
constexpr int kLineWords = 32;
constexpr uint32_t kProbeOdd = 0x9E3779B1u;

__device__ __forceinline__ void probe_sum(long long v, unsigned long long *part) {
    __shared__ long long waves[kMbThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) waves[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
#pragma unroll
        for (int w = 0; w < kMbThreads / 64; ++w) t += waves[w];
        part[blockIdx.x] = (unsigned long long)t;
    }
}

__global__ __launch_bounds__(kMbThreads) void k_probe_stream(const int4 *buf, int64_t n4,
                                                             unsigned long long *part) {
    long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * kMbThreads + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * kMbThreads) {
        const int4 q = buf[i];
        acc += (long long)q.x + q.y + q.z + q.w;
    }
    probe_sum(acc, part);
}

// grid: exactly lines / 256 workgroups (lines is a power of two >= 1024)
__global__ __launch_bounds__(kMbThreads) void k_probe_scatter(const int32_t *buf, uint32_t mask,
                                                              unsigned long long *part) {
    const uint32_t line = ((blockIdx.x * kMbThreads + threadIdx.x) * kProbeOdd) & mask;
    probe_sum(buf[(size_t)line * kLineWords], part);
}

__global__ __launch_bounds__(kMbThreads) void k_probe_atomic(int32_t *buf, uint32_t mask,
                                                             unsigned long long *part) {
    const uint32_t line = ((blockIdx.x * kMbThreads + threadIdx.x) * kProbeOdd) & mask;
    probe_sum(atomicAdd(&buf[(size_t)line * kLineWords], 1), part);
}

}  // namespace
}  // namespace seeds

using namespace seeds;

extern "C" seeds_status seeds_traffic_probe(int64_t lines, double *us, void *hip_stream) {
    if (!us) return set_error(SEEDS_E_INVAL, "output is NULL");
    if (lines < 1024 || lines > (int64_t)1 << 22 || (lines & (lines - 1)))
        return set_error(SEEDS_E_INVAL, "lines %lld is not a power of two in [2^10, 2^22]",
                         (long long)lines);
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t bytes = (size_t)lines * kLineWords * sizeof(int32_t);
    const int groups = (int)(lines / kMbThreads);
    const int sgroups = std::min(groups * 2, 4096);  // the streaming read's grid
    const int nparts = sgroups + 2 * groups;         // one word per workgroup of each probe
    int32_t *buf = nullptr;
    unsigned long long *part = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipError_t e = hipMalloc(&buf, bytes);
    if (e == hipSuccess) e = hipMalloc(&part, nparts * sizeof(unsigned long long));
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    // every word 0x01010101
    if (e == hipSuccess) e = hipMemsetAsync(buf, 1, bytes, s);
    const uint32_t mask = (uint32_t)(lines - 1);
    // untimed warm-up: one workgroup of each probe, so the timed launches do
    // not include loading the kernels (its atomics add 1 to the probed word of
    // the 256 lines of workgroup 0, which every timed probe then reads)
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_probe_stream, dim3(1), dim3(kMbThreads), 0, s, (const int4 *)buf,
                           (int64_t)kMbThreads, part);
        hipLaunchKernelGGL(k_probe_scatter, dim3(1), dim3(kMbThreads), 0, s, buf, mask, part);
        hipLaunchKernelGGL(k_probe_atomic, dim3(1), dim3(kMbThreads), 0, s, buf, mask, part);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_probe_stream, dim3(sgroups), dim3(kMbThreads), 0, s,
                           (const int4 *)buf, (int64_t)(bytes / sizeof(int4)), part);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_probe_scatter, dim3(groups), dim3(kMbThreads), 0, s, buf, mask,
                           part + sgroups);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(ev[2], s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_probe_atomic, dim3(groups), dim3(kMbThreads), 0, s, buf, mask,
                           part + sgroups + groups);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(ev[3], s);
    std::vector<unsigned long long> h(nparts, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), part, nparts * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        us[i] = ms * 1e3;
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (buf) (void)hipFree(buf);
    if (part) (void)hipFree(part);
    if (e != hipSuccess) return set_error(SEEDS_E_DEVICE, "traffic probe: %s", hipGetErrorString(e));
    unsigned long long got[3] = {0, 0, 0};
    for (int i = 0; i < nparts; ++i) got[i < sgroups ? 0 : i < sgroups + groups ? 1 : 2] += h[i];
    const unsigned long long word = 0x01010101ull, n = (unsigned long long)lines;
    // the warm-up's atomics added 1 to one word of each of 256 lines
    if (got[0] != n * kLineWords * word + kMbThreads || got[1] != n * word + kMbThreads ||
        got[2] != n * word + kMbThreads)
        return set_error(SEEDS_E_DEVICE, "traffic probe: sums %llu %llu %llu", got[0], got[1],
                         got[2]);
    return SEEDS_OK;
}

extern "C" seeds_status seeds_launch_floor(int32_t groups, int32_t launches, double *us,
                                           void *hip_stream) {
    if (!us) return set_error(SEEDS_E_INVAL, "output is NULL");
    if (groups < 1 || groups > 65536)
        return set_error(SEEDS_E_INVAL, "groups %d outside [1,65536]", groups);
    if (launches < 1 || launches > 4096)
        return set_error(SEEDS_E_INVAL, "launches %d outside [1,4096]", launches);
    hipStream_t caller = (hipStream_t)hip_stream;
    const size_t plane_elems = (size_t)groups * kFloorRows * kMbThreads;
    uint16_t *plane = nullptr;
    int32_t *table = nullptr, *out = nullptr;
    hipStream_t cs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamSynchronize(caller);
    if (e == hipSuccess) e = hipMalloc(&plane, plane_elems * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMalloc(&table, kFloorTable * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&out, kFloorTable * sizeof(int32_t));
    if (e == hipSuccess) {  // pseudo-random plane values, a zero table and output
        std::vector<uint16_t> h(plane_elems);
        uint32_t x = 12345u;
        for (auto &v : h) v = (uint16_t)((x = x * 1664525u + 1013904223u) >> 16);
        e = hipMemcpy(plane, h.data(), plane_elems * sizeof(uint16_t), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(table, 0, kFloorTable * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(out, 0, kFloorTable * sizeof(int32_t));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int kind = 0; kind < 3 && e == hipSuccess; ++kind) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        for (int i = 0; i < launches && e == hipSuccess; ++i) {
            if (kind == 0)
                hipLaunchKernelGGL(k_floor_empty, dim3(groups), dim3(kMbThreads), 0, cs, out);
            else if (kind == 1)
                hipLaunchKernelGGL(k_floor_one, dim3(groups), dim3(kMbThreads), 0, cs, plane, out,
                                   -1);
            else
                hipLaunchKernelGGL(k_floor_two, dim3(groups), dim3(kMbThreads), 0, cs, plane, table,
                                   out, -1);
            e = hipGetLastError();
        }
        const hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = ec;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        float best = 0.f;
        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // rep 0 warms up
            e = hipEventRecord(e0, cs);
            if (e == hipSuccess) e = hipGraphLaunch(exec, cs);
            if (e == hipSuccess) e = hipEventRecord(e1, cs);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && rep > 0 && (best == 0.f || ms < best)) best = ms;
        }
        if (e == hipSuccess) us[kind] = best * 1e3 / launches;
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (cs) (void)hipStreamDestroy(cs);
    if (plane) (void)hipFree(plane);
    if (table) (void)hipFree(table);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return set_error(SEEDS_E_DEVICE, "launch floor benchmark: %s", hipGetErrorString(e));
    return SEEDS_OK;
}

extern "C" seeds_status seeds_lds_atomic_rate(double *ginst_per_s, void *hip_stream) {
    if (!ginst_per_s) return set_error(SEEDS_E_INVAL, "output is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    int32_t *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&out, kMbGroups * sizeof(int32_t));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 0.f;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // rep 0 warms up
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_lds_atomics, dim3(kMbGroups), dim3(kMbThreads), 0, s, out);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0 && (best == 0.f || ms < best)) best = ms;
    }
    int32_t check = 0;
    if (e == hipSuccess) e = hipMemcpy(&check, out, 4, hipMemcpyDeviceToHost);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return set_error(SEEDS_E_DEVICE, "LDS atomic benchmark: %s", hipGetErrorString(e));
    if (check != kMbIters) return set_error(SEEDS_E_DEVICE, "LDS atomic benchmark: count %d", check);
    const double insts = (double)kMbGroups * (kMbThreads / 64) * kMbIters;
    *ginst_per_s = insts / (best * 1e-3) / 1e9;
    return SEEDS_OK;
}
