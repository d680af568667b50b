// Measurement hooks. The LDS-atomic throughput of the device, the secondary
// roof of the refinement kernels (their per-workgroup histograms and delta
// tables are LDS integer atomics). Every lane adds to its own LDS word, so a
// wavefront instruction touches 64 distinct words in distinct banks and
// nothing conflicts; the rate is wavefront instructions per second.
#include <hip/hip_runtime.h>

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

}  // namespace
}  // namespace seeds

using namespace seeds;

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
