// Measurement hook: the LDS-atomic throughput of the device, the secondary
// roof of the refinement kernels (their per-workgroup histograms and delta
// tables are LDS integer atomics). Every lane adds to its own LDS word, so a
// wavefront instruction touches 64 distinct words in distinct banks and
// nothing conflicts; the rate is wavefront instructions per second.
#include <hip/hip_runtime.h>

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

}  // namespace
}  // namespace seeds

using namespace seeds;

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
