// Label readback of many images of a batch context in one launch: the list
// of (16-bit source plane, int32 output, pixel count) travels in the kernel
// arguments, at most kReadbackMax images per launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace seeds {

constexpr int kReadbackMax = 64;

struct ReadbackList {
    int count;
    const uint16_t *src[kReadbackMax];
    int32_t *dst[kReadbackMax];
    int64_t n[kReadbackMax];
};

// Widen every listed 16-bit label plane into its int32 output (stream-ordered).
hipError_t launch_widen_list(const ReadbackList &l, hipStream_t s);

}  // namespace seeds
