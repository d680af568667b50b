// Internal declarations shared by the host side (seeds_capi.cpp) and the
// kernels (seeds_kernels.hip) of libseeds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "seeds.h"

namespace seeds {

// Histogram rows are padded so every row starts on a 32-byte boundary.
inline int hist_stride(int nbins) { return (nbins + 7) & ~7; }

struct Dims {
    int H, W;        // image
    int B, nb, hs;   // bins per channel, B^3, padded histogram row stride
    int L, I;        // levels, sweeps per level
    int gamma, rule;
    int gx, gy, K;   // superpixel grid, K = gx * gy
    int T;           // top block side 2^(L-1)
};

// Unit grid of level l: ceil(W / 2^l) x ceil(H / 2^l).
inline int units_w(const Dims &d, int level) { return (d.W + (1 << level) - 1) >> level; }
inline int units_h(const Dims &d, int level) { return (d.H + (1 << level) - 1) >> level; }

// Number of units of class c (3 (uy mod 3) + (ux mod 3)) on a uw x uh grid.
__host__ __device__ inline int class_cols(int uw, int cls) { return cls % 3 < uw ? (uw - cls % 3 + 2) / 3 : 0; }
__host__ __device__ inline int class_rows(int uh, int cls) { return cls / 3 < uh ? (uh - cls / 3 + 2) / 3 : 0; }

struct Buffers {
    uint8_t *bins;   // H*W colour bin of every pixel
    int32_t *lab;    // H*W pixel labels (valid at level 0)
    int32_t *bl[2];  // block-label grids, ping-pong (levels >= 1)
    int32_t *hist;   // K*hs colour histograms in pixel counts
    int32_t *size;   // K superpixel sizes
    int32_t *src;    // K phase stamps of move sources (exact rule's drop rule)
    int32_t *pend;   // one decision per class unit: target label or -1
};

// Launchers (seeds_kernels.hip). They only enqueue work and return the launch
// status; shapes are checked by the caller.
hipError_t launch_fill(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_init(const Dims &d, const Buffers &b, const uint8_t *rgb, int64_t pitch,
                       int32_t *top_labels, hipStream_t s);
hipError_t launch_phase(const Dims &d, const Buffers &b, int level, const int32_t *blab,
                        int32_t *blab_w, int cls, uint32_t stamp, hipStream_t s);
hipError_t launch_upsample(const int32_t *from, int fw, int fh, int32_t *to, int tw, int th,
                           hipStream_t s);
hipError_t launch_expand(const Dims &d, const int32_t *blab, int level, int32_t *out,
                         hipStream_t s);

}  // namespace seeds
