// Test hook: the energies of a state in count form, as 64-bit sums.
//   H' = sum_k sum_j h_k(j)^2 over the colour histograms (the colour term of
//        Sec. 4 without its normalisation);
//   G' = sum_i sum_k b_i(k)^2 over the 3x3 patches N_i of the pixel labels
//        (the boundary term of Sec. 4), patches clipped at the image border.
// For one patch, sum_k b(k)^2 is the number of ordered pairs of its cells
// with equal labels, which needs no per-patch table.
//
// Test hook: boundary units of a unit grid (Sec. 5.2: a block or pixel is a
// boundary unit when a 4-neighbour in the image carries another label; only
// those units are proposed for a move), counted for one unit class or all,
// with the image pixels they cover.
#include <algorithm>

#include "seeds_internal.h"

namespace seeds {
namespace {

constexpr int kET = 256;

// Wavefront sum, then one atomic per wavefront.
__device__ __forceinline__ void add_wave(unsigned long long *out, unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}

__global__ __launch_bounds__(kET) void k_energy_h(const int32_t *hist, int K, int nb, int hs,
                                                  unsigned long long *out) {
    unsigned long long sum = 0;
    const int64_t n = (int64_t)K * nb;
    for (int64_t i = (int64_t)blockIdx.x * kET + threadIdx.x; i < n; i += (int64_t)gridDim.x * kET) {
        const int64_t k = i / nb, j = i - k * nb;
        const int64_t v = hist[k * hs + j];
        sum += (unsigned long long)(v * v);
    }
    add_wave(out, sum);
}

__global__ __launch_bounds__(kET) void k_energy_g(const int32_t *lab, int H, int W,
                                                  unsigned long long *out) {
    unsigned long long sum = 0;
    const int64_t n = (int64_t)H * W;
    for (int64_t i = (int64_t)blockIdx.x * kET + threadIdx.x; i < n; i += (int64_t)gridDim.x * kET) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        int l[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int yy = y + q / 3 - 1, xx = x + q % 3 - 1;
            l[q] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? lab[(int64_t)yy * W + xx] : -1;
        }
        int pairs = 0;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            if (l[a] < 0) continue;
            pairs += 1;
#pragma unroll
            for (int b = a + 1; b < 9; ++b) pairs += l[b] == l[a] ? 2 : 0;
        }
        sum += (unsigned long long)pairs;
    }
    add_wave(out, sum);
}

// out[0] += boundary units of class cls (cls < 0: every class) on the
// uw x uh grid of side `side`, out[1] += the in-image pixels they cover. The
// labels come from a grid `up` levels coarser (cw columns): unit (ux, uy)
// carries the label of its ancestor (ux >> up, uy >> up).
__global__ __launch_bounds__(kET) void k_boundary(const int32_t *units, int cw, int up, int uw,
                                                  int uh, int side, int H, int W, int cls,
                                                  unsigned long long *out) {
    unsigned long long nu = 0, np = 0;
    const int64_t n = (int64_t)uw * uh;
    auto at = [&](int x, int y) { return units[(int64_t)(y >> up) * cw + (x >> up)]; };
    for (int64_t i = (int64_t)blockIdx.x * kET + threadIdx.x; i < n; i += (int64_t)gridDim.x * kET) {
        const int uy = (int)(i / uw), ux = (int)(i - (int64_t)uy * uw);
        if (cls >= 0 && 3 * (uy % 3) + ux % 3 != cls) continue;
        const int32_t k = at(ux, uy);
        const bool boundary = (uy > 0 && at(ux, uy - 1) != k) || (uy + 1 < uh && at(ux, uy + 1) != k) ||
                              (ux > 0 && at(ux - 1, uy) != k) || (ux + 1 < uw && at(ux + 1, uy) != k);
        if (!boundary) continue;
        nu += 1;
        np += (unsigned long long)(min(side, W - ux * side) * min(side, H - uy * side));
    }
    add_wave(out, nu);
    add_wave(out + 1, np);
}

int grid_for(int64_t n) { return (int)std::min<int64_t>(2048, std::max<int64_t>(1, (n + kET - 1) / kET)); }

}  // namespace

hipError_t launch_energy(const int32_t *hist, const Dims &d, const int32_t *lab,
                         unsigned long long *out, hipStream_t s) {
    hipError_t e = launch_fill((int32_t *)out, 0, 4, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_h, dim3(grid_for((int64_t)d.K * d.nb)), dim3(kET), 0, s, hist, d.K,
                       d.nb, d.hs, out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_g, dim3(grid_for((int64_t)d.H * d.W)), dim3(kET), 0, s, lab, d.H,
                       d.W, out + 1);
    return hipGetLastError();
}

hipError_t launch_boundary(const int32_t *units, const Dims &d, int units_level, int level,
                           int cls, unsigned long long *out, hipStream_t s) {
    const int uw = units_w(d, level), uh = units_h(d, level);
    hipLaunchKernelGGL(k_boundary, dim3(grid_for((int64_t)uw * uh)), dim3(kET), 0, s, units,
                       units_w(d, units_level), units_level - level, uw, uh, 1 << level, d.H, d.W,
                       cls, out);
    return hipGetLastError();
}

}  // namespace seeds
