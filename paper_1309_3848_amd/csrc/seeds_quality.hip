// Quality metrics of a segmentation against ground truth (Sec. 6.1): the
// overlap counts |s_k & g_i| behind UE, CUE and ASA, and boundary recall.
//
// Boundary reading: a pixel lies on the boundary of a segmentation when one
// of its in-image 4-neighbours carries another segment; BR counts the
// ground-truth boundary pixels with a segmentation boundary pixel at
// Euclidean distance < eps.
#include "seeds_device.h"

namespace seeds {
namespace {

constexpr int kQT = 256;
constexpr int kQTW = 64, kQTH = 16;          // pixel tile of one workgroup
constexpr int kQPx = kQTW * kQTH / kQT;      // pixels per thread
constexpr int kQBits = 10, kQSize = 1 << kQBits, kQProbes = 32;

// counters: [0] UE, [1] ASA, [2] CUE, [3] BR hits, [4] |B(g)|, [5] range errors
struct QTable {
    int32_t key[kQSize];
    int32_t val[kQSize];
};

__device__ __forceinline__ bool seg_boundary(const int32_t *__restrict__ seg, int H, int W, int x,
                                             int y) {
    const int64_t i = (int64_t)y * W + x;
    const int32_t v = seg[i];
    return (x > 0 && seg[i - 1] != v) || (x + 1 < W && seg[i + 1] != v) ||
           (y > 0 && seg[i - W] != v) || (y + 1 < H && seg[i + W] != v);
}

__device__ __forceinline__ void wave_add(unsigned long long *dst, bool pred) {
    const unsigned long long b = __ballot(pred);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(dst, (unsigned long long)__popcll(b));
}

// Overlap counts (LDS-aggregated per tile, merged once per distinct (k, i))
// and the boundary-recall counts of one tile.
__global__ __launch_bounds__(kQT) void k_q_count(const int32_t *__restrict__ lab,
                                                 const int32_t *__restrict__ gt, int H, int W,
                                                 int K, int R, int eps,
                                                 int32_t *__restrict__ table,
                                                 unsigned long long *__restrict__ cnt) {
    __shared__ QTable t;
    for (int i = threadIdx.x; i < kQSize; i += kQT) {
        t.key[i] = -1;
        t.val[i] = 0;
    }
    __syncthreads();
    const int tiles_x = (W + kQTW - 1) / kQTW;
    const int tile = xcd_group();
    const int x = (tile % tiles_x) * kQTW + (int)(threadIdx.x % kQTW);
    const int y0 = (tile / tiles_x) * kQTH + (int)(threadIdx.x / kQTW);
    const int e2 = eps * eps;
#pragma unroll
    for (int q = 0; q < kQPx; ++q) {
        const int y = y0 + q * (kQT / kQTW);
        const bool in = x < W && y < H;
        bool tb = false, hit = false, bad = false;
        if (in) {
            const int64_t p = (int64_t)y * W + x;
            const int32_t k = lab[p], g = gt[p];
            bad = k < 0 || k >= K || g < 0 || g >= R;
            if (!bad) {
                const int32_t key = k * R + g;
                uint32_t h = ((uint32_t)key * 2654435761u) >> (32 - kQBits);
                bool done = false;
#pragma nounroll
                for (int pr = 0; pr < kQProbes && !done; ++pr, h = (h + 1) & (kQSize - 1)) {
                    const int32_t prev = atomicCAS(&t.key[h], -1, key);
                    if (prev == -1 || prev == key) {
                        atomicAdd(&t.val[h], 1);
                        done = true;
                    }
                }
                if (!done) atomicAdd(&table[key], 1);
                tb = seg_boundary(gt, H, W, x, y);
                if (tb) {
                    for (int dy = -eps + 1; dy < eps && !hit; ++dy)
                        for (int dx = -eps + 1; dx < eps && !hit; ++dx) {
                            if (dx * dx + dy * dy >= e2) continue;
                            const int qx = x + dx, qy = y + dy;
                            if (qx < 0 || qy < 0 || qx >= W || qy >= H) continue;
                            hit = seg_boundary(lab, H, W, qx, qy);
                        }
                }
            }
        }
        wave_add(&cnt[3], hit);
        wave_add(&cnt[4], tb);
        wave_add(&cnt[5], bad);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kQSize; i += kQT)
        if (t.key[i] >= 0) atomicAdd(&table[t.key[i]], t.val[i]);
}

// One wavefront per superpixel k: |s_k|, max_i |s_k & g_i| and the number of
// segments it meets. UE = sum_k (meets_k - 1) |s_k|, ASA = sum_k max_k,
// CUE = sum_k (|s_k| - max_k).
__global__ __launch_bounds__(kQT) void k_q_rows(const int32_t *__restrict__ table, int K, int R,
                                                unsigned long long *__restrict__ cnt) {
    const int k = blockIdx.x * (kQT / 64) + (int)(threadIdx.x / 64);
    const int lane = threadIdx.x & 63;
    if (k >= K) return;
    long long sum = 0, meets = 0;
    int mx = 0;
    for (int i = lane; i < R; i += 64) {
        const int v = table[(int64_t)k * R + i];
        sum += v;
        meets += v > 0;
        mx = max(mx, v);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sum += __shfl_xor(sum, off);
        meets += __shfl_xor(meets, off);
        mx = max(mx, __shfl_xor(mx, off));
    }
    if (lane == 0 && sum > 0) {
        atomicAdd(&cnt[0], (unsigned long long)((meets - 1) * sum));
        atomicAdd(&cnt[1], (unsigned long long)mx);
        atomicAdd(&cnt[2], (unsigned long long)(sum - mx));
    }
}

}  // namespace

hipError_t launch_quality(const int32_t *lab, const int32_t *gt, int H, int W, int K, int R,
                          int eps, int32_t *table, unsigned long long *cnt, hipStream_t s) {
    hipError_t e = launch_fill(table, 0, (int64_t)K * R, s);
    if (e == hipSuccess) e = launch_fill((int32_t *)cnt, 0, 12, s);
    if (e != hipSuccess) return e;
    const int tiles = ((W + kQTW - 1) / kQTW) * ((H + kQTH - 1) / kQTH);
    hipLaunchKernelGGL(k_q_count, dim3(tiles), dim3(kQT), 0, s, lab, gt, H, W, K, R, eps, table,
                       cnt);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_q_rows, dim3((K + kQT / 64 - 1) / (kQT / 64)), dim3(kQT), 0, s, table, K,
                       R, cnt);
    return hipGetLastError();
}

}  // namespace seeds
