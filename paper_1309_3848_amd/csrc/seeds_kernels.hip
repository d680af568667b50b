// SEEDS kernels for gfx950: fills, initialisation (quantise, grid,
// histograms), the warm start of a stream frame and label expansion. The phases themselves are in
// seeds_phase.hip (one launch per phase) and seeds_persistent.hip (one
// launch per refinement).
#include "seeds_device.h"
#include "seeds_readback.h"

namespace seeds {
namespace {

constexpr int kThreads = 256;

__global__ void k_fill(int32_t *__restrict__ p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// Initialisation (Sec. 5.1): bins of every pixel, labels of the top blocks,
// colour histograms and sizes of every superpixel.
//
// A workgroup covers a 64 x 16 pixel tile. The superpixels of the initial
// grid are rectangles, so a tile meets a small rectangle of them; their
// histograms are accumulated in LDS and merged into the global ones once
// per (superpixel, bin). Tiles that meet more than kMaxSlots superpixels
// (tiny superpixels) fall back to global atomics.
constexpr int kMaxSlots = 32, kMaxHs = 224;  // hs <= 224 for B <= 6

__device__ __forceinline__ int grid_col(int x, const Dims &d, int bw) {
    return (int)(((int64_t)(x / d.T) * d.gx) / bw);
}
__device__ __forceinline__ int grid_row(int y, const Dims &d, int bh) {
    return (int)(((int64_t)(y / d.T) * d.gy) / bh);
}

// The slots' histograms (kMaxSlots x hs) live in dynamic LDS sized for the
// launch's row stride, so that small histograms leave room for more
// workgroups per CU.
extern __shared__ int32_t dyn_hist[];
struct InitSlots {
    int32_t size[kMaxSlots];
    int32_t col[kInitTW], row[kMaxInitTH];  // superpixel column / row of the tile's columns / rows
};

// One tile of kInitTW x TH pixels of one image (TH / 4 pixels per thread).
// st0 / st1: the image's state in both copies.
template <int TH>
__device__ void init_tile(const Dims &d, const uint8_t *__restrict__ rgb, int64_t pitch,
                          uint8_t *__restrict__ bins, int32_t *__restrict__ top,
                          uint16_t *__restrict__ top16, int32_t *__restrict__ st0,
                          int32_t *__restrict__ st1, int tile, InitSlots &sl) {
    const int64_t khs = (int64_t)d.K * d.hs;
    const int bw = (d.W + d.T - 1) / d.T, bh = (d.H + d.T - 1) / d.T;
    const int tiles_x = (d.W + kInitTW - 1) / kInitTW;
    const int x0 = (tile % tiles_x) * kInitTW, y0 = (tile / tiles_x) * TH;
    const int x1 = min(x0 + kInitTW, d.W) - 1, y1 = min(y0 + TH, d.H) - 1;
    const int sx_lo = grid_col(x0, d, bw), sx_hi = grid_col(x1, d, bw);
    const int sy_lo = grid_row(y0, d, bh), sy_hi = grid_row(y1, d, bh);
    const int nsx = sx_hi - sx_lo + 1;
    const int nslots = nsx * (sy_hi - sy_lo + 1);
    const bool local = nslots <= kMaxSlots;
    // every pixel's colour is loaded first, from addresses clamped into the
    // image (a load behind a branch is waited for at the end of the branch)
    constexpr int kRows = TH * kInitTW / kThreads;
    const int x = x0 + (int)(threadIdx.x % kInitTW), xc = min(x, d.W - 1);
    uint8_t c0[kRows], c1[kRows], c2[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        const int yc = min(y0 + (int)(threadIdx.x / kInitTW) + q * (kThreads / kInitTW), d.H - 1);
        const uint8_t *p = rgb + (int64_t)yc * pitch + 3 * (int64_t)xc;
        c0[q] = p[0];
        c1[q] = p[1];
        c2[q] = p[2];
    }
    if (local) {
        for (int i = threadIdx.x; i < nslots * d.hs; i += kThreads) dyn_hist[i] = 0;
        for (int i = threadIdx.x; i < nslots; i += kThreads) sl.size[i] = 0;
    }
    // the grid position of each column and row of the tile, one division
    // each instead of two 64-bit divisions per pixel
    if (threadIdx.x < kInitTW)
        sl.col[threadIdx.x] = grid_col(min(x0 + (int)threadIdx.x, d.W - 1), d, bw);
    else if (threadIdx.x < kInitTW + TH)
        sl.row[threadIdx.x - kInitTW] = grid_row(min(y0 + (int)threadIdx.x - kInitTW, d.H - 1), d, bh);
    __syncthreads();
    const int sh = __builtin_ctz(d.T);  // T is a power of two
    const int sx = sl.col[threadIdx.x % kInitTW];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
        const int r = (int)(threadIdx.x / kInitTW) + q * (kThreads / kInitTW);
        const int y = y0 + r;
        if (x >= d.W || y >= d.H) continue;
        const int j = (((c0[q] * d.B) >> 8) * d.B + ((c1[q] * d.B) >> 8)) * d.B + ((c2[q] * d.B) >> 8);
        bins[(int64_t)y * d.W + x] = (uint8_t)j;
        const int sy = sl.row[r];
        const int label = sy * d.gx + sx;
        if (((x | y) & (d.T - 1)) == 0) {
            if (top16)
                top16[(int64_t)(y >> sh) * bw + (x >> sh)] = (uint16_t)label;
            else
                top[(int64_t)(y >> sh) * bw + (x >> sh)] = label;
        }
        if (local) {
            const int slot = (sy - sy_lo) * nsx + (sx - sx_lo);
            atomicAdd(&dyn_hist[slot * d.hs + j], 1);
        } else {
            atomicAdd(&st0[(int64_t)label * d.hs + j], 1);
            atomicAdd(&st0[khs + label], 1);
            atomicAdd(&st1[(int64_t)label * d.hs + j], 1);
            atomicAdd(&st1[khs + label], 1);
        }
    }
    __syncthreads();
    if (!local) return;
    for (int i = threadIdx.x; i < nslots * d.hs; i += kThreads) {
        const int v = dyn_hist[i];
        if (!v) continue;
        const int slot = i / d.hs, j = i - slot * d.hs;
        const int label = (sy_lo + slot / nsx) * d.gx + sx_lo + slot % nsx;
        atomicAdd(&st0[(int64_t)label * d.hs + j], v);
        atomicAdd(&st1[(int64_t)label * d.hs + j], v);
        // sizes from the non-zero cells (far fewer LDS atomics on one address
        // than counting every pixel)
        atomicAdd(&sl.size[slot], v);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nslots; i += kThreads) {
        const int v = sl.size[i];
        if (!v) continue;
        const int label = (sy_lo + i / nsx) * d.gx + sx_lo + i % nsx;
        atomicAdd(&st0[khs + label], v);
        atomicAdd(&st1[khs + label], v);
    }
}

template <int TH>
__device__ __forceinline__ void init_image(const BatchArgs &b, const ImageDesc &g,
                                           const uint8_t *rgb, int64_t pitch, int tile,
                                           InitSlots &sl) {
    const Dims &d = g.d;
    // the top blocks' grid (level L-1) lives in block-grid buffer (L-1) % 2;
    // with one level the top blocks are the pixels (int32 or 16-bit plane)
    int32_t *top = d.L > 1 ? b.ar.bl + g.bl[(d.L - 1) & 1] : (b.ar.lab ? b.ar.lab + g.lab : nullptr);
    uint16_t *top16 = d.L == 1 && b.ar.lab16 ? b.ar.lab16 + g.lab : nullptr;
    init_tile<TH>(d, rgb, pitch, b.ar.bins + g.bins, top, top16, b.ar.state[0] + g.state,
                  b.ar.state[1] + g.state, tile, sl);
}

template <int TH>
__global__ __launch_bounds__(kThreads) void k_init(BatchArgs b, ImageDesc one,
                                                   const uint8_t *rgb_one, int64_t pitch_one,
                                                   const int2 *map,
                                                   const uint8_t *const *rgb_table,
                                                   const int64_t *pitch_table) {
    __shared__ InitSlots sl;
    const int lg = xcd_group();
    if (b.nimg == 1) {
        init_image<TH>(b, one, rgb_one, pitch_one, lg, sl);
        return;
    }
    const int2 e = map[lg];
    init_image<TH>(b, b.imgs[e.x], rgb_table[e.x], pitch_table[e.x], e.y, sl);
}

// Serving engine: items of newly admitted images. Their state regions are
// zeroed by one launch (both copies), then initialised by the next.
__global__ __launch_bounds__(kThreads) void k_zero_mixed(BatchArgs b, TickList l) {
    const int lg = xcd_group();
    const TickItem &it = l.items[find_tick_item(l, lg)];
    const int64_t n = (int64_t)it.g.d.K * it.g.d.hs + it.g.d.K;
    const int64_t lo = (int64_t)(lg - it.first) * kZeroPerGroup;
    const int64_t hi = min(n, lo + kZeroPerGroup);
    int32_t *s0 = b.ar.state[0] + it.g.state, *s1 = b.ar.state[1] + it.g.state;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
        s0[i] = 0;
        s1[i] = 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_init_mixed(BatchArgs b, TickList l) {
    __shared__ InitSlots sl;
    const int lg = xcd_group();
    const TickItem &it = l.items[find_tick_item(l, lg)];
    init_image<kInitTH>(b, it.g, it.rgb, it.pitch, lg - it.first, sl);
}

// ---------------------------------------------------------------------------
// Warm start on a new frame: bins of every pixel from the new frame (Sec.
// 4.1) and the colour histograms and sizes of the superpixels from the labels
// the pixels already carry (eq. eqColorHistogram).
//
// A workgroup covers a 64 x 16 pixel tile, as in the initialisation, but the
// labels are arbitrary: the tile's distinct labels are first collected in a
// small LDS hash table, each gets an LDS histogram slot, the pixels are
// counted there and every non-zero count is merged once. Labels beyond the
// table or the slots (tiny superpixels) go straight to global atomics.
constexpr int kRehistKeys = 64, kRehistSlots = 32;

struct RehistLds {
    int32_t key[kRehistKeys];   // label, or -1
    int32_t slot[kRehistKeys];  // histogram slot of the label, or -1 (global)
    int32_t nslots;  // histograms: kRehistSlots x hs in dynamic LDS (dyn_hist)
    int32_t size[kRehistSlots];
    int32_t label[kRehistSlots];
};

// Entry of label k in the key table (inserting it when `insert`), or -1.
__device__ __forceinline__ int rehist_entry(RehistLds &r, int32_t k, bool insert) {
    uint32_t h = ((uint32_t)k * 2654435761u) >> 26;  // 6 bits
#pragma nounroll
    for (int p = 0; p < kRehistKeys; ++p, h = (h + 1) & (kRehistKeys - 1)) {
        const int32_t cur = insert ? atomicCAS(&r.key[h], -1, k) : r.key[h];
        if (cur == k || (insert && cur == -1)) return (int)h;
        if (cur == -1) return -1;
    }
    return -1;
}

template <typename LabT, int TH>
__device__ void rehist_tile(const Dims &d, const uint8_t *__restrict__ rgb, int64_t pitch,
                            uint8_t *__restrict__ bins, const LabT *__restrict__ lab,
                            int32_t *__restrict__ st0, int32_t *__restrict__ st1, int tile,
                            RehistLds &r) {
    constexpr int kRehistPx = kInitTW * TH / kThreads;  // pixels per thread
    const int64_t khs = (int64_t)d.K * d.hs;
    const int tiles_x = (d.W + kInitTW - 1) / kInitTW;
    const int x0 = (tile % tiles_x) * kInitTW, y0 = (tile / tiles_x) * TH;
    for (int i = threadIdx.x; i < kRehistKeys; i += kThreads) {
        r.key[i] = -1;
        r.slot[i] = -1;
    }
    if (threadIdx.x == 0) r.nslots = 0;
    __syncthreads();
    // the thread's pixels: bins (written now) and labels, kept in registers.
    // Every pixel's loads go out first, from addresses clamped into the image
    // (a load behind a branch is waited for at the end of the branch).
    int32_t k[kRehistPx], j[kRehistPx], ent[kRehistPx];
    uint8_t c0[kRehistPx], c1[kRehistPx], c2[kRehistPx];
    const int x = x0 + (int)(threadIdx.x % kInitTW), xc = min(x, d.W - 1);
#pragma unroll
    for (int q = 0; q < kRehistPx; ++q) {
        const int y = y0 + (int)(threadIdx.x / kInitTW) + q * (kThreads / kInitTW);
        const int yc = min(y, d.H - 1);
        const uint8_t *p = rgb + (int64_t)yc * pitch + 3 * (int64_t)xc;
        c0[q] = p[0];
        c1[q] = p[1];
        c2[q] = p[2];
        k[q] = (int32_t)lab[(int64_t)yc * d.W + xc];
    }
    const int lane = threadIdx.x & 63;
    // the wavefront's last four (label, entry) pairs: the rows of one thread
    // are 4 apart and mostly meet the same labels
    constexpr int kSeen = 4;
    int seen_key[kSeen], seen_ent[kSeen];
#pragma unroll
    for (int c = 0; c < kSeen; ++c) seen_key[c] = seen_ent[c] = -1;
#pragma unroll
    for (int q = 0; q < kRehistPx; ++q) {
        const int y = y0 + (int)(threadIdx.x / kInitTW) + q * (kThreads / kInitTW);
        j[q] = 0;
        if (x < d.W && y < d.H) {
            j[q] = (((c0[q] * d.B) >> 8) * d.B + ((c1[q] * d.B) >> 8)) * d.B + ((c2[q] * d.B) >> 8);
            bins[(int64_t)y * d.W + x] = (uint8_t)j[q];
        } else {
            k[q] = -1;
        }
        // each distinct label of the wavefront is inserted once, by its first
        // lane (neighbouring pixels mostly share labels: one insert per lane
        // would queue on a single LDS address); every lane with that label
        // keeps the entry, so the counting pass needs no second look-up
        ent[q] = -1;
        uint64_t pending = __ballot(k[q] >= 0);
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;  // wave-uniform
            const int key = __builtin_amdgcn_readlane(k[q], leader);
            int h = -2;
#pragma unroll
            for (int c = 0; c < kSeen; ++c)
                if (seen_key[c] == key) h = seen_ent[c];
            if (h == -2) {
                h = -1;
                if (lane == leader) h = rehist_entry(r, key, true);
                h = __builtin_amdgcn_readlane(h, leader);
#pragma unroll
                for (int c = kSeen - 1; c > 0; --c) {
                    seen_key[c] = seen_key[c - 1];
                    seen_ent[c] = seen_ent[c - 1];
                }
                seen_key[0] = key;
                seen_ent[0] = h;
            }
            const bool mine = k[q] == key;
            if (mine) ent[q] = h;
            pending &= ~__ballot(mine);
        }
    }
    __syncthreads();
    // a slot per distinct label while slots last
    for (int i = threadIdx.x; i < kRehistKeys; i += kThreads) {
        if (r.key[i] < 0) continue;
        const int s = atomicAdd(&r.nslots, 1);
        if (s < kRehistSlots) {
            r.slot[i] = s;
            r.label[s] = r.key[i];
        }
    }
    __syncthreads();
    const int ns = min(r.nslots, kRehistSlots);
    for (int i = threadIdx.x; i < ns * d.hs; i += kThreads) dyn_hist[i] = 0;
    for (int i = threadIdx.x; i < ns; i += kThreads) r.size[i] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRehistPx; ++q) {
        if (k[q] < 0) continue;
        const int s = ent[q] >= 0 ? r.slot[ent[q]] : -1;
        if (s >= 0) {
            atomicAdd(&dyn_hist[s * d.hs + j[q]], 1);
        } else {
            atomicAdd(&st0[(int64_t)k[q] * d.hs + j[q]], 1);
            atomicAdd(&st0[khs + k[q]], 1);
            atomicAdd(&st1[(int64_t)k[q] * d.hs + j[q]], 1);
            atomicAdd(&st1[khs + k[q]], 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ns * d.hs; i += kThreads) {
        const int v = dyn_hist[i];
        if (!v) continue;
        const int s = i / d.hs, jj = i - s * d.hs;
        atomicAdd(&st0[(int64_t)r.label[s] * d.hs + jj], v);
        atomicAdd(&st1[(int64_t)r.label[s] * d.hs + jj], v);
        atomicAdd(&r.size[s], v);  // sizes from the non-zero cells
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ns; i += kThreads) {
        const int v = r.size[i];
        if (!v) continue;
        atomicAdd(&st0[khs + r.label[i]], v);
        atomicAdd(&st1[khs + r.label[i]], v);
    }
}

template <typename LabT>
__device__ __forceinline__ const LabT *rehist_plane(const Arenas &a);
template <>
__device__ __forceinline__ const int32_t *rehist_plane<int32_t>(const Arenas &a) { return a.lab; }
template <>
__device__ __forceinline__ const uint16_t *rehist_plane<uint16_t>(const Arenas &a) { return a.lab16; }

template <typename LabT, int TH>
__global__ __launch_bounds__(kThreads) void k_rehist(BatchArgs b, ImageDesc one,
                                                     const uint8_t *rgb_one, int64_t pitch_one,
                                                     const int2 *map,
                                                     const uint8_t *const *rgb_table,
                                                     const int64_t *pitch_table) {
    __shared__ RehistLds r;
    const int lg = xcd_group();
    const LabT *lab = rehist_plane<LabT>(b.ar);
    if (b.nimg == 1) {
        rehist_tile<LabT, TH>(one.d, rgb_one, pitch_one, b.ar.bins, lab, b.ar.state[0],
                              b.ar.state[1], lg, r);
        return;
    }
    const int2 e = map[lg];
    const ImageDesc g = b.imgs[e.x];
    rehist_tile<LabT, TH>(g.d, rgb_table[e.x], pitch_table[e.x], b.ar.bins + g.bins, lab + g.lab,
                          b.ar.state[0] + g.state, b.ar.state[1] + g.state, e.y, r);
}

// 16-bit pixel labels to int32 and back (readback, snapshots), over the
// whole device.
__global__ __launch_bounds__(kThreads) void k_widen(int32_t *__restrict__ dst,
                                                    const uint16_t *__restrict__ src, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
        dst[i] = (int32_t)src[i];
}

// The same for every image of a readback list in one launch: workgroup row
// blockIdx.y serves image blockIdx.y, its gridDim.x workgroups stride over it.
__global__ __launch_bounds__(kThreads) void k_widen_list(ReadbackList l) {
    const int i = blockIdx.y;
    const uint16_t *__restrict__ src = l.src[i];
    int32_t *__restrict__ dst = l.dst[i];
    const int64_t n = l.n[i], stride = (int64_t)gridDim.x * kThreads;
    for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < n; k += stride)
        dst[k] = (int32_t)src[k];
}

__global__ __launch_bounds__(kThreads) void k_narrow(uint16_t *__restrict__ dst,
                                                     const int32_t *__restrict__ src, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
        dst[i] = (uint16_t)src[i];
}

// ---------------------------------------------------------------------------
// Pixel labels of one image from a block grid of a level (output of a state
// stopped at a block level).
// One workgroup per (row, chunk of kThreads columns).
__global__ __launch_bounds__(kThreads) void k_expand(const int32_t *__restrict__ blab, int uw,
                                                     int level, int W, int chunks,
                                                     int32_t *__restrict__ out) {
    const int it = xcd_group();
    const int y = it / chunks, x = (it - y * chunks) * kThreads + (int)threadIdx.x;
    if (x < W) out[(int64_t)y * W + x] = blab[(int64_t)(y >> level) * uw + (x >> level)];
}

// Copy of labels. Out to pinned host memory it runs as a narrow kernel: a few
// workgroups stream the copy over PCIe while the rest of the device keeps
// refining; device to device it spreads over the whole device. The source is
// 16-byte aligned; the destination takes 16-byte stores when it is.
__global__ __launch_bounds__(kThreads) void k_copy_out(int32_t *__restrict__ dst,
                                                       const int32_t *__restrict__ src,
                                                       int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    int64_t done = 0;
    if (((uintptr_t)dst & 15) == 0) {
        const int64_t n4 = n / 4;
        for (int64_t k = i; k < n4; k += stride)
            reinterpret_cast<int4 *>(dst)[k] = reinterpret_cast<const int4 *>(src)[k];
        done = n4 * 4;
    }
    for (int64_t k = done + i; k < n; k += stride) dst[k] = src[k];
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_fill(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned g = blocks_for(n, kThreads) < 4096u ? blocks_for(n, kThreads) : 4096u;
    hipLaunchKernelGGL(k_fill, dim3(g), dim3(kThreads), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_init(const BatchArgs &b, const ImageDesc &one, const uint8_t *rgb_one,
                       int64_t pitch_one, const int2 *map, const uint8_t *const *rgb_table,
                       const int64_t *pitch_table, int groups, int rows, hipStream_t s) {
    decltype(&k_init<kInitTH>) fn = rows == 8 ? k_init<8> : rows == 32 ? k_init<32> : k_init<16>;
    hipLaunchKernelGGL(fn, dim3(groups), dim3(kThreads), kMaxSlots * one.d.hs * 4, s, b, one,
                       rgb_one, pitch_one, map, rgb_table, pitch_table);
    return hipGetLastError();
}

hipError_t launch_zero_mixed(const BatchArgs &b, const TickList &l, int groups, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_mixed, dim3(groups), dim3(kThreads), 0, s, b, l);
    return hipGetLastError();
}

hipError_t launch_init_mixed(const BatchArgs &b, const TickList &l, int groups, hipStream_t s) {
    hipLaunchKernelGGL(k_init_mixed, dim3(groups), dim3(kThreads), kMaxSlots * l.hs * 4, s, b, l);
    return hipGetLastError();
}

hipError_t launch_rehist(const BatchArgs &b, const ImageDesc &one, const uint8_t *rgb_one,
                         int64_t pitch_one, const int2 *map, const uint8_t *const *rgb_table,
                         const int64_t *pitch_table, int groups, int rows, hipStream_t s) {
    decltype(&k_rehist<int32_t, kInitTH>) fn;
    if (b.ar.lab16)
        fn = rows == 8 ? k_rehist<uint16_t, 8> : rows == 32 ? k_rehist<uint16_t, 32>
                                                            : k_rehist<uint16_t, 16>;
    else
        fn = rows == 8 ? k_rehist<int32_t, 8> : rows == 32 ? k_rehist<int32_t, 32>
                                                           : k_rehist<int32_t, 16>;
    hipLaunchKernelGGL(fn, dim3(groups), dim3(kThreads), kRehistSlots * one.d.hs * 4, s, b, one,
                       rgb_one, pitch_one, map, rgb_table, pitch_table);
    return hipGetLastError();
}

hipError_t launch_copy_labels(int32_t *dst, const Arenas &a, int64_t at, int64_t n, hipStream_t s) {
    if (!a.lab16) return launch_copy(dst, a.lab + at, n, s);
    if (n <= 0) return hipSuccess;
    const unsigned want = blocks_for(n, kThreads);
    hipLaunchKernelGGL(k_widen, dim3(want > 8192u ? 8192u : want), dim3(kThreads), 0, s, dst,
                       a.lab16 + at, n);
    return hipGetLastError();
}

hipError_t launch_widen_list(const ReadbackList &l, hipStream_t s) {
    if (l.count <= 0) return hipSuccess;
    int64_t most = 0;
    for (int i = 0; i < l.count; ++i) most = l.n[i] > most ? l.n[i] : most;
    if (most <= 0) return hipSuccess;
    // about 8192 workgroups in all, at least one per image, none idle on the largest
    const unsigned per = (unsigned)(8192 / l.count), want = blocks_for(most, kThreads);
    const unsigned gx = want < per ? want : (per > 0 ? per : 1u);
    hipLaunchKernelGGL(k_widen_list, dim3(gx, (unsigned)l.count), dim3(kThreads), 0, s, l);
    return hipGetLastError();
}

hipError_t launch_narrow_labels(const Arenas &a, int64_t at, const int32_t *src, int64_t n,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned want = blocks_for(n, kThreads);
    hipLaunchKernelGGL(k_narrow, dim3(want > 8192u ? 8192u : want), dim3(kThreads), 0, s,
                       a.lab16 + at, src, n);
    return hipGetLastError();
}

hipError_t launch_copy_out(int32_t *dst, const int32_t *src, int64_t n, hipStream_t s) {
    constexpr int kCopyGroups = 16;
    hipLaunchKernelGGL(k_copy_out, dim3(kCopyGroups), dim3(kThreads), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_copy(int32_t *dst, const int32_t *src, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if ((uintptr_t)src & 15)
        return hipMemcpyAsync(dst, src, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
    // the same copy over the whole device: one 16-byte piece per lane
    const unsigned want = blocks_for((n + 3) / 4, kThreads);
    const unsigned g = want > 8192u ? 8192u : want;
    hipLaunchKernelGGL(k_copy_out, dim3(g), dim3(kThreads), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_expand(const Dims &d, const int32_t *blab, int level, int32_t *out,
                         hipStream_t s) {
    const int chunks = (int)blocks_for(d.W, kThreads);
    hipLaunchKernelGGL(k_expand, dim3((unsigned)(chunks * d.H)), dim3(kThreads), 0, s, blab,
                       units_w(d, level), level, d.W, chunks, out);
    return hipGetLastError();
}

}  // namespace seeds
