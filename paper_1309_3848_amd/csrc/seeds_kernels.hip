// SEEDS kernels for gfx950: initialisation (quantise, grid, histograms),
// block-level and pixel-level phases (decide, apply), level transitions.
//
// Every phase is two launches: "decide" reads the state at the start of the
// phase and writes one decision per unit of the class; "apply" moves the
// accepted units and updates the colour histograms (Sec. 5.3.3). The kernel
// boundary between them is the phase snapshot.
#include "seeds_internal.h"

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
constexpr int kInitTW = 64, kInitTH = 16;
constexpr int kMaxSlots = 32, kMaxHs = 224;  // hs <= 224 for B <= 6

__device__ __forceinline__ int grid_col(int x, const Dims &d, int bw) {
    return (int)(((int64_t)(x / d.T) * d.gx) / bw);
}
__device__ __forceinline__ int grid_row(int y, const Dims &d, int bh) {
    return (int)(((int64_t)(y / d.T) * d.gy) / bh);
}

__global__ __launch_bounds__(kThreads) void k_init(Dims d, const uint8_t *__restrict__ rgb,
                                                   int64_t pitch, uint8_t *__restrict__ bins,
                                                   int32_t *__restrict__ top,
                                                   int32_t *__restrict__ hist,
                                                   int32_t *__restrict__ size) {
    __shared__ int32_t sh_hist[kMaxSlots * kMaxHs];
    __shared__ int32_t sh_size[kMaxSlots];
    const int bw = (d.W + d.T - 1) / d.T, bh = (d.H + d.T - 1) / d.T;
    const int tiles_x = (d.W + kInitTW - 1) / kInitTW;
    const int x0 = (int)(blockIdx.x % tiles_x) * kInitTW, y0 = (int)(blockIdx.x / tiles_x) * kInitTH;
    const int x1 = min(x0 + kInitTW, d.W) - 1, y1 = min(y0 + kInitTH, d.H) - 1;
    const int sx_lo = grid_col(x0, d, bw), sx_hi = grid_col(x1, d, bw);
    const int sy_lo = grid_row(y0, d, bh), sy_hi = grid_row(y1, d, bh);
    const int nsx = sx_hi - sx_lo + 1;
    const int nslots = nsx * (sy_hi - sy_lo + 1);
    const bool local = nslots <= kMaxSlots;
    if (local) {
        for (int i = threadIdx.x; i < nslots * d.hs; i += kThreads) sh_hist[i] = 0;
        for (int i = threadIdx.x; i < nslots; i += kThreads) sh_size[i] = 0;
    }
    __syncthreads();
    const int x = x0 + (int)(threadIdx.x % kInitTW);
    for (int r = threadIdx.x / kInitTW; r < kInitTH; r += kThreads / kInitTW) {
        const int y = y0 + r;
        if (x >= d.W || y >= d.H) continue;
        const uint8_t *p = rgb + (int64_t)y * pitch + 3 * (int64_t)x;
        const int j = (((p[0] * d.B) >> 8) * d.B + ((p[1] * d.B) >> 8)) * d.B + ((p[2] * d.B) >> 8);
        bins[(int64_t)y * d.W + x] = (uint8_t)j;
        const int sx = grid_col(x, d, bw), sy = grid_row(y, d, bh);
        const int label = sy * d.gx + sx;
        if (x % d.T == 0 && y % d.T == 0) top[(int64_t)(y / d.T) * bw + x / d.T] = label;
        if (local) {
            const int slot = (sy - sy_lo) * nsx + (sx - sx_lo);
            atomicAdd(&sh_hist[slot * d.hs + j], 1);
            atomicAdd(&sh_size[slot], 1);
        } else {
            atomicAdd(&hist[(int64_t)label * d.hs + j], 1);
            atomicAdd(&size[label], 1);
        }
    }
    __syncthreads();
    if (!local) return;
    for (int i = threadIdx.x; i < nslots * d.hs; i += kThreads) {
        const int v = sh_hist[i];
        if (!v) continue;
        const int slot = i / d.hs, j = i - slot * d.hs;
        const int label = (sy_lo + slot / nsx) * d.gx + sx_lo + slot % nsx;
        atomicAdd(&hist[(int64_t)label * d.hs + j], v);
    }
    for (int i = threadIdx.x; i < nslots; i += kThreads) {
        const int v = sh_size[i];
        if (v) atomicAdd(&size[(sy_lo + i / nsx) * d.gx + sx_lo + i % nsx], v);
    }
}

// ---------------------------------------------------------------------------
// Neighbourhood of a unit on a unit grid: the ring mask (bit i: ring cell i
// of N, NE, E, SE, S, SW, W, NW carries label k), the distinct labels other
// than k among the four edge neighbours in ascending order (unused slots
// hold kNoLabel, which sorts last), and whether k stays connected without the
// unit.
constexpr int kNoLabel = 0x7FFFFFFF;

struct Neighbourhood {
    int k;
    int nc;
    int cand[4];
    bool movable;  // boundary unit whose removal keeps k connected
};

// k stays 4-connected around the unit iff the edge neighbours of label k lie
// in one cyclic run of k cells on the ring (consecutive ring cells are
// 4-adjacent); a run made of a lone corner touches no edge neighbour and does
// not count. With no edge neighbour of label k the unit is all of k.
__device__ __forceinline__ bool ring_keeps_connected(uint32_t r) {
    if (!(r & 0x55u)) return false;
    if (r == 0xFFu) return true;
    const uint32_t prev = ((r << 1) | (r >> 7)) & 0xFFu;  // bit i: cell i-1
    const uint32_t next = ((r >> 1) | (r << 7)) & 0xFFu;  // bit i: cell i+1
    const uint32_t starts = r & ~prev;
    const uint32_t lone_corners = r & ~prev & ~next & 0xAAu;
    return __popc(starts) - __popc(lone_corners) == 1;
}

__device__ __forceinline__ Neighbourhood neighbourhood(const int32_t *__restrict__ units, int uw,
                                                       int uh, int ux, int uy) {
    Neighbourhood nb;
    const int64_t row = (int64_t)uy * uw;
    nb.k = units[row + ux];
    const bool hasN = uy > 0, hasS = uy + 1 < uh, hasW = ux > 0, hasE = ux + 1 < uw;
    const int lN = hasN ? units[row - uw + ux] : -1;
    const int lS = hasS ? units[row + uw + ux] : -1;
    const int lW = hasW ? units[row + ux - 1] : -1;
    const int lE = hasE ? units[row + ux + 1] : -1;
    const int lNE = hasN && hasE ? units[row - uw + ux + 1] : -1;
    const int lSE = hasS && hasE ? units[row + uw + ux + 1] : -1;
    const int lSW = hasS && hasW ? units[row + uw + ux - 1] : -1;
    const int lNW = hasN && hasW ? units[row - uw + ux - 1] : -1;
    const int k = nb.k;
    const uint32_t r = (lN == k) | (lNE == k) << 1 | (lE == k) << 2 | (lSE == k) << 3 |
                       (lS == k) << 4 | (lSW == k) << 5 | (lW == k) << 6 | (lNW == k) << 7;
    // edge neighbours, keeping the first occurrence of each other label
    int c0 = (lN < 0 || lN == k) ? kNoLabel : lN;
    int c1 = (lE < 0 || lE == k || lE == c0) ? kNoLabel : lE;
    int c2 = (lS < 0 || lS == k || lS == c0 || lS == c1) ? kNoLabel : lS;
    int c3 = (lW < 0 || lW == k || lW == c0 || lW == c1 || lW == c2) ? kNoLabel : lW;
    // sorting network on four values
#define SEEDS_CSWAP(a, b)              \
    {                                  \
        const int lo = min(a, b);      \
        b = max(a, b);                 \
        a = lo;                        \
    }
    SEEDS_CSWAP(c0, c1) SEEDS_CSWAP(c2, c3) SEEDS_CSWAP(c0, c2) SEEDS_CSWAP(c1, c3)
    SEEDS_CSWAP(c1, c2)
#undef SEEDS_CSWAP
    nb.cand[0] = c0;
    nb.cand[1] = c1;
    nb.cand[2] = c2;
    nb.cand[3] = c3;
    const int nc = (c0 != kNoLabel) + (c1 != kNoLabel) + (c2 != kNoLabel) + (c3 != kNoLabel);
    nb.nc = nc;
    nb.movable = nc > 0 && ring_keeps_connected(r);
    return nb;
}

// ---------------------------------------------------------------------------
// Block level, decide. A segment of SEG lanes handles one block of side
// s = 2^level (SEG * PPL = s * s pixels). The block's bins are staged in LDS;
// every pixel that is the first of its bin in the block contributes, for its
// bin j with block count h_l(j):
//   INTERSECT: min(h_x(j) m, h_l(j) A_x) to S_x for every candidate x, and
//              min((h_k(j) - h_l(j)) m, h_l(j) (A_k - m)) to S_{k\l};
//   EXACT:     h_l(j) (h_x(j) - h_k(j) + h_l(j)) to g_x.
// The sums are reduced over the segment; its first lane decides.
template <int SEG>
__device__ __forceinline__ int64_t segment_sum(int64_t v) {
#pragma unroll
    for (int off = SEG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, SEG);
    return v;
}

template <int SEG, int PPL, int THREADS>
__global__ __launch_bounds__(THREADS) void k_block_decide(
    Dims d, int level, int cls, const int32_t *__restrict__ units, int uw, int uh,
    const uint8_t *__restrict__ bins, const int32_t *__restrict__ hist,
    const int32_t *__restrict__ size, int32_t *__restrict__ pend, int32_t *__restrict__ src,
    uint32_t stamp) {
    constexpr int SEGS = THREADS / SEG;
    constexpr int NPX = SEG * PPL;
    __shared__ uint8_t sbin[SEGS * NPX];
    const int s = 1 << level;
    const int seg = threadIdx.x / SEG, lane = threadIdx.x % SEG;
    const int ncx = class_cols(uw, cls), ncy = class_rows(uh, cls);
    const int unit = blockIdx.x * SEGS + seg;
    const bool in_range = unit < ncx * ncy;
    int ux = 0, uy = 0;
    Neighbourhood nb;
    nb.movable = false;
    nb.k = -1;
    nb.nc = 0;
    if (in_range) {
        ux = cls % 3 + 3 * (unit % ncx);
        uy = cls / 3 + 3 * (unit / ncx);
        nb = neighbourhood(units, uw, uh, ux, uy);
    }
    uint8_t *mine = sbin + seg * NPX;
#pragma unroll
    for (int t = 0; t < PPL; ++t) {
        const int q = lane + t * SEG;
        const int x = ux * s + (q & (s - 1)), y = uy * s + (q >> level);
        mine[q] = (nb.movable && x < d.W && y < d.H) ? bins[(int64_t)y * d.W + x] : 0xFF;
    }
    __syncthreads();
    if (!nb.movable) {
        if (in_range && lane == 0) pend[unit] = -1;
        return;
    }
    const int64_t m = (int64_t)min(s, d.W - ux * s) * min(s, d.H - uy * s);
    const int k = nb.k;
    const int64_t Ak = size[k];
    int64_t An[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (c < nb.nc) An[c] = size[nb.cand[c]];
    int64_t acc[4] = {0, 0, 0, 0}, acc_kl = 0;
    const bool exact = d.rule == SEEDS_BLOCK_EXACT;
#pragma unroll
    for (int t = 0; t < PPL; ++t) {
        const int q = lane + t * SEG;
        const int j = mine[q];
        if (j == 0xFF) continue;
        int cnt = 0;
        bool first = true;
        for (int q2 = 0; q2 < NPX; ++q2) {
            const bool same = mine[q2] == j;
            cnt += same;
            first &= !(same && q2 < q);
        }
        if (!first) continue;
        const int64_t hl = cnt;
        const int64_t hk = hist[(int64_t)k * d.hs + j];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= nb.nc) break;
            const int64_t hn = hist[(int64_t)nb.cand[c] * d.hs + j];
            if (exact) {
                acc[c] += hl * (hn - hk + hl);
            } else {
                const int64_t a = hn * m, b = hl * An[c];
                acc[c] += a < b ? a : b;
            }
        }
        if (!exact) {
            const int64_t a = (hk - hl) * m, b = hl * (Ak - m);
            acc_kl += a < b ? a : b;
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = segment_sum<SEG>(acc[c]);
    acc_kl = segment_sum<SEG>(acc_kl);
    if (lane != 0) return;
    // best candidate: largest g (EXACT) or largest S_x / A_x (INTERSECT);
    // candidates are ascending, so a strict comparison keeps the smaller label
    int64_t bS = acc[0], bA = An[0];
    int bn = nb.cand[0];
#pragma unroll
    for (int c = 1; c < 4; ++c) {
        if (c >= nb.nc) break;
        const bool better = exact ? acc[c] > bS : acc[c] * bA > bS * An[c];
        if (better) {
            bS = acc[c];
            bA = An[c];
            bn = nb.cand[c];
        }
    }
    const bool accept = exact ? bS > 0 : bS * (Ak - m) > acc_kl * bA;
    pend[unit] = accept ? bn : -1;
    if (accept && exact) __hip_atomic_store(&src[k], (int32_t)stamp, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
}

// Block level, apply: move accepted blocks (unless dropped under the exact
// rule) and move their pixels between the two colour histograms.
__global__ __launch_bounds__(kThreads) void k_block_apply(
    Dims d, int level, int cls, int32_t *__restrict__ units, int uw, int uh,
    const uint8_t *__restrict__ bins, int32_t *__restrict__ hist, int32_t *__restrict__ size,
    const int32_t *__restrict__ pend, const int32_t *__restrict__ src, uint32_t stamp) {
    const int ncx = class_cols(uw, cls), ncy = class_rows(uh, cls);
    const int unit = blockIdx.x * blockDim.x + threadIdx.x;
    if (unit >= ncx * ncy) return;
    const int n = pend[unit];
    if (n < 0) return;
    if (d.rule == SEEDS_BLOCK_EXACT && src[n] == (int32_t)stamp) return;
    const int s = 1 << level;
    const int ux = cls % 3 + 3 * (unit % ncx), uy = cls / 3 + 3 * (unit / ncx);
    int32_t *cell = &units[(int64_t)uy * uw + ux];
    const int k = *cell;
    *cell = n;
    const int xe = min((ux + 1) * s, d.W), ye = min((uy + 1) * s, d.H);
    int m = 0;
    for (int y = uy * s; y < ye; ++y)
        for (int x = ux * s; x < xe; ++x) {
            const int j = bins[(int64_t)y * d.W + x];
            atomicAdd(&hist[(int64_t)n * d.hs + j], 1);
            atomicSub(&hist[(int64_t)k * d.hs + j], 1);
            ++m;
        }
    atomicAdd(&size[n], m);
    atomicSub(&size[k], m);
}

// ---------------------------------------------------------------------------
// Pixel level, decide. One thread per pixel of the class.
//   colour part (Prop. 1, one look-up per side): h_n(j) - h_k(j) + 1
//   boundary part (Prop. 2): W_n + |K_p| - W_k, where W_x weighs label x over
//   the 5x5 window by how many in-image 3x3 patches around p's neighbours
//   contain the cell: per axis, |[p-1, p+1] clipped to the image  n  [q-1, q+1]|.
__device__ __forceinline__ int axis_weight(int p, int q, int n) {
    if (q < 0 || q >= n) return 0;
    const int lo = max(max(p - 1, 0), q - 1), hi = min(min(p + 1, n - 1), q + 1);
    return hi >= lo ? hi - lo + 1 : 0;
}

__global__ __launch_bounds__(kThreads) void k_pixel_decide(
    Dims d, int cls, const int32_t *__restrict__ lab, const uint8_t *__restrict__ bins,
    const int32_t *__restrict__ hist, int32_t *__restrict__ pend) {
    const int ncx = class_cols(d.W, cls), ncy = class_rows(d.H, cls);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncx * ncy) return;
    const int x = cls % 3 + 3 * (i % ncx), y = cls / 3 + 3 * (i / ncx);
    const Neighbourhood nb = neighbourhood(lab, d.W, d.H, x, y);
    if (!nb.movable) {
        pend[i] = -1;
        return;
    }
    const int k = nb.k;
    const int j = bins[(int64_t)y * d.W + x];
    const int hk = hist[(int64_t)k * d.hs + j];
    int g[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        g[c] = c < nb.nc ? hist[(int64_t)nb.cand[c] * d.hs + j] - hk + 1 : INT32_MIN / 2;
    if (d.gamma) {
        int wk = 0, wn[4] = {0, 0, 0, 0};
#pragma unroll
        for (int dy = -2; dy <= 2; ++dy) {
            const int wy = axis_weight(y, y + dy, d.H);
            if (!wy) continue;
#pragma unroll
            for (int dx = -2; dx <= 2; ++dx) {
                const int wx = axis_weight(x, x + dx, d.W);
                if (!wx) continue;
                const int l = lab[(int64_t)(y + dy) * d.W + x + dx];
                const int w = wx * wy;
                wk += l == k ? w : 0;
#pragma unroll
                for (int c = 0; c < 4; ++c) wn[c] += l == nb.cand[c] ? w : 0;
            }
        }
        const int kp = (min(x + 1, d.W - 1) - max(x - 1, 0) + 1) *
                       (min(y + 1, d.H - 1) - max(y - 1, 0) + 1);
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < nb.nc) g[c] += d.gamma * (wn[c] + kp - wk);
    }
    // ascending candidates and a strict ">" keep the smaller label on ties
    int bg = g[0], bn = nb.cand[0];
#pragma unroll
    for (int c = 1; c < 4; ++c)
        if (c < nb.nc && g[c] > bg) {
            bg = g[c];
            bn = nb.cand[c];
        }
    pend[i] = bg > 0 ? bn : -1;
}

__global__ __launch_bounds__(kThreads) void k_pixel_apply(
    Dims d, int cls, int32_t *__restrict__ lab, const uint8_t *__restrict__ bins,
    int32_t *__restrict__ hist, int32_t *__restrict__ size, const int32_t *__restrict__ pend) {
    const int ncx = class_cols(d.W, cls), ncy = class_rows(d.H, cls);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncx * ncy) return;
    const int n = pend[i];
    if (n < 0) return;
    const int x = cls % 3 + 3 * (i % ncx), y = cls / 3 + 3 * (i / ncx);
    const int64_t p = (int64_t)y * d.W + x;
    const int k = lab[p];
    lab[p] = n;
    const int j = bins[p];
    atomicAdd(&hist[(int64_t)n * d.hs + j], 1);
    atomicSub(&hist[(int64_t)k * d.hs + j], 1);
    atomicAdd(&size[n], 1);
    atomicSub(&size[k], 1);
}

// ---------------------------------------------------------------------------
// Level transitions: split every block into its 2x2 children (Sec. 5.1),
// or expand a block grid of a level into pixel labels.
__global__ __launch_bounds__(kThreads) void k_upsample(const int32_t *__restrict__ from, int fw,
                                                       int32_t *__restrict__ to, int tw, int th) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)tw * th) return;
    const int x = (int)(i % tw), y = (int)(i / tw);
    to[i] = from[(int64_t)(y >> 1) * fw + (x >> 1)];
}

__global__ __launch_bounds__(kThreads) void k_expand(const int32_t *__restrict__ blab, int uw,
                                                     int level, int W, int H,
                                                     int32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)W * H) return;
    const int x = (int)(i % W), y = (int)(i / W);
    out[i] = blab[(int64_t)(y >> level) * uw + (x >> level)];
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <int SEG, int PPL, int THREADS>
void block_decide(const Dims &d, const Buffers &b, int level, const int32_t *units, int cls,
                  uint32_t stamp, hipStream_t s) {
    const int uw = units_w(d, level), uh = units_h(d, level);
    const int n = class_cols(uw, cls) * class_rows(uh, cls);
    if (!n) return;
    constexpr int SEGS = THREADS / SEG;
    hipLaunchKernelGGL((k_block_decide<SEG, PPL, THREADS>), dim3(blocks_for(n, SEGS)),
                       dim3(THREADS), 0, s, d, level, cls, units, uw, uh, b.bins, b.hist, b.size,
                       b.pend, b.src, stamp);
}

}  // namespace

hipError_t launch_fill(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned g = blocks_for(n, kThreads) < 4096u ? blocks_for(n, kThreads) : 4096u;
    hipLaunchKernelGGL(k_fill, dim3(g), dim3(kThreads), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_init(const Dims &d, const Buffers &b, const uint8_t *rgb, int64_t pitch,
                       int32_t *top_labels, hipStream_t s) {
    hipError_t e = launch_fill(b.hist, 0, (int64_t)d.K * d.hs, s);
    if (e != hipSuccess) return e;
    if ((e = launch_fill(b.size, 0, d.K, s)) != hipSuccess) return e;
    const unsigned tiles = blocks_for(d.W, kInitTW) * blocks_for(d.H, kInitTH);
    hipLaunchKernelGGL(k_init, dim3(tiles), dim3(kThreads), 0, s, d, rgb, pitch, b.bins, top_labels,
                       b.hist, b.size);
    return hipGetLastError();
}

hipError_t launch_phase(const Dims &d, const Buffers &b, int level, const int32_t *units,
                        int32_t *units_w_, int cls, uint32_t stamp, hipStream_t s) {
    const int uw = units_w(d, level), uh = units_h(d, level);
    const int n = class_cols(uw, cls) * class_rows(uh, cls);
    if (!n) return hipSuccess;
    if (level == 0) {
        hipLaunchKernelGGL(k_pixel_decide, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, d,
                           cls, units, b.bins, b.hist, b.pend);
        hipLaunchKernelGGL(k_pixel_apply, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, d,
                           cls, units_w_, b.bins, b.hist, b.size, b.pend);
        return hipGetLastError();
    }
    switch (level) {
        case 1: block_decide<4, 1, 256>(d, b, level, units, cls, stamp, s); break;
        case 2: block_decide<16, 1, 256>(d, b, level, units, cls, stamp, s); break;
        case 3: block_decide<64, 1, 256>(d, b, level, units, cls, stamp, s); break;
        case 4: block_decide<64, 4, 64>(d, b, level, units, cls, stamp, s); break;
        case 5: block_decide<64, 16, 64>(d, b, level, units, cls, stamp, s); break;
        case 6: block_decide<64, 64, 64>(d, b, level, units, cls, stamp, s); break;
        case 7: block_decide<64, 256, 64>(d, b, level, units, cls, stamp, s); break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_block_apply, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, d,
                       level, cls, units_w_, uw, uh, b.bins, b.hist, b.size, b.pend, b.src, stamp);
    return hipGetLastError();
}

hipError_t launch_upsample(const int32_t *from, int fw, int fh, int32_t *to, int tw, int th,
                           hipStream_t s) {
    (void)fh;
    const int64_t n = (int64_t)tw * th;
    hipLaunchKernelGGL(k_upsample, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, from, fw,
                       to, tw, th);
    return hipGetLastError();
}

hipError_t launch_expand(const Dims &d, const int32_t *blab, int level, int32_t *out,
                         hipStream_t s) {
    const int64_t n = (int64_t)d.W * d.H;
    hipLaunchKernelGGL(k_expand, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, blab,
                       units_w(d, level), level, d.W, d.H, out);
    return hipGetLastError();
}

}  // namespace seeds
