// Device helpers shared by the per-step kernels and the persistent kernel.
#pragma once

#include "seeds_internal.h"

namespace seeds {

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

// Neighbourhood from the labels of the unit and its 8-ring (-1 outside).
__device__ __forceinline__ Neighbourhood neighbourhood9(int k, int lN, int lNE, int lE, int lSE,
                                                        int lS, int lSW, int lW, int lNW) {
    Neighbourhood nb;
    nb.k = k;
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

// Labels of a unit and its 8-ring on a unit grid (-1 outside), in the order
// unit, N, NE, E, SE, S, SW, W, NW. Loading apart from the test lets a caller
// issue other independent loads before it waits for these.
struct Ring {
    int l[9];
};

__device__ __forceinline__ Ring load_ring(const int32_t *__restrict__ units, int uw, int uh, int ux,
                                          int uy) {
    const int64_t row = (int64_t)uy * uw;
    const bool hasN = uy > 0, hasS = uy + 1 < uh, hasW = ux > 0, hasE = ux + 1 < uw;
    Ring r;
    r.l[0] = units[row + ux];
    r.l[1] = hasN ? units[row - uw + ux] : -1;
    r.l[2] = hasN && hasE ? units[row - uw + ux + 1] : -1;
    r.l[3] = hasE ? units[row + ux + 1] : -1;
    r.l[4] = hasS && hasE ? units[row + uw + ux + 1] : -1;
    r.l[5] = hasS ? units[row + uw + ux] : -1;
    r.l[6] = hasS && hasW ? units[row + uw + ux - 1] : -1;
    r.l[7] = hasW ? units[row + ux - 1] : -1;
    r.l[8] = hasN && hasW ? units[row - uw + ux - 1] : -1;
    return r;
}

__device__ __forceinline__ Neighbourhood neighbourhood(const Ring &r) {
    return neighbourhood9(r.l[0], r.l[1], r.l[2], r.l[3], r.l[4], r.l[5], r.l[6], r.l[7], r.l[8]);
}

// Workgroups are dispatched round-robin over the eight XCDs (workgroup b runs
// on XCD b mod 8), each with its own L2. Renumbering them so that every XCD
// gets a contiguous run of work keeps each XCD on one band of the image, so
// its L2 fetches that band's labels and only the histograms of the
// superpixels there. The renumbering is a bijection; results do not depend
// on it.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_group() {
    const int G = gridDim.x, b = blockIdx.x;
    const int q = G / kXcds, r = G % kXcds;
    const int x = b % kXcds, i = b / kXcds;
    return x * q + min(x, r) + i;
}

// Segment-wide sum over SEG consecutive lanes of a wavefront (SEG <= 64).
template <int SEG>
__device__ __forceinline__ int64_t segment_sum(int64_t v) {
#pragma unroll
    for (int off = SEG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, SEG);
    return v;
}

template <int SEG>
__device__ __forceinline__ int32_t segment_sum32(int32_t v) {
#pragma unroll
    for (int off = SEG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, SEG);
    return v;
}

// Pixel level, boundary term (Prop. 2): W_x weighs label x over the 5x5
// window around p by how many in-image 3x3 patches centred on p's 3x3
// neighbours contain the cell; per axis that is
// |([p-1, p+1] clipped to the image) n [q-1, q+1]| for cell coordinate q.
__device__ __forceinline__ int axis_weight(int p, int q, int n) {
    const int lo = max(max(p - 1, 0), q - 1), hi = min(min(p + 1, n - 1), q + 1);
    return (q >= 0 && q < n) ? max(hi - lo + 1, 0) : 0;
}


// Pixel level, first test: is the pixel at the centre of window w (5x5
// labels with row stride kWinW, -1 outside the image) a boundary pixel whose
// label stays connected without it? Only the 3x3 neighbourhood is read.
__device__ __forceinline__ bool pixel_movable(const int32_t *w) {
    const int32_t *c = w + 2 * kWinW + 2;
    return neighbourhood9(c[0], c[-kWinW], c[-kWinW + 1], c[1], c[kWinW + 1], c[kWinW],
                          c[kWinW - 1], c[-1], c[-kWinW - 1])
        .movable;
}

// Pixel level decision for pixel (x, y) with colour bin j, from the 5x5
// window w of labels around it (row stride kWinW, -1 outside the image; the
// boundary term reads all of it, the rest only the 3x3 ring) and the
// histograms hist: best 4-neighbour label n of the gain
//   g = (h_n(j) - h_k(j) + 1) + gamma (W_n + |K_p| - W_k)
// (colour part: Prop. 1 with one look-up per side; boundary part: Prop. 2),
// ties to the smaller label, taken only if g > 0.
struct PixelMove {
    int n;  // target label, -1 for no move
    int k;  // current label
};

// Boundary term of the gain (Prop. 2) for the first Q candidates:
// g[q] += gamma (W_n + |K_p| - W_k). INTERIOR: p lies at least 2 cells from
// every image border, so every axis weight is 3 - |offset| and |K_p| = 9.
template <int Q, bool INTERIOR>
__device__ __forceinline__ void boundary_term(const Dims &d, const int32_t *w,
                                              const Neighbourhood &nb, int x, int y,
                                              int (&g)[4]) {
    int wk = 0, wn[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) wn[q] = 0;
    // row by row: per row, the sums of the column weights of the cells
    // holding k and each candidate, then weighted by the row's weight
    int wx[5];
#pragma unroll
    for (int dx = -2; dx <= 2; ++dx)
        wx[dx + 2] = INTERIOR ? 3 - (dx < 0 ? -dx : dx) : axis_weight(x, x + dx, d.W);
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy) {
        const int wy = INTERIOR ? 3 - (dy < 0 ? -dy : dy) : axis_weight(y, y + dy, d.H);
        int rk = 0, rn[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) rn[q] = 0;
#pragma unroll
        for (int dx = -2; dx <= 2; ++dx) {
            const int l = w[(dy + 2) * kWinW + dx + 2];
            rk += l == nb.k ? wx[dx + 2] : 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) rn[q] += l == nb.cand[q] ? wx[dx + 2] : 0;
        }
        wk += wy * rk;
#pragma unroll
        for (int q = 0; q < Q; ++q) wn[q] += wy * rn[q];
    }
    const int kp = INTERIOR ? 9
                            : (min(x + 1, d.W - 1) - max(x - 1, 0) + 1) *
                                  (min(y + 1, d.H - 1) - max(y - 1, 0) + 1);
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (q < nb.nc) g[q] += d.gamma * (wn[q] + kp - wk);
}

// CONST_W: take the constant-weight form of the boundary term when every
// deciding pixel of the wavefront is an interior one (the compacting pixel
// phase has no registers to spare for a second form and keeps the general one).
template <bool CONST_W = true>
__device__ __forceinline__ PixelMove pixel_decision(const Dims &d, const int32_t *w, int j,
                                                    const int32_t *__restrict__ hist, int x,
                                                    int y) {
    PixelMove mv;
    mv.n = -1;
    const int32_t *c = w + 2 * kWinW + 2;
    const Neighbourhood nb = neighbourhood9(c[0], c[-kWinW], c[-kWinW + 1], c[1], c[kWinW + 1],
                                            c[kWinW], c[kWinW - 1], c[-1], c[-kWinW - 1]);
    mv.k = nb.k;
    if (!nb.movable) return mv;
    const int k = nb.k;
    const int hk = hist[(int64_t)k * d.hs + j];
    int g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        g[q] = q < nb.nc ? hist[(int64_t)nb.cand[q] * d.hs + j] - hk + 1 : INT32_MIN / 2;
    if (d.gamma) {
        // when every deciding pixel of the wavefront is an interior one the
        // weights are constants (about a fifth of the term's instructions)
        const bool interior = x >= 2 && x + 2 < d.W && y >= 2 && y + 2 < d.H;
        if (CONST_W && __all(interior))
            boundary_term<4, true>(d, w, nb, x, y, g);
        else
            boundary_term<4, false>(d, w, nb, x, y, g);
    }
    // candidates are ascending, so a strict ">" keeps the smaller label on ties
    int bg = g[0], bn = nb.cand[0];
#pragma unroll
    for (int q = 1; q < 4; ++q)
        if (q < nb.nc && g[q] > bg) {
            bg = g[q];
            bn = nb.cand[q];
        }
    mv.n = bg > 0 ? bn : -1;
    return mv;
}

}  // namespace seeds
