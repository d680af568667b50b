/*
 * seeds_oracle.c - plain CPU oracle for the SEEDS hill-climbing refinement
 * (Van den Bergh, Boix, Roig, Van Gool: "SEEDS: Superpixels Extracted via
 * Energy-Driven Sampling").
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The HIP library never
 * calls it and shares no code, header or table with it.
 *
 * What it computes, in the paper's terms:
 *   - bins H_j: every RGB channel is cut into B equal-width intervals
 *     (Sec. 4.1, eq. eqColorHistogram; 5 bins per channel in Sec. 6.2);
 *   - a regular grid of superpixels built from the largest blocks of the
 *     block hierarchy (Sec. 5.1, Fig. "blocks");
 *   - hill climbing (Sec. 5): block-level moves from the largest block size
 *     down to 2x2, then pixel-level moves (Sec. 5.2), each judged by the
 *     colour term H (Prop. 1, Sec. 5.3.1) and, for pixels, the boundary term G
 *     (Prop. 2, Sec. 5.3.2), with the histogram updates of Sec. 5.3.3.
 *
 * Readings taken where the paper is silent (all stated in the design notes):
 *   - moves are proposed for every boundary unit of one colour class
 *     (3x3 lattice classes) per phase instead of one random unit, each moving
 *     to its best 4-neighbour label (ties: smaller label); all decisions of a
 *     phase read the state at the start of the phase;
 *   - under the exact block rule (not Prop. 1), a block move k->n is dropped
 *     when n is itself the source of an accepted block move in the same phase,
 *     so that simultaneous block moves cannot lower H';
 *   - energies are used in count form: H' = sum_k sum_j h_k(j)^2 and
 *     G' = sum_i sum_k b_i(k)^2, with E' = H' + gamma G' at pixel level;
 *   - acceptance is strict (the energy must increase);
 *   - superpixels are 4-connected; a unit may leave label k only if the
 *     k-cells among its four direct neighbours stay connected inside its 3x3
 *     neighbourhood (checked here by a flood fill);
 *   - patches and neighbourhoods are clipped to the image.
 *
 * Everything is integer. Counts are int64; products that compare normalised
 * intersections use __int128 so no bound needs to be argued here.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_RULE_INTERSECT 0
#define ORACLE_RULE_EXACT 1

typedef struct {
    int32_t ux, uy;     /* unit coordinates on the unit grid of the level     */
    int32_t k;          /* label of the unit at the start of the phase        */
    int32_t boundary;   /* 1 if a 4-neighbour unit carries another label      */
    int32_t connect_ok; /* 1 if k stays locally connected without the unit    */
    int32_t n;          /* best neighbour label, -1 if none was evaluated     */
    int32_t accepted;   /* 1 if the energy test for n passed                  */
    int32_t dropped;    /* 1 if the move was discarded by the drop rule       */
    int64_t gain;       /* pixel / EXACT: gain of n; INTERSECT: S_n           */
    int64_t aux;        /* INTERSECT: S of k without the block; else 0        */
    int64_t an;         /* INTERSECT: |A_n|                                   */
    int64_t akl;        /* INTERSECT: |A_k| - |A_k^l|                         */
} oracle_decision;

typedef struct {
    int H, W;
    int B, nbins;
    int L, I, gamma, rule;
    int gx, gy, K;
    uint8_t *bin;       /* H*W: colour bin index of every pixel               */
    int level;          /* current level: L-1 .. 0; 0 = pixels                */
    int side;           /* unit side 2^level                                  */
    int uw, uh;         /* unit grid size: ceil(W/side) x ceil(H/side)         */
    int32_t *label;     /* uh*uw labels of the current unit grid              */
    int64_t *hist;      /* K*nbins: h_k(j) as pixel counts                    */
    int64_t *size;      /* K: |A_k|                                           */
    /* schedule cursor: position of the next phase                           */
    int cur_level, cur_sweep, cur_class;
    int cold;           /* 1 while the first (hierarchical) schedule runs     */
} oracle_state;

/* ------------------------------------------------------------------ */
/* Colour bins (Sec. 4.1): H_j are the cells of a B x B x B partition of
 * the RGB cube; channel value c falls in interval floor(c*B/256).       */
static int channel_bin(int c, int B) { return (c * B) / 256; }

void oracle_quantise(const uint8_t *rgb, int H, int W, int64_t pitch, int B,
                     uint8_t *bins) {
    for (int y = 0; y < H; ++y) {
        const uint8_t *row = rgb + (int64_t)y * pitch;
        for (int x = 0; x < W; ++x) {
            int r = channel_bin(row[3 * x + 0], B);
            int g = channel_bin(row[3 * x + 1], B);
            int b = channel_bin(row[3 * x + 2], B);
            bins[(int64_t)y * W + x] = (uint8_t)((r * B + g) * B + b);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Superpixel grid (Sec. 5.1): gx columns and gy rows of superpixels, chosen
 * so that gx*gy is close to K with near-square cells:
 *   gx = round(sqrt(K*W/H)),  gy = round(K/gx)   (halves round up).
 * Computed with integers only: gx is the largest g >= 1 with
 * (2g-1)^2 * H <= 4*K*W.                                               */
int oracle_grid(int H, int W, int K, int L, int *gx_out, int *gy_out) {
    if (H < 1 || W < 1 || K < 1 || L < 1 || L > 8) return -1;
    int64_t lhs_k = 4 * (int64_t)K * (int64_t)W;
    int gx = 1;
    while ((int64_t)(2 * (gx + 1) - 1) * (2 * (gx + 1) - 1) * (int64_t)H <= lhs_k)
        gx++;
    int gy = (int)((2 * (int64_t)K + gx) / (2 * (int64_t)gx));
    if (gy < 1) gy = 1;
    int T = 1 << (L - 1);
    int bw = (W + T - 1) / T, bh = (H + T - 1) / T;
    if (gx > bw || gy > bh) return -1;
    *gx_out = gx;
    *gy_out = gy;
    return 0;
}

/* ------------------------------------------------------------------ */
static int32_t *lab_at(oracle_state *st, int ux, int uy) {
    return &st->label[(int64_t)uy * st->uw + ux];
}
static int in_grid(const oracle_state *st, int ux, int uy) {
    return ux >= 0 && uy >= 0 && ux < st->uw && uy < st->uh;
}
static int label_or(const oracle_state *st, int ux, int uy, int fallback) {
    if (!in_grid(st, ux, uy)) return fallback;
    return st->label[(int64_t)uy * st->uw + ux];
}
static void set_level(oracle_state *st, int level) {
    st->level = level;
    st->side = 1 << level;
    st->uw = (st->W + st->side - 1) / st->side;
    st->uh = (st->H + st->side - 1) / st->side;
}

/* Label of pixel (x, y) under the current unit grid. */
static int pixel_label(const oracle_state *st, int x, int y) {
    return st->label[(int64_t)(y / st->side) * st->uw + (x / st->side)];
}

/* Recount h_k(j) and |A_k| from scratch (eq. eqColorHistogram, in counts). */
static void recount(oracle_state *st) {
    memset(st->hist, 0, sizeof(int64_t) * (size_t)st->K * st->nbins);
    memset(st->size, 0, sizeof(int64_t) * (size_t)st->K);
    for (int y = 0; y < st->H; ++y)
        for (int x = 0; x < st->W; ++x) {
            int k = pixel_label(st, x, y);
            st->hist[(int64_t)k * st->nbins + st->bin[(int64_t)y * st->W + x]] += 1;
            st->size[k] += 1;
        }
}

void oracle_free(oracle_state *st) {
    if (!st) return;
    free(st->bin);
    free(st->label);
    free(st->hist);
    free(st->size);
    free(st);
}

/* Create the oracle state: bins, the grid of Sec. 5.1 on the largest block
 * size 2^(L-1), and the colour histograms of every superpixel.           */
oracle_state *oracle_create(const uint8_t *rgb, int H, int W, int64_t pitch, int K,
                            int L, int B, int I, int gamma, int rule) {
    int gx, gy;
    if (B < 1 || B > 6 || I < 0 || gamma < 0 || (rule != 0 && rule != 1)) return NULL;
    if ((int64_t)H * W >= ((int64_t)1 << 23)) return NULL;
    if (oracle_grid(H, W, K, L, &gx, &gy) != 0) return NULL;
    if ((1 << (L - 1)) > (H < W ? H : W)) return NULL;
    oracle_state *st = (oracle_state *)calloc(1, sizeof(oracle_state));
    st->H = H; st->W = W; st->B = B; st->nbins = B * B * B;
    st->L = L; st->I = I; st->gamma = gamma; st->rule = rule;
    st->gx = gx; st->gy = gy; st->K = gx * gy;
    st->bin = (uint8_t *)malloc((size_t)H * W);
    oracle_quantise(rgb, H, W, pitch, B, st->bin);
    st->label = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W);
    st->hist = (int64_t *)malloc(sizeof(int64_t) * (size_t)st->K * st->nbins);
    st->size = (int64_t *)malloc(sizeof(int64_t) * (size_t)st->K);
    set_level(st, L - 1);
    /* top block (bx, by) belongs to superpixel row floor(by*gy/bh) and column
     * floor(bx*gx/bw); each superpixel is a rectangle of whole top blocks.  */
    for (int by = 0; by < st->uh; ++by)
        for (int bx = 0; bx < st->uw; ++bx) {
            int sy = (int)((int64_t)by * gy / st->uh);
            int sx = (int)((int64_t)bx * gx / st->uw);
            *lab_at(st, bx, by) = sy * gx + sx;
        }
    recount(st);
    st->cur_level = L - 1; st->cur_sweep = 0; st->cur_class = 0; st->cold = 1;
    return st;
}

/* Replace the partition by arbitrary pixel labels (level 0) and recount.
 * Used by tests to start from hand-made or random partitions.           */
int oracle_set_pixel_labels(oracle_state *st, const int32_t *labels) {
    for (int64_t i = 0; i < (int64_t)st->H * st->W; ++i)
        if (labels[i] < 0 || labels[i] >= st->K) return -1;
    set_level(st, 0);
    memcpy(st->label, labels, sizeof(int32_t) * (size_t)st->H * st->W);
    recount(st);
    st->cur_level = 0; st->cur_sweep = 0; st->cur_class = 0; st->cold = 0;
    return 0;
}

/* Warm start on the next frame of a stream. The paper names video as an
 * input the framework adapts to (Sec. 7) and lets the refinement stop and
 * resume at any time (Sec. 5.4); the reading taken here: keep the pixel
 * labels of the previous frame, bin the new frame (Sec. 4.1), recount the
 * colour histograms and sizes of every superpixel from those labels and bins
 * (eq. eqColorHistogram), and mark the schedule finished, so that the next
 * run does I pixel-level sweeps. Only a state at pixel level can be warm
 * started (returns -1 otherwise).                                       */
int oracle_warm_start(oracle_state *st, const uint8_t *rgb, int64_t pitch) {
    if (st->level != 0) return -1;
    oracle_quantise(rgb, st->H, st->W, pitch, st->B, st->bin);
    recount(st);
    st->cur_level = -1; st->cur_sweep = 0; st->cur_class = 0; st->cold = 0;
    return 0;
}

/* Replace the partition by arbitrary labels on the unit grid of a level
 * (level 0 = pixels) and recount; the schedule then continues from the
 * first phase of that level.                                            */
int oracle_set_unit_labels(oracle_state *st, int level, const int32_t *labels) {
    if (level < 0 || level >= st->L) return -1;
    set_level(st, level);
    for (int64_t i = 0; i < (int64_t)st->uw * st->uh; ++i)
        if (labels[i] < 0 || labels[i] >= st->K) return -1;
    memcpy(st->label, labels, sizeof(int32_t) * (size_t)st->uw * st->uh);
    recount(st);
    st->cur_level = level; st->cur_sweep = 0; st->cur_class = 0; st->cold = level > 0;
    return 0;
}

/* Move from block level l to level l-1: every block is split into its 2x2
 * children, which inherit its label (Sec. 5.1, hierarchy of blocks).      */
static void descend(oracle_state *st) {
    int old_uw = st->uw;
    int32_t *old = (int32_t *)malloc(sizeof(int32_t) * (size_t)st->uw * st->uh);
    memcpy(old, st->label, sizeof(int32_t) * (size_t)st->uw * st->uh);
    set_level(st, st->level - 1);
    for (int uy = 0; uy < st->uh; ++uy)
        for (int ux = 0; ux < st->uw; ++ux)
            *lab_at(st, ux, uy) = old[(int64_t)(uy / 2) * old_uw + ux / 2];
    free(old);
}

/* ------------------------------------------------------------------ */
/* Sec. 3: superpixels are connected blobs; moving a unit out of k must not
 * split k. Local test on the 3x3 neighbourhood: the unit is removed, and
 * every k-cell that touches the unit through an edge must be reachable
 * from the others by 4-steps over k-cells inside the 3x3 window.
 * No edge-touching k-cell at all means the unit is all of k: refused.    */
static int local_connectivity_ok(const oracle_state *st, int ux, int uy, int k) {
    int isk[3][3], seen[3][3];
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            isk[dy + 1][dx + 1] = label_or(st, ux + dx, uy + dy, -1) == k;
            seen[dy + 1][dx + 1] = 0;
        }
    isk[1][1] = 0; /* the unit itself leaves k */
    static const int edge_r[4] = {0, 1, 2, 1}, edge_c[4] = {1, 2, 1, 0};
    int start = -1, need = 0;
    for (int e = 0; e < 4; ++e)
        if (isk[edge_r[e]][edge_c[e]]) {
            need++;
            if (start < 0) start = e;
        }
    if (start < 0) return 0;
    int qr[9], qc[9], head = 0, tail = 0;
    qr[tail] = edge_r[start]; qc[tail] = edge_c[start]; tail++;
    seen[edge_r[start]][edge_c[start]] = 1;
    while (head < tail) {
        int r = qr[head], c = qc[head]; head++;
        static const int dr[4] = {-1, 0, 1, 0}, dc[4] = {0, 1, 0, -1};
        for (int d = 0; d < 4; ++d) {
            int nr = r + dr[d], nc = c + dc[d];
            if (nr < 0 || nr > 2 || nc < 0 || nc > 2) continue;
            if (!isk[nr][nc] || seen[nr][nc]) continue;
            seen[nr][nc] = 1;
            qr[tail] = nr; qc[tail] = nc; tail++;
        }
    }
    int got = 0;
    for (int e = 0; e < 4; ++e)
        if (isk[edge_r[e]][edge_c[e]] && seen[edge_r[e]][edge_c[e]]) got++;
    return got == need;
}

/* Distinct labels other than k among the 4-neighbour units, ascending. */
static int neighbour_candidates(const oracle_state *st, int ux, int uy, int k,
                                int cand[4]) {
    static const int dx[4] = {0, 1, 0, -1}, dy[4] = {-1, 0, 1, 0};
    int nc = 0;
    for (int d = 0; d < 4; ++d) {
        int l = label_or(st, ux + dx[d], uy + dy[d], -1);
        if (l < 0 || l == k) continue;
        int dup = 0;
        for (int i = 0; i < nc; ++i) dup |= cand[i] == l;
        if (!dup) cand[nc++] = l;
    }
    /* insertion sort: ties in the gain are resolved towards smaller labels */
    for (int i = 1; i < nc; ++i)
        for (int j = i; j > 0 && cand[j - 1] > cand[j]; --j) {
            int t = cand[j]; cand[j] = cand[j - 1]; cand[j - 1] = t;
        }
    return nc;
}

/* eq. boundaryterm in counts: b_{N_i}(x) = number of pixels with label x in
 * the 3x3 patch N_i centred on pixel i (clipped to the image). Level 0 only. */
static int64_t patch_count(const oracle_state *st, int ix, int iy, int x) {
    int64_t c = 0;
    for (int qy = iy - 1; qy <= iy + 1; ++qy)
        for (int qx = ix - 1; qx <= ix + 1; ++qx)
            if (in_grid(st, qx, qy) && st->label[(int64_t)qy * st->uw + qx] == x) c++;
    return c;
}

/* Prop. 2: for a pixel p moving from k to n,
 *   sum_{i in K_p} (b_{N_i}(n) + 1) - sum_{i in K_p} b_{N_i}(k)
 * where K_p are the (in-image) pixels whose patch contains p. This equals
 * half the change of G' = sum_i sum_k b_{N_i}(k)^2.                     */
static int64_t boundary_gain(const oracle_state *st, int px, int py, int k, int n) {
    int64_t plus = 0, minus = 0;
    for (int iy = py - 1; iy <= py + 1; ++iy)
        for (int ix = px - 1; ix <= px + 1; ++ix) {
            if (!in_grid(st, ix, iy)) continue;
            plus += patch_count(st, ix, iy, n) + 1;
            minus += patch_count(st, ix, iy, k);
        }
    return plus - minus;
}

/* Prop. 1 for a single pixel of colour bin j (one memory look-up each side,
 * Sec. 5.3.1): in counts the test compares the number of pixels of bin j in
 * A_n with the number in A_k without the pixel, i.e. h_n(j) vs h_k(j) - 1.
 * The difference is half the change of H' = sum_k sum_j h_k(j)^2.       */
static int64_t colour_gain_pixel(const oracle_state *st, int j, int k, int n) {
    return st->hist[(int64_t)n * st->nbins + j] - (st->hist[(int64_t)k * st->nbins + j] - 1);
}

/* Colour histogram of one unit (block), h_l(j), and its pixel count m. */
static int64_t unit_histogram(const oracle_state *st, int ux, int uy, int64_t *hl) {
    int64_t m = 0;
    for (int j = 0; j < st->nbins; ++j) hl[j] = 0;
    int x0 = ux * st->side, y0 = uy * st->side;
    for (int y = y0; y < y0 + st->side && y < st->H; ++y)
        for (int x = x0; x < x0 + st->side && x < st->W; ++x) {
            hl[st->bin[(int64_t)y * st->W + x]] += 1;
            m++;
        }
    return m;
}

/* Histogram intersection of Sec. 5.3.1 between superpixel histogram
 * (counts h, size A) and the block histogram (counts hl, size m), both
 * normalised by their sizes:
 *   int(c_A, c_l) = sum_j min(h(j)/A, hl(j)/m) = S / (A*m),
 *   S = sum_j min(h(j)*m, hl(j)*A).
 * Returns the numerator S; the denominator is A*m.                    */
static int64_t intersection_numerator(const int64_t *h, int64_t A, const int64_t *hl,
                                      int64_t m, int nbins) {
    int64_t S = 0;
    for (int j = 0; j < nbins; ++j) {
        int64_t a = h[j] * m, b = hl[j] * A;
        S += a < b ? a : b;
    }
    return S;
}

/* a/b > c/d for positive denominators */
static int frac_gt(int64_t a, int64_t b, int64_t c, int64_t d) {
    return (__int128)a * d > (__int128)c * b;
}

/* Decide the move of one unit from the current state (no update). */
static void decide_unit(const oracle_state *st, int ux, int uy, oracle_decision *d,
                        int64_t *hl, int64_t *hkl) {
    memset(d, 0, sizeof(*d));
    int k = st->label[(int64_t)uy * st->uw + ux];
    d->ux = ux; d->uy = uy; d->k = k; d->n = -1;
    int cand[4];
    int nc = neighbour_candidates(st, ux, uy, k, cand);
    d->boundary = nc > 0;
    if (!nc) return;
    d->connect_ok = local_connectivity_ok(st, ux, uy, k);
    if (!d->connect_ok) return;

    if (st->level == 0) {
        /* pixel-level move: E' = H' + gamma G', gain = dE'/2 */
        int j = st->bin[(int64_t)uy * st->W + ux];
        int64_t best = 0;
        int bn = -1;
        for (int c = 0; c < nc; ++c) {
            int64_t g = colour_gain_pixel(st, j, k, cand[c]) +
                        (int64_t)st->gamma * boundary_gain(st, ux, uy, k, cand[c]);
            if (bn < 0 || g > best) { best = g; bn = cand[c]; }
        }
        d->n = bn; d->gain = best; d->accepted = best > 0;
        return;
    }

    int64_t m = unit_histogram(st, ux, uy, hl);
    const int64_t *hk = &st->hist[(int64_t)k * st->nbins];
    if (st->rule == ORACLE_RULE_EXACT) {
        /* change of H' when A_k^l moves from k to n, halved:
         * sum_j hl(j) * (h_n(j) - h_k(j) + hl(j))                      */
        int64_t best = 0;
        int bn = -1;
        for (int c = 0; c < nc; ++c) {
            const int64_t *hn = &st->hist[(int64_t)cand[c] * st->nbins];
            int64_t g = 0;
            for (int j = 0; j < st->nbins; ++j) g += hl[j] * (hn[j] - hk[j] + hl[j]);
            if (bn < 0 || g > best) { best = g; bn = cand[c]; }
        }
        d->n = bn; d->gain = best; d->accepted = best > 0;
        return;
    }
    /* Prop. 1: move when int(c_n, c_l) > int(c_{k \ l}, c_l) */
    for (int j = 0; j < st->nbins; ++j) hkl[j] = hk[j] - hl[j];
    int64_t Akl = st->size[k] - m;
    int64_t Skl = intersection_numerator(hkl, Akl, hl, m, st->nbins);
    int64_t bestS = 0, bestA = 1;
    int bn = -1;
    for (int c = 0; c < nc; ++c) {
        int n = cand[c];
        int64_t An = st->size[n];
        int64_t S = intersection_numerator(&st->hist[(int64_t)n * st->nbins], An, hl, m,
                                           st->nbins);
        /* compare S/(An*m) with bestS/(bestA*m) */
        if (bn < 0 || frac_gt(S, An, bestS, bestA)) { bestS = S; bestA = An; bn = n; }
    }
    d->n = bn; d->gain = bestS; d->aux = Skl; d->an = bestA; d->akl = Akl;
    d->accepted = frac_gt(bestS, bestA, Skl, Akl);
}

/* Decide all units of colour class cls (units (ux,uy) with ux%3 = cls%3 and
 * uy%3 = cls/3) at the current level from the current state, without
 * updating anything. Returns the number of class units written to out
 * (at most max_out; pass out = NULL to count only).                    */
int oracle_decide_class(const oracle_state *st, int cls, oracle_decision *out, int max_out) {
#ifdef _OPENMP
    /* All-core build (gcc -fopenmp): the decisions of a phase read only the
     * phase-start state, so the rows of the class lattice are decided in
     * parallel; each decision goes to its raster position among the class
     * units, which gives the same array as the loop below.              */
    const int rows = st->uh > cls / 3 ? (st->uh - cls / 3 + 2) / 3 : 0;
    const int cols = st->uw > cls % 3 ? (st->uw - cls % 3 + 2) / 3 : 0;
#pragma omp parallel
    {
        int64_t *thl = (int64_t *)malloc(sizeof(int64_t) * st->nbins);
        int64_t *thkl = (int64_t *)malloc(sizeof(int64_t) * st->nbins);
#pragma omp for schedule(dynamic, 4)
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) {
                oracle_decision d;
                decide_unit(st, cls % 3 + 3 * c, cls / 3 + 3 * r, &d, thl, thkl);
                const int at = r * cols + c;
                if (out && at < max_out) out[at] = d;
            }
        free(thl);
        free(thkl);
    }
    return rows * cols;
#endif
    int64_t *hl = (int64_t *)malloc(sizeof(int64_t) * st->nbins);
    int64_t *hkl = (int64_t *)malloc(sizeof(int64_t) * st->nbins);
    int cnt = 0;
    for (int uy = cls / 3; uy < st->uh; uy += 3)
        for (int ux = cls % 3; ux < st->uw; ux += 3) {
            oracle_decision d;
            decide_unit(st, ux, uy, &d, hl, hkl);
            if (out && cnt < max_out) out[cnt] = d;
            cnt++;
        }
    free(hl);
    free(hkl);
    return cnt;
}

/* Move unit (ux,uy) from k to n and update the two histograms (Sec. 5.3.3:
 * subtract c_{A_k^l} from c_{A_k}, add it to c_{A_n}).                  */
static void apply_move(oracle_state *st, int ux, int uy, int k, int n) {
    int x0 = ux * st->side, y0 = uy * st->side;
    for (int y = y0; y < y0 + st->side && y < st->H; ++y)
        for (int x = x0; x < x0 + st->side && x < st->W; ++x) {
            int j = st->bin[(int64_t)y * st->W + x];
            st->hist[(int64_t)k * st->nbins + j] -= 1;
            st->hist[(int64_t)n * st->nbins + j] += 1;
            st->size[k] -= 1;
            st->size[n] += 1;
        }
    *lab_at(st, ux, uy) = n;
}

/* One phase: decide every unit of class cls from the phase-start state,
 * apply the drop rule at block levels under the exact rule, then apply the
 * surviving moves. Returns the number of moves applied.                */
int oracle_phase(oracle_state *st, int cls) {
    int cnt = oracle_decide_class(st, cls, NULL, 0);
    oracle_decision *dec = (oracle_decision *)malloc(sizeof(oracle_decision) * (cnt + 1));
    oracle_decide_class(st, cls, dec, cnt);
    if (st->level > 0 && st->rule == ORACLE_RULE_EXACT) {
        char *is_source = (char *)calloc((size_t)st->K, 1);
        for (int i = 0; i < cnt; ++i)
            if (dec[i].accepted) is_source[dec[i].k] = 1;
        for (int i = 0; i < cnt; ++i)
            if (dec[i].accepted && is_source[dec[i].n]) dec[i].dropped = 1;
        free(is_source);
    }
    int moved = 0;
    for (int i = 0; i < cnt; ++i)
        if (dec[i].accepted && !dec[i].dropped) {
            apply_move(st, dec[i].ux, dec[i].uy, dec[i].k, dec[i].n);
            moved++;
        }
    free(dec);
    return moved;
}

/* ------------------------------------------------------------------ */
/* Schedule (Sec. 5.2): levels from the largest block down to pixels; at
 * each level I sweeps; a sweep visits the nine classes in order.
 * The first run after creation walks the whole hierarchy; later runs
 * repeat I sweeps at pixel level only.
 * oracle_run executes at most max_phases phases (negative: no limit) and
 * returns the number executed. When no phase of the schedule is left the
 * state is brought to pixel level.                                       */
int oracle_run(oracle_state *st, int max_phases) {
    int done = 0;
    if (!st->cold && st->cur_level < 0) {
        /* a finished schedule: a new run does I pixel-level sweeps */
        st->cur_level = 0; st->cur_sweep = 0; st->cur_class = 0;
    }
    while (st->cur_level >= 0) {
        if (st->cur_sweep >= st->I) {
            st->cur_level--; st->cur_sweep = 0; st->cur_class = 0;
            continue;
        }
        if (max_phases >= 0 && done >= max_phases) break;
        while (st->level > st->cur_level) descend(st);
        oracle_phase(st, st->cur_class);
        done++;
        if (++st->cur_class == 9) { st->cur_class = 0; st->cur_sweep++; }
    }
    if (st->cur_level < 0) {
        while (st->level > 0) descend(st);
        st->cold = 0;
    }
    return done;
}

/* Class of the next phase of the schedule, with the state brought to that
 * phase's level as oracle_run would before executing it; -1 when no phase
 * of the current schedule is left. Lets a caller inspect the decisions of
 * every phase (oracle_decide_class) before running it (oracle_run(st, 1)). */
int oracle_next_phase(oracle_state *st) {
    while (st->cur_level >= 0 && st->cur_sweep >= st->I) {
        st->cur_level--; st->cur_sweep = 0; st->cur_class = 0;
    }
    if (st->cur_level < 0) return -1;
    while (st->level > st->cur_level) descend(st);
    return st->cur_class;
}

/* Sequential variant: same levels and sweeps, units in raster order, every
 * decision sees all earlier moves, no classes and no drop rule.          */
void oracle_run_sequential(oracle_state *st) {
    int64_t *hl = (int64_t *)malloc(sizeof(int64_t) * st->nbins);
    int64_t *hkl = (int64_t *)malloc(sizeof(int64_t) * st->nbins);
    for (int lev = st->level; lev >= 0; --lev) {
        while (st->level > lev) descend(st);
        for (int t = 0; t < st->I; ++t)
            for (int uy = 0; uy < st->uh; ++uy)
                for (int ux = 0; ux < st->uw; ++ux) {
                    oracle_decision d;
                    decide_unit(st, ux, uy, &d, hl, hkl);
                    if (d.accepted) apply_move(st, ux, uy, d.k, d.n);
                }
    }
    free(hl);
    free(hkl);
    st->cur_level = -1; st->cold = 0;
}

/* ------------------------------------------------------------------ */
/* Accessors */
/* Threads a phase's decisions use: omp_get_max_threads() in the all-core
 * build, 1 otherwise.                                                   */
#ifdef _OPENMP
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
#else
int oracle_threads(void) { return 1; }
#endif

int oracle_num_superpixels(const oracle_state *st) { return st->K; }
int oracle_level(const oracle_state *st) { return st->level; }
void oracle_unit_grid(const oracle_state *st, int *uw, int *uh) { *uw = st->uw; *uh = st->uh; }
void oracle_grid_dims(const oracle_state *st, int *gx, int *gy) { *gx = st->gx; *gy = st->gy; }

void oracle_unit_labels(const oracle_state *st, int32_t *out) {
    memcpy(out, st->label, sizeof(int32_t) * (size_t)st->uw * st->uh);
}
void oracle_pixel_labels(const oracle_state *st, int32_t *out) {
    for (int y = 0; y < st->H; ++y)
        for (int x = 0; x < st->W; ++x) out[(int64_t)y * st->W + x] = pixel_label(st, x, y);
}
void oracle_bins(const oracle_state *st, uint8_t *out) {
    memcpy(out, st->bin, (size_t)st->H * st->W);
}
void oracle_histograms(const oracle_state *st, int64_t *hist, int64_t *size) {
    if (hist) memcpy(hist, st->hist, sizeof(int64_t) * (size_t)st->K * st->nbins);
    if (size) memcpy(size, st->size, sizeof(int64_t) * (size_t)st->K);
}

/* Energies in count form from scratch, on the pixel labels:
 *   H' = sum_k sum_j h_k(j)^2        (eqs. eqColorSum, eqColorMain)
 *   G' = sum_i sum_k b_{N_i}(k)^2    (eq. eqBoundaryMain), 3x3 patches. */
void oracle_energy(const oracle_state *st, int64_t *Hc, int64_t *Gc) {
    int64_t *h = (int64_t *)calloc((size_t)st->K * st->nbins, sizeof(int64_t));
    for (int y = 0; y < st->H; ++y)
        for (int x = 0; x < st->W; ++x)
            h[(int64_t)pixel_label(st, x, y) * st->nbins + st->bin[(int64_t)y * st->W + x]]++;
    int64_t hs = 0;
    for (int64_t i = 0; i < (int64_t)st->K * st->nbins; ++i) hs += h[i] * h[i];
    free(h);
    int64_t gs = 0;
    for (int y = 0; y < st->H; ++y)
        for (int x = 0; x < st->W; ++x) {
            int labs[9], cnts[9], nl = 0;
            for (int qy = y - 1; qy <= y + 1; ++qy)
                for (int qx = x - 1; qx <= x + 1; ++qx) {
                    if (qx < 0 || qy < 0 || qx >= st->W || qy >= st->H) continue;
                    int l = pixel_label(st, qx, qy), f = -1;
                    for (int i = 0; i < nl; ++i)
                        if (labs[i] == l) f = i;
                    if (f < 0) { labs[nl] = l; cnts[nl] = 1; nl++; }
                    else cnts[f]++;
                }
            for (int i = 0; i < nl; ++i) gs += (int64_t)cnts[i] * cnts[i];
        }
    *Hc = hs;
    *Gc = gs;
}

/* Every superpixel non-empty and 4-connected on the pixel grid (Sec. 3).
 * Returns the number of labels that are empty or split (0 = valid).    */
int oracle_invalid_superpixels(const oracle_state *st) {
    int64_t N = (int64_t)st->H * st->W;
    int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * N);
    oracle_pixel_labels(st, lab);
    int *comps = (int *)calloc((size_t)st->K, sizeof(int));
    char *seen = (char *)calloc((size_t)N, 1);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * N);
    for (int64_t s = 0; s < N; ++s) {
        if (seen[s]) continue;
        int l = lab[s];
        comps[l]++;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        seen[s] = 1;
        while (head < tail) {
            int64_t p = queue[head++];
            int px = (int)(p % st->W), py = (int)(p / st->W);
            static const int dx[4] = {0, 1, 0, -1}, dy[4] = {-1, 0, 1, 0};
            for (int d = 0; d < 4; ++d) {
                int qx = px + dx[d], qy = py + dy[d];
                if (qx < 0 || qy < 0 || qx >= st->W || qy >= st->H) continue;
                int64_t q = (int64_t)qy * st->W + qx;
                if (seen[q] || lab[q] != l) continue;
                seen[q] = 1;
                queue[tail++] = q;
            }
        }
    }
    int bad = 0;
    for (int k = 0; k < st->K; ++k) bad += comps[k] != 1;
    free(lab); free(comps); free(seen); free(queue);
    return bad;
}

/* One-shot helper: create, run the whole schedule (or at most max_phases
 * phases), write pixel labels (H*W), histograms (K*B^3) and sizes (K).
 * Returns K, or -1 if the parameters are invalid.                     */
int oracle_seeds(const uint8_t *rgb, int H, int W, int64_t pitch, int K, int L, int B,
                 int I, int gamma, int rule, int max_phases, int32_t *labels,
                 int64_t *hist, int64_t *size) {
    oracle_state *st = oracle_create(rgb, H, W, pitch, K, L, B, I, gamma, rule);
    if (!st) return -1;
    oracle_run(st, max_phases);
    if (labels) oracle_pixel_labels(st, labels);
    oracle_histograms(st, hist, size);
    int k = st->K;
    oracle_free(st);
    return k;
}

/* ------------------------------------------------------------------ */
/* Quality metrics of a segmentation s (labels in [0,K)) against ground
 * truth g (segments in [0,R)), as defined in Sec. 6.1. Returned as integer
 * numerators over N = H*W (UE, CUE, ASA) and over |B(g)| (BR):
 *   out[0] N
 *   out[1] UE numerator   sum_i sum_{k: s_k meets g_i} |s_k - g_i|     (eq. ue)
 *   out[2] ASA numerator  sum_k max_i |s_k & g_i|
 *   out[3] CUE numerator  sum_k |s_k - g_max(s_k)|, g_max the segment of
 *                         largest overlap (ties: the smaller index)
 *   out[4] BR hits        pixels p of B(g) with some q of B(s), |p-q| < eps
 *   out[5] |B(g)|
 * Reading: a pixel lies on the boundary B(.) of a segmentation when one of
 * its in-image 4-neighbours carries another segment; distances are
 * Euclidean between pixel positions. Returns -1 on an out-of-range value. */
static int on_boundary(const int32_t *seg, int H, int W, int x, int y) {
    const int32_t v = seg[(int64_t)y * W + x];
    if (x > 0 && seg[(int64_t)y * W + x - 1] != v) return 1;
    if (x + 1 < W && seg[(int64_t)y * W + x + 1] != v) return 1;
    if (y > 0 && seg[(int64_t)(y - 1) * W + x] != v) return 1;
    if (y + 1 < H && seg[(int64_t)(y + 1) * W + x] != v) return 1;
    return 0;
}

int oracle_quality(const int32_t *labels, const int32_t *truth, int H, int W, int K, int R,
                   int eps, int64_t *out) {
    const int64_t N = (int64_t)H * W;
    for (int64_t p = 0; p < N; ++p)
        if (labels[p] < 0 || labels[p] >= K || truth[p] < 0 || truth[p] >= R) return -1;
    /* overlaps |s_k & g_i| and sizes |s_k| */
    int64_t *ov = (int64_t *)calloc((size_t)K * R, sizeof(int64_t));
    int64_t *sk = (int64_t *)calloc((size_t)K, sizeof(int64_t));
    for (int64_t p = 0; p < N; ++p) {
        ov[(int64_t)labels[p] * R + truth[p]] += 1;
        sk[labels[p]] += 1;
    }
    int64_t ue = 0, asa = 0, cue = 0;
    for (int i = 0; i < R; ++i)
        for (int k = 0; k < K; ++k)
            if (ov[(int64_t)k * R + i] > 0) ue += sk[k] - ov[(int64_t)k * R + i];
    for (int k = 0; k < K; ++k) {
        int best = 0;
        for (int i = 1; i < R; ++i)
            if (ov[(int64_t)k * R + i] > ov[(int64_t)k * R + best]) best = i;
        asa += ov[(int64_t)k * R + best];
        cue += sk[k] - ov[(int64_t)k * R + best];
    }
    /* boundary recall */
    int64_t hits = 0, total = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            if (!on_boundary(truth, H, W, x, y)) continue;
            total++;
            int found = 0;
            for (int dy = -eps; dy <= eps && !found; ++dy)
                for (int dx = -eps; dx <= eps && !found; ++dx) {
                    if (dx * dx + dy * dy >= eps * eps) continue;
                    const int qx = x + dx, qy = y + dy;
                    if (qx < 0 || qy < 0 || qx >= W || qy >= H) continue;
                    found = on_boundary(labels, H, W, qx, qy);
                }
            hits += found;
        }
    out[0] = N; out[1] = ue; out[2] = asa; out[3] = cue; out[4] = hits; out[5] = total;
    free(ov); free(sk);
    return 0;
}
