/* Driver for the sanitizer build of the CPU oracle (test infrastructure):
 * runs the oracle's entry points over odd sizes, every block rule, one to
 * four levels, partial schedules, warm starts, the sequential variant and the
 * quality metrics on pseudo-random images, so that AddressSanitizer and
 * UndefinedBehaviorSanitizer see every code path. Exit status 0 when every
 * call succeeded; the sanitizers abort on the first error they find. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle_state oracle_state;
oracle_state *oracle_create(const uint8_t *rgb, int H, int W, int64_t pitch, int K, int L, int B,
                            int I, int gamma, int rule);
void oracle_free(oracle_state *st);
int oracle_run(oracle_state *st, int max_phases);
int oracle_warm_start(oracle_state *st, const uint8_t *rgb, int64_t pitch);
void oracle_run_sequential(oracle_state *st);
void oracle_energy(const oracle_state *st, int64_t *Hc, int64_t *Gc);
void oracle_pixel_labels(const oracle_state *st, int32_t *out);
int oracle_invalid_superpixels(const oracle_state *st);
int oracle_num_superpixels(const oracle_state *st);
int oracle_quality(const int32_t *labels, const int32_t *truth, int H, int W, int K, int R,
                   int eps, int64_t *out);

static uint32_t lcg = 12345u;
static uint32_t next(void) { lcg = lcg * 1664525u + 1013904223u; return lcg >> 8; }

/* blocky colours plus noise, pitch wider than 3 W */
static uint8_t *image(int H, int W, int64_t pitch) {
    uint8_t *p = (uint8_t *)malloc((size_t)H * pitch);
    int cell = 3 + (int)(next() % 9);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < 3; ++c) {
                int base = (int)(((x / cell) * 37 + (y / cell) * 91 + c * 53) % 256);
                int v = base + (int)(next() % 41) - 20;
                p[(int64_t)y * pitch + 3 * x + c] = (uint8_t)(v < 0 ? 0 : v > 255 ? 255 : v);
            }
    return p;
}

int main(void) {
    int runs = 0;
    for (int t = 0; t < 40; ++t) {
        int H = 5 + (int)(next() % 60), W = 5 + (int)(next() % 60);
        int L = 1 + (int)(next() % 4), B = 1 + (int)(next() % 6), rule = (int)(next() % 2);
        int gamma = (int)(next() % 3), I = 1 + (int)(next() % 3);
        int64_t pitch = 3 * (int64_t)W + (int64_t)(next() % 5);
        int K = 1 + (int)(next() % 40);
        uint8_t *rgb = image(H, W, pitch);
        oracle_state *st = oracle_create(rgb, H, W, pitch, K, L, B, I, gamma, rule);
        if (!st) { free(rgb); continue; }   /* refused parameters are fine */
        oracle_run(st, (int)(next() % 20));
        oracle_run(st, -1);
        uint8_t *rgb2 = image(H, W, pitch);
        if (oracle_warm_start(st, rgb2, pitch) != 0) return 1;
        oracle_run(st, -1);
        int64_t hc, gc;
        oracle_energy(st, &hc, &gc);
        if (oracle_invalid_superpixels(st) != 0) return 2;
        int Keff = oracle_num_superpixels(st);
        int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W);
        int32_t *truth = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W);
        oracle_pixel_labels(st, lab);
        for (int64_t i = 0; i < (int64_t)H * W; ++i) truth[i] = (int32_t)((i % W) * 3 / W);
        int64_t q[6];
        if (oracle_quality(lab, truth, H, W, Keff, 3, 2, q) != 0) return 3;
        oracle_free(st);
        st = oracle_create(rgb, H, W, pitch, K, L, B, I, gamma, rule);
        oracle_run_sequential(st);
        if (oracle_invalid_superpixels(st) != 0) return 4;
        oracle_free(st);
        free(lab); free(truth); free(rgb); free(rgb2);
        ++runs;
    }
    printf("sanitized oracle runs: %d\n", runs);
    return runs > 10 ? 0 : 5;
}
