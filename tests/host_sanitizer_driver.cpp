// Host-side sanitizer driver: the library's host code (argument checks,
// arena and map layout, schedules, graph caching, snapshots, the server's
// admission and tick logic) compiled with AddressSanitizer and
// UndefinedBehaviorSanitizer, device code unchanged, linked into this program
// (no preloading). It calls every entry point of the C ABI on small images and
// checks that paths which must agree do agree: a batch of one and a single
// context, a resumed snapshot and an uninterrupted run, the server, the
// allocation-free call and a context, and the graph and step launch modes. Any memory
// error or undefined behaviour in host code ends the run with a report; a disagreement
// exits with status 1. Prints "host sanitizer runs: ok" at the end.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "seeds.h"

namespace {

int g_failures = 0;

#define CHECK(cond)                                                                       \
    do {                                                                                  \
        if (!(cond)) {                                                                    \
            std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond,    \
                         seeds_last_error());                                             \
            ++g_failures;                                                                 \
        }                                                                                 \
    } while (0)

#define HIP_OK(x)                                                                         \
    do {                                                                                  \
        if ((x) != hipSuccess) {                                                          \
            std::fprintf(stderr, "HIP call failed at line %d: %s\n", __LINE__, #x);       \
            std::exit(2);                                                                 \
        }                                                                                 \
    } while (0)

// A pseudo-random image of smooth regions (a small linear congruential
// generator, so the program needs nothing but itself).
std::vector<uint8_t> make_image(int H, int W, uint32_t seed) {
    uint32_t s = seed * 2654435761u + 1u;
    auto next = [&]() {
        s = s * 1664525u + 1013904223u;
        return s >> 8;
    };
    const int nc = 6;
    int cx[nc], cy[nc], col[nc][3];
    for (int i = 0; i < nc; ++i) {
        cx[i] = (int)(next() % (uint32_t)W);
        cy[i] = (int)(next() % (uint32_t)H);
        for (int c = 0; c < 3; ++c) col[i][c] = (int)(next() % 256u);
    }
    std::vector<uint8_t> img((size_t)H * W * 3);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int best = 0;
            long bd = -1;
            for (int i = 0; i < nc; ++i) {
                const long d = (long)(x - cx[i]) * (x - cx[i]) + (long)(y - cy[i]) * (y - cy[i]);
                if (bd < 0 || d < bd) bd = d, best = i;
            }
            for (int c = 0; c < 3; ++c) {
                const int v = col[best][c] + (int)(next() % 17u) - 8;
                img[((size_t)y * W + x) * 3 + c] = (uint8_t)(v < 0 ? 0 : v > 255 ? 255 : v);
            }
        }
    return img;
}

struct DevImage {
    uint8_t *d = nullptr;
    int H, W;
    DevImage(int h, int w, uint32_t seed) : H(h), W(w) {
        const std::vector<uint8_t> img = make_image(h, w, seed);
        HIP_OK(hipMalloc(&d, img.size()));
        HIP_OK(hipMemcpy(d, img.data(), img.size(), hipMemcpyHostToDevice));
    }
    ~DevImage() { (void)hipFree(d); }
    DevImage(const DevImage &) = delete;
    DevImage &operator=(const DevImage &) = delete;
};

seeds_params params(int L, int B, int I, int gamma, int rule) {
    seeds_params p;
    CHECK(seeds_default_params(&p) == SEEDS_OK);
    p.levels = L;
    p.bins_per_channel = B;
    p.iters_per_level = I;
    p.gamma = gamma;
    p.block_rule = rule;
    return p;
}

std::vector<int32_t> labels_of(seeds_ctx *ctx, int H, int W) {
    std::vector<int32_t> lab((size_t)H * W, -7);
    CHECK(seeds_labels(ctx, lab.data(), 1, nullptr) == SEEDS_OK);
    return lab;
}

// One image end to end in a launch mode, with every query along the way.
std::vector<int32_t> single(const DevImage &im, int K, const seeds_params &p, int mode) {
    seeds_ctx *ctx = nullptr;
    CHECK(seeds_init(&ctx, im.d, im.H, im.W, 3 * im.W, K, &p, nullptr) == SEEDS_OK);
    if (!ctx) return {};
    CHECK(seeds_set_launch_mode(ctx, mode) == SEEDS_OK);
    int32_t done = 0;
    CHECK(seeds_refine_phases(ctx, 5, &done, nullptr) == SEEDS_OK);
    CHECK(seeds_refine(ctx, nullptr) == SEEDS_OK);
    CHECK(seeds_level(ctx) == 0);
    const int keff = seeds_num_superpixels(ctx);
    CHECK(keff > 0);
    const int nb = p.bins_per_channel * p.bins_per_channel * p.bins_per_channel;
    std::vector<int32_t> hist((size_t)keff * nb), size(keff);
    CHECK(seeds_histograms(ctx, hist.data(), size.data(), 1, nullptr) == SEEDS_OK);
    int64_t total = 0;
    for (int k = 0; k < keff; ++k) total += size[k];
    CHECK(total == (int64_t)im.H * im.W);
    int64_t h = 0, g = 0, units = 0, pixels = 0;
    CHECK(seeds_energy(ctx, &h, &g, nullptr) == SEEDS_OK);
    CHECK(seeds_boundary_units(ctx, 0, -1, &units, &pixels, nullptr) == SEEDS_OK);
    std::vector<int32_t> lab = labels_of(ctx, im.H, im.W);
    // labels into device memory as well, then compared
    int32_t *d_lab = nullptr;
    HIP_OK(hipMalloc(&d_lab, lab.size() * 4));
    CHECK(seeds_labels(ctx, d_lab, 0, nullptr) == SEEDS_OK);
    CHECK(seeds_sync(ctx, nullptr) == SEEDS_OK);
    std::vector<int32_t> lab2(lab.size());
    HIP_OK(hipMemcpy(lab2.data(), d_lab, lab.size() * 4, hipMemcpyDeviceToHost));
    HIP_OK(hipFree(d_lab));
    CHECK(lab == lab2);
    // a second refine (further pixel sweeps) and a re-initialisation
    CHECK(seeds_refine(ctx, nullptr) == SEEDS_OK);
    CHECK(seeds_reinit(ctx, im.d, 3 * im.W, nullptr) == SEEDS_OK);
    CHECK(seeds_refine(ctx, nullptr) == SEEDS_OK);
    CHECK(labels_of(ctx, im.H, im.W) == lab);
    CHECK(seeds_destroy(ctx) == SEEDS_OK);
    return lab;
}

void test_singles_and_modes() {
    const int shapes[][4] = {{97, 131, 40, 3}, {33, 47, 6, 2}, {1, 1, 1, 1}, {5, 200, 9, 2},
                             {120, 90, 25, 4}};
    uint32_t seed = 1;
    for (const auto &s : shapes)
        for (int rule = 0; rule < 2; ++rule) {
            DevImage im(s[0], s[1], seed++);
            const seeds_params p = params(s[3], 4, 2, 1, rule);
            // (the persistent mode's cooperative launches need a device-wide
            // resource that another process using the GPU, such as a test
            // runner that started this program, may hold; the in-process tests
            // cover that mode)
            const std::vector<int32_t> ref = single(im, s[2], p, SEEDS_LAUNCH_GRAPH);
            CHECK(single(im, s[2], p, SEEDS_LAUNCH_STEPS) == ref);
        }
}

void test_tuning_and_snapshots() {
    DevImage im(150, 170, 11);
    const seeds_params p = params(4, 5, 2, 1, 1);
    const std::vector<int32_t> ref = single(im, 60, p, SEEDS_LAUNCH_GRAPH);
    seeds_ctx *ctx = nullptr;
    CHECK(seeds_init(&ctx, im.d, im.H, im.W, 3 * im.W, 60, &p, nullptr) == SEEDS_OK);
    if (!ctx) return;
    const seeds_tuning settings[] = {{0, 1, 1, 16, 16, 1}, {1, 0, 2, 8, 32, 4}, {0, 0, 4, 32, 8, 4}};
    for (const auto &t : settings) {
        CHECK(seeds_set_tuning(ctx, &t) == SEEDS_OK);
        seeds_tuning back;
        CHECK(seeds_get_tuning(ctx, &back) == SEEDS_OK);
        CHECK(std::memcmp(&back, &t, sizeof t) == 0);
        CHECK(seeds_reinit(ctx, im.d, 3 * im.W, nullptr) == SEEDS_OK);
        // stop part way, snapshot, resume in a fresh context, finish
        int32_t done = 0;
        CHECK(seeds_refine_phases(ctx, 23, &done, nullptr) == SEEDS_OK);
        int64_t bytes = 0;
        CHECK(seeds_snapshot_size(ctx, &bytes) == SEEDS_OK);
        std::vector<uint8_t> snap((size_t)bytes);
        CHECK(seeds_snapshot(ctx, snap.data(), bytes, nullptr) == SEEDS_OK);
        CHECK(seeds_snapshot(ctx, snap.data(), bytes - 1, nullptr) == SEEDS_E_INVAL);
        seeds_ctx *other = nullptr;
        CHECK(seeds_init(&other, im.d, im.H, im.W, 3 * im.W, 60, &p, nullptr) == SEEDS_OK);
        if (other) {
            CHECK(seeds_restore(other, snap.data(), bytes - 8, nullptr) == SEEDS_E_INVAL);
            CHECK(seeds_restore(other, snap.data(), bytes, nullptr) == SEEDS_OK);
            CHECK(seeds_refine(other, nullptr) == SEEDS_OK);
            CHECK(labels_of(other, im.H, im.W) == ref);
            CHECK(seeds_destroy(other) == SEEDS_OK);
        }
        CHECK(seeds_refine(ctx, nullptr) == SEEDS_OK);
        CHECK(labels_of(ctx, im.H, im.W) == ref);
    }
    seeds_tuning chosen;
    std::vector<float> ms(SEEDS_TUNE_VARIANTS);
    CHECK(seeds_autotune(ctx, 1, &chosen, ms.data(), nullptr) == SEEDS_OK);
    CHECK(seeds_refine(ctx, nullptr) == SEEDS_OK);
    CHECK(labels_of(ctx, im.H, im.W) == ref);
    // the warm start on the same image: refine again from the kept labels
    CHECK(seeds_warm_start(ctx, im.d, 3 * im.W, nullptr) == SEEDS_OK);
    CHECK(seeds_refine(ctx, nullptr) == SEEDS_OK);
    const seeds_tuning bad = {0, 1, 3, 16, 16, 1};
    CHECK(seeds_set_tuning(ctx, &bad) == SEEDS_E_INVAL);
    CHECK(seeds_destroy(ctx) == SEEDS_OK);
}

void test_batches() {
    const int specs[][4] = {{97, 131, 40, 3}, {60, 80, 12, 4}, {33, 47, 6, 1}, {150, 170, 60, 4}};
    const int n = 4;
    std::vector<DevImage *> ims;
    for (int i = 0; i < n; ++i) ims.push_back(new DevImage(specs[i][0], specs[i][1], 40 + i));
    for (int rule = 0; rule < 2; ++rule) {
        const seeds_params p = params(4, 5, 2, 1, rule);
        std::vector<seeds_image> desc(n);
        for (int i = 0; i < n; ++i)
            desc[i] = {ims[i]->d, ims[i]->H, ims[i]->W, 3 * (int64_t)ims[i]->W, specs[i][2],
                       specs[i][3]};
        seeds_ctx *ctx = nullptr;
        CHECK(seeds_batch_init(&ctx, desc.data(), n, &p, nullptr) == SEEDS_OK);
        if (!ctx) continue;
        CHECK(seeds_batch_count(ctx) == n);
        for (int ppl : {1, 4}) {
            const seeds_tuning t = {0, 1, 1, 16, 16, ppl};
            CHECK(seeds_set_tuning(ctx, &t) == SEEDS_OK);
            std::vector<const uint8_t *> rgb(n);
            std::vector<int64_t> pitch(n);
            for (int i = 0; i < n; ++i) rgb[i] = ims[i]->d, pitch[i] = 3 * (int64_t)ims[i]->W;
            CHECK(seeds_batch_reinit(ctx, rgb.data(), pitch.data(), nullptr) == SEEDS_OK);
            CHECK(seeds_refine(ctx, nullptr) == SEEDS_OK);
            for (int i = 0; i < n; ++i) {
                seeds_params pi = p;
                pi.levels = specs[i][3];
                const std::vector<int32_t> ref = single(*ims[i], specs[i][2], pi, SEEDS_LAUNCH_GRAPH);
                std::vector<int32_t> lab((size_t)ims[i]->H * ims[i]->W);
                CHECK(seeds_batch_labels(ctx, i, lab.data(), 1, nullptr) == SEEDS_OK);
                CHECK(lab == ref);
                const int keff = seeds_batch_num_superpixels(ctx, i);
                std::vector<int32_t> hist((size_t)keff * 125), size(keff);
                CHECK(seeds_batch_histograms(ctx, i, hist.data(), size.data(), 1, nullptr) == SEEDS_OK);
                int64_t h = 0, g = 0;
                CHECK(seeds_batch_energy(ctx, i, &h, &g, nullptr) == SEEDS_OK);
            }
            CHECK(seeds_batch_warm_start(ctx, rgb.data(), pitch.data(), nullptr) == SEEDS_OK);
            CHECK(seeds_refine(ctx, nullptr) == SEEDS_OK);
        }
        std::vector<int32_t> lab(16);
        CHECK(seeds_batch_labels(ctx, n, lab.data(), 1, nullptr) == SEEDS_E_INVAL);
        CHECK(seeds_destroy(ctx) == SEEDS_OK);
    }
    for (auto *im : ims) delete im;
}

void test_server_and_noalloc() {
    const seeds_params p = params(3, 5, 2, 1, 0);
    const int specs[][3] = {{97, 131, 40}, {60, 80, 12}, {150, 170, 60}, {33, 47, 6}, {97, 131, 40}};
    const int n = 5;
    std::vector<DevImage *> ims;
    for (int i = 0; i < n; ++i) ims.push_back(new DevImage(specs[i][0], specs[i][1], 70 + i));
    seeds_server_params sp;
    CHECK(seeds_server_default_params(&sp) == SEEDS_OK);
    sp.bins_per_channel = 5;
    sp.iters_per_level = 2;
    sp.gamma = 1;
    sp.max_levels = 3;
    sp.hbm_budget_bytes = (int64_t)64 << 20;
    sp.max_inflight = 3;
    seeds_server *sv = nullptr;
    CHECK(seeds_server_create(&sv, &sp, nullptr) == SEEDS_OK);
    std::vector<std::vector<int32_t>> out(n);
    if (sv) {
        std::vector<int64_t> ids(n, -1);
        for (int i = 0; i < n; ++i) {
            out[i].assign((size_t)ims[i]->H * ims[i]->W, -7);
            CHECK(seeds_server_submit(sv, ims[i]->d, ims[i]->H, ims[i]->W, 3 * ims[i]->W,
                                      specs[i][2], 3, out[i].data(), 1, &ids[i]) == SEEDS_OK);
            CHECK(i == 0 || ids[i] > ids[i - 1]);  // distinct, in submission order
        }
        int32_t pending = 1;
        int64_t done_ids[8];
        int32_t n_done = 0;
        std::vector<int> reported(n, 0);
        auto note = [&]() {
            for (int e = 0; e < n_done; ++e)
                for (int i = 0; i < n; ++i) reported[i] += done_ids[e] == ids[i];
        };
        for (int tick = 0; pending > 0 && tick < 100000; ++tick) {
            CHECK(seeds_server_step(sv, &pending) == SEEDS_OK);
            CHECK(seeds_server_poll(sv, done_ids, 8, &n_done) == SEEDS_OK);
            note();
        }
        for (int round = 0; round < 100; ++round) {  // reports still in flight
            CHECK(seeds_server_poll(sv, done_ids, 8, &n_done) == SEEDS_OK);
            note();
            int all = 1;
            for (int i = 0; i < n; ++i) all &= reported[i] == 1;
            if (all) break;
            CHECK(hipDeviceSynchronize() == hipSuccess);
        }
        for (int i = 0; i < n; ++i) CHECK(reported[i] == 1);  // each exactly once
        seeds_server_stats st;
        CHECK(seeds_server_get_stats(sv, &st) == SEEDS_OK);
        CHECK(st.completed == n);
        CHECK(seeds_server_destroy(sv) == SEEDS_OK);
    }
    for (int i = 0; i < n; ++i) {
        const std::vector<int32_t> ref = single(*ims[i], specs[i][2], p, SEEDS_LAUNCH_GRAPH);
        CHECK(out[i] == ref);
        // the allocation-free call, twice
        int32_t *d_lab = nullptr;
        HIP_OK(hipMalloc(&d_lab, ref.size() * 4));
        for (int rep = 0; rep < 2; ++rep) {
            CHECK(seeds_segment_noalloc(ims[i]->d, ims[i]->H, ims[i]->W, 3 * ims[i]->W,
                                        specs[i][2], &p, d_lab, nullptr) == SEEDS_OK);
            std::vector<int32_t> lab(ref.size());
            HIP_OK(hipDeviceSynchronize());
            HIP_OK(hipMemcpy(lab.data(), d_lab, ref.size() * 4, hipMemcpyDeviceToHost));
            CHECK(lab == ref);
        }
        // quality metrics of the labels against themselves: no error, no leak
        int32_t *d_truth = nullptr;
        HIP_OK(hipMalloc(&d_truth, ref.size() * 4));
        HIP_OK(hipMemcpy(d_truth, ref.data(), ref.size() * 4, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d_lab, ref.data(), ref.size() * 4, hipMemcpyHostToDevice));
        int32_t maxl = 0;
        for (int32_t v : ref) maxl = v > maxl ? v : maxl;
        seeds_quality q;
        CHECK(seeds_quality_metrics(d_lab, d_truth, ims[i]->H, ims[i]->W, maxl + 1, maxl + 1, 2,
                                    &q, nullptr) == SEEDS_OK);
        CHECK(q.pixels == (int64_t)ref.size() && q.ue == 0);
        HIP_OK(hipFree(d_truth));
        HIP_OK(hipFree(d_lab));
    }
    for (auto *im : ims) delete im;
}

void test_error_paths() {
    DevImage im(40, 50, 99);
    const seeds_params p = params(3, 5, 2, 1, 0);
    seeds_ctx *ctx = nullptr;
    CHECK(seeds_init(nullptr, im.d, 40, 50, 150, 10, &p, nullptr) == SEEDS_E_INVAL);
    CHECK(seeds_init(&ctx, im.d, 40, 50, 149, 10, &p, nullptr) == SEEDS_E_INVAL);
    CHECK(seeds_init(&ctx, im.d, 0, 50, 150, 10, &p, nullptr) == SEEDS_E_INVAL);
    seeds_params badp = p;
    badp.levels = 9;
    CHECK(seeds_init(&ctx, im.d, 40, 50, 150, 10, &badp, nullptr) == SEEDS_E_INVAL);
    CHECK(std::strlen(seeds_last_error()) > 0);
    CHECK(seeds_refine(nullptr, nullptr) != SEEDS_OK);
    CHECK(seeds_destroy(nullptr) == SEEDS_OK);
    int32_t gx = 0, gy = 0;
    CHECK(seeds_grid(40, 50, 10, 3, &gx, &gy) == SEEDS_OK && gx * gy > 0);
    // allocation failure at creation, then a launch failure that poisons
    CHECK(seeds_debug_inject_fault(SEEDS_FAULT_ALLOC, 0) == SEEDS_OK);
    CHECK(seeds_init(&ctx, im.d, 40, 50, 150, 10, &p, nullptr) == SEEDS_E_NOMEM);
    CHECK(seeds_debug_inject_fault(SEEDS_FAULT_ALLOC, -1) == SEEDS_OK);
    CHECK(seeds_init(&ctx, im.d, 40, 50, 150, 10, &p, nullptr) == SEEDS_OK);
    if (ctx) {
        CHECK(seeds_debug_inject_fault(SEEDS_FAULT_LAUNCH, 3) == SEEDS_OK);
        CHECK(seeds_refine(ctx, nullptr) == SEEDS_E_DEVICE);
        CHECK(seeds_debug_inject_fault(SEEDS_FAULT_LAUNCH, -1) == SEEDS_OK);
        CHECK(seeds_refine(ctx, nullptr) == SEEDS_E_STATE);
        CHECK(seeds_destroy(ctx) == SEEDS_OK);
    }
    seeds_server_params sp;
    CHECK(seeds_server_default_params(&sp) == SEEDS_OK);
    sp.items_per_group = 3;
    seeds_server *sv = nullptr;
    CHECK(seeds_server_create(&sv, &sp, nullptr) == SEEDS_E_INVAL);
}

}  // namespace

int main() {
    int dev = 0;
    if (hipGetDeviceCount(&dev) != hipSuccess || dev < 1) {
        std::fprintf(stderr, "no GPU\n");
        return 2;
    }
    std::printf("step: singles and launch modes\n");
    std::fflush(stdout);
    test_singles_and_modes();
    std::printf("step: tuning and snapshots\n");
    std::fflush(stdout);
    test_tuning_and_snapshots();
    std::printf("step: batches\n");
    std::fflush(stdout);
    test_batches();
    std::printf("step: server, allocation-free call, quality\n");
    std::fflush(stdout);
    test_server_and_noalloc();
    std::printf("step: error paths\n");
    std::fflush(stdout);
    test_error_paths();
    if (g_failures) {
        std::printf("host sanitizer runs: %d checks failed\n", g_failures);
        return 1;
    }
    std::printf("host sanitizer runs: ok\n");
    return 0;
}
