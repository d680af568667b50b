// Allocation-free refinement of one image, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, hosts
// that forbid it). Every buffer the path needs beyond the caller's input and
// output lives in one file-scope device array; the kernels and the schedule
// are those of seeds_init / seeds_refine / seeds_labels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "seeds.h"
#include "seeds_internal.h"

namespace seeds {
namespace {

// The whole state of one refinement: bins, pixel labels, both block grids,
// both state copies, drop-rule stamps and decisions, move logs, error flag.
// In host code `scratch` names a host-side stand-in; its device address comes
// from hipGetSymbolAddress, once per device.
static __device__ __align__(256) uint8_t scratch[SEEDS_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
void *g_scratch_dev[kMaxDevices];  // device address of `scratch` per device
std::mutex g_scratch_mu;

// Device address of this device's array, resolved on the first call with
// the device current.
seeds_status scratch_of(int dev, uint8_t **out) {
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(SEEDS_E_DEVICE, "device %d outside [0,%d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return set_error(SEEDS_E_DEVICE, "hipGetSymbolAddress(scratch): %s",
                             hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    *out = (uint8_t *)g_scratch_dev[dev];
    return SEEDS_OK;
}

size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }
size_t up64(size_t v) { return (v + 63) & ~(size_t)63; }

// Offsets of every buffer of one image in the array (the single-image layout
// of a context: image 0 at offset 0 of every arena), and the total.
struct Layout {
    size_t bins, lab, bl, state, src, pend, log, log_n, sync, total;
    int64_t bl_elems, state_elems, src_elems;
    int log_groups, log_cap;
};

Layout layout_of(const Dims &d) {
    Layout o{};
    const size_t N = (size_t)d.H * d.W;
    const size_t blk = d.L > 1 ? (size_t)units_w(d, 1) * units_h(d, 1) : 0;
    o.bl_elems = (int64_t)up64(blk);
    o.state_elems = (int64_t)up64((size_t)d.K * d.hs + d.K);
    o.src_elems = (int64_t)up64(d.K);
    const size_t pend = d.L > 1 ? up64(class_units(d, 1, 0)) : 0;  // class 0 is the largest
    o.log_groups = 1;
    o.log_cap = 1;
    for (int l = 0; l < d.L; ++l) {
        for (int c = 0; c < 9; ++c) o.log_groups = std::max(o.log_groups, phase_groups(d, l, c));
        o.log_cap = std::max(o.log_cap, deltas_per_round(d, l));
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += up256(bytes);
        return at;
    };
    o.bins = take(up64(N));
    o.lab = take(up64(N) * (d.K <= kLab16MaxK ? 2 : 4));
    o.bl = take(2 * (size_t)o.bl_elems * 4);
    o.state = take(2 * (size_t)o.state_elems * 4);
    o.src = take((size_t)o.src_elems * 4);
    o.pend = take(pend * 4);
    o.log = take(2 * (size_t)o.log_groups * o.log_cap * sizeof(int2));
    o.log_n = take(2 * (size_t)o.log_groups * 4);
    o.sync = take(16);
    o.total = off;
    return o;
}

}  // namespace
}  // namespace seeds

using namespace seeds;

extern "C" seeds_status seeds_segment_noalloc(const uint8_t *rgb, int32_t H, int32_t W,
                                              int64_t row_pitch_bytes, int32_t num_superpixels,
                                              const seeds_params *p, int32_t *labels_out,
                                              void *hip_stream) {
    if (!rgb || !labels_out) return set_error(SEEDS_E_INVAL, "rgb or labels_out is NULL");
    Dims d;
    seeds_status st = check_params(H, W, num_superpixels, p, &d);
    if (st != SEEDS_OK) return st;
    if (row_pitch_bytes < 3 * (int64_t)W)
        return set_error(SEEDS_E_INVAL, "row pitch %lld < 3 W", (long long)row_pitch_bytes);
    const Layout o = layout_of(d);
    if (o.total > (size_t)SEEDS_NOALLOC_MAX_BYTES)
        return set_error(SEEDS_E_INVAL,
                         "%d x %d image with %d superpixels and %d levels needs %zu bytes of "
                         "state, more than the %u of the allocation-free path",
                         W, H, d.K, d.L, o.total, (unsigned)SEEDS_NOALLOC_MAX_BYTES);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(SEEDS_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    uint8_t *base = nullptr;
    st = scratch_of(dev, &base);
    if (st != SEEDS_OK) return st;
    hipStream_t s = (hipStream_t)hip_stream;

    ScheduleArgs a;
    a.one.d = d;
    a.one.bins = a.one.lab = a.one.state = a.one.src = a.one.pend = 0;
    a.one.bl[0] = 0;
    a.one.bl[1] = o.bl_elems;
    a.top = d;
    a.src_elems = o.src_elems;
    a.trace = false;  // nothing but kernel launches on this path
    BatchArgs &b = a.b;
    b.imgs = nullptr;  // single-image kernels take the image from `one`
    b.nimg = 1;
    b.ar.bins = base + o.bins;
    const bool lab16 = d.K <= kLab16MaxK;  // as a context would store them
    b.ar.lab = lab16 ? nullptr : (int32_t *)(base + o.lab);
    b.ar.lab16 = lab16 ? (uint16_t *)(base + o.lab) : nullptr;
    b.ar.bl = (int32_t *)(base + o.bl);
    b.ar.state[0] = (int32_t *)(base + o.state);
    b.ar.state[1] = b.ar.state[0] + o.state_elems;
    b.ar.src = (int32_t *)(base + o.src);
    b.ar.pend = (int32_t *)(base + o.pend);
    b.ar.log = (int2 *)(base + o.log);
    b.ar.log_n = (int32_t *)(base + o.log_n);
    b.ar.sync = (uint32_t *)(base + o.sync);
    b.log_cap = o.log_cap;
    b.log_groups = o.log_groups;

    // The array keeps the previous call's contents: the error flag, the
    // drop-rule stamps and both state copies start at zero (fill kernels, no
    // memset nodes under capture).
    e = launch_fill((int32_t *)b.ar.sync, 0, 4, s);
    if (e == hipSuccess) e = launch_fill(b.ar.src, 0, o.src_elems, s);
    if (e == hipSuccess) e = launch_fill(b.ar.state[0], 0, 2 * o.state_elems, s);
    if (e == hipSuccess)
        e = launch_init(b, a.one, rgb, row_pitch_bytes, nullptr, nullptr, nullptr,
                        init_groups(d), kInitTH, s);
    Sched sched;
    sched.level = sched.cur_level = d.L - 1;
    sched.cur_sweep = sched.cur_class = 0;
    if (e == hipSuccess) e = enqueue_schedule(a, sched, -1, nullptr, s);
    if (e == hipSuccess) e = launch_copy_labels(labels_out, b.ar, 0, (int64_t)H * W, s);
    if (e != hipSuccess)
        return set_error(SEEDS_E_DEVICE, "allocation-free refinement: %s", hipGetErrorString(e));
    return SEEDS_OK;
}
