// C-ABI entry points of the spike reconstruction library (declared in
// include/spk.h): argument checks, the per-device table of sorted output
// times, and kernel launches on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "recon_core.h"
#include "spk.h"
#include "spk_internal.h"

namespace {

// Device tables derived from one t_out list: cnt_le[t] = number of output
// times <= t (t in [0, T)), the sorted-index -> plane map and the sorted
// times.  Kept in a small per-device cache
// so repeated calls with the same output times upload nothing; a slot is
// only overwritten after the device has drained (hipDeviceSynchronize), so
// a kernel still reading it on another stream is never disturbed.  The
// upload is queued on the stream of the call that filled the slot; `ready`
// is recorded after it, and a call on any other stream that finds the slot
// makes its stream wait for that event before its kernels read the tables.
struct TableSlot {
    int dev = -1;
    int32_t T = 0;
    std::vector<int32_t> key;  // the t_out list as given
    int32_t *d_buf = nullptr;  // [T] cnt_le, [n_out] plane map, [n_out] sorted times
    int32_t *h_buf = nullptr;  // pinned staging of the same
    size_t cap = 0;            // ints allocated in both buffers
    bool identity = true;
    uint64_t stamp = 0;
    hipEvent_t ready = nullptr;     // recorded after the upload (on slot.dev)
    int ev_dev = -1;                // device the event belongs to
    hipStream_t owner = nullptr;    // stream the upload was queued on
};

constexpr int kSlots = 8;
std::mutex g_mu;
TableSlot g_slots[kSlots];
uint64_t g_clock = 0;
int g_dev_ok[64];  // 0 unknown, 1 gfx950, -1 unsupported

int check_device(int *dev_out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPK_EHIP;
    if (dev < 0 || dev >= 64) return SPK_EUNSUPPORTED;
    if (g_dev_ok[dev] == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return SPK_EHIP;
        g_dev_ok[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    }
    if (g_dev_ok[dev] < 0) return SPK_EUNSUPPORTED;
    *dev_out = dev;
    return SPK_OK;
}

// Returns the slot holding the tables of (T, t_out) on device dev, uploading
// them on the caller's stream if needed.
int get_tables(int dev, int32_t T, const int32_t *t_out, int32_t n_out, hipStream_t stream,
               TableSlot **out)
{
    for (auto &s : g_slots) {
        if (s.dev == dev && s.T == T && (int32_t)s.key.size() == n_out &&
            std::equal(s.key.begin(), s.key.end(), t_out)) {
            // the upload may still be queued on another stream: order this
            // stream's kernels after it
            if (stream != s.owner && hipStreamWaitEvent(stream, s.ready, 0) != hipSuccess)
                return SPK_EHIP;
            s.stamp = ++g_clock;
            *out = &s;
            return SPK_OK;
        }
    }
    TableSlot *victim = &g_slots[0];
    for (auto &s : g_slots)
        if (s.stamp < victim->stamp) victim = &s;
    if (victim->dev >= 0) {
        // the slot may still be read by queued kernels on its device
        int cur = dev;
        if (hipSetDevice(victim->dev) != hipSuccess) return SPK_EHIP;
        hipError_t e = hipDeviceSynchronize();
        if (hipSetDevice(cur) != hipSuccess || e != hipSuccess) return SPK_EHIP;
    }
    const size_t need = (size_t)T + 2 * (size_t)n_out;
    if (victim->cap < need || victim->dev != dev) {
        if (victim->d_buf) {
            int cur = dev;
            hipSetDevice(victim->dev);
            hipFree(victim->d_buf);
            hipHostFree(victim->h_buf);
            hipSetDevice(cur);
        }
        victim->d_buf = nullptr;
        victim->h_buf = nullptr;
        victim->cap = 0;
        victim->dev = -1;
        if (hipMalloc((void **)&victim->d_buf, need * sizeof(int32_t)) != hipSuccess)
            return SPK_ENOMEM;
        if (hipHostMalloc((void **)&victim->h_buf, need * sizeof(int32_t), 0) != hipSuccess) {
            hipFree(victim->d_buf);
            victim->d_buf = nullptr;
            return SPK_ENOMEM;
        }
        victim->cap = need;
    }
    // sort output indices by time (stable: duplicates keep their order)
    std::vector<int32_t> order(n_out);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return t_out[a] < t_out[b]; });
    bool identity = true;
    for (int32_t k = 0; k < n_out; k++) {
        if (order[k] != k) identity = false;
        if (k > 0 && t_out[order[k]] == t_out[order[k - 1]]) identity = false;
    }
    int32_t *cnt = victim->h_buf, *plane = victim->h_buf + T, *tsort = plane + n_out;
    int32_t k = 0;
    for (int32_t t = 0; t < T; t++) {
        while (k < n_out && t_out[order[k]] <= t) k++;
        cnt[t] = k;
    }
    for (int32_t j = 0; j < n_out; j++) {
        plane[j] = order[j];
        tsort[j] = t_out[order[j]];
    }
    if (victim->ready && victim->ev_dev != dev) {
        int cur = dev;
        hipSetDevice(victim->ev_dev);
        hipEventDestroy(victim->ready);
        hipSetDevice(cur);
        victim->ready = nullptr;
        victim->ev_dev = -1;
    }
    if (!victim->ready) {
        if (hipEventCreateWithFlags(&victim->ready, hipEventDisableTiming) != hipSuccess) {
            victim->ready = nullptr;
            return SPK_EHIP;
        }
        victim->ev_dev = dev;
    }
    if (hipMemcpyAsync(victim->d_buf, victim->h_buf, need * sizeof(int32_t),
                       hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipEventRecord(victim->ready, stream) != hipSuccess) {
        victim->dev = -1;  // contents unknown: never matched again
        victim->key.clear();
        return SPK_EHIP;
    }
    victim->owner = stream;
    victim->dev = dev;
    victim->T = T;
    victim->key.assign(t_out, t_out + n_out);
    victim->identity = identity;
    victim->stamp = ++g_clock;
    *out = victim;
    return SPK_OK;
}

// Device scratch for the per-chunk records, one buffer per (device, stream)
// so that calls on different streams never share it.  Grows on demand;
// growing waits for the device so a buffer still in use is never freed.
struct Scratch {
    int dev = -1;
    hipStream_t stream = nullptr;
    int32_t *buf = nullptr;
    size_t ints = 0;
};
std::vector<Scratch> g_scratch;

int get_scratch(int dev, hipStream_t stream, size_t ints, int32_t **out)
{
    *out = nullptr;
    if (ints == 0) return SPK_OK;
    Scratch *s = nullptr;
    for (auto &e : g_scratch)
        if (e.dev == dev && e.stream == stream) s = &e;
    if (!s) {
        g_scratch.push_back(Scratch{dev, stream, nullptr, 0});
        s = &g_scratch.back();
    }
    if (s->ints < ints) {
        if (s->buf) {
            if (hipDeviceSynchronize() != hipSuccess) return SPK_EHIP;
            hipFree(s->buf);
            s->buf = nullptr;
            s->ints = 0;
        }
        if (hipMalloc((void **)&s->buf, ints * sizeof(int32_t)) != hipSuccess) return SPK_ENOMEM;
        s->ints = ints;
    }
    *out = s->buf;
    return SPK_OK;
}

// Chunk count for long streams: 0 = automatic (SPK_CHUNKS in the
// environment, else sized to fill the chip); set by spk_set_option.
int g_chunks = -1;

int requested_chunks()
{
    if (g_chunks < 0) {
        const char *e = std::getenv("SPK_CHUNKS");
        g_chunks = e ? std::max(0, std::atoi(e)) : 0;
    }
    return g_chunks;
}

// Warm-up tiles before each speculative chunk: -1 = automatic (SPK_WARM in
// the environment, else min(4, half a chunk)); set by spk_set_option.
int g_warm = -2;  // -2: not read yet

int requested_warm()
{
    if (g_warm == -2) {
        const char *e = std::getenv("SPK_WARM");
        g_warm = e ? std::max(0, std::atoi(e)) : -1;
    }
    return g_warm;
}

int check_common(const uint8_t *stream, int32_t H, int32_t W, int32_t T, int32_t order)
{
    if (!stream || H <= 0 || W <= 0 || T <= 0) return SPK_EINVAL;
    // frames are read as 8- and 16-byte words
    if ((uintptr_t)stream & 15u) return SPK_EINVAL;
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX - 128) return SPK_EINVAL;
    if (order != SPK_FSR && order != SPK_SSR && order != SPK_TFI && order != SPK_TSR)
        return SPK_EINVAL;
    const size_t fb = spk_frame_bytes(H, W);
    if ((size_t)T > SIZE_MAX / fb) return SPK_EINVAL;
    return SPK_OK;
}

// The static / motion mask written by the reconstruction pass itself.
struct MotionOut {
    uint8_t *mask;
    const int32_t *first_spike;
    int32_t window;
};

int reconstruct_impl(const uint8_t *stream, int32_t H, int32_t W, int32_t T, float theta,
                     const int32_t *t_out, int32_t n_out, float *out, int32_t *wf,
                     int32_t *wl, int32_t *wn, int32_t order, void *hip_stream,
                     const MotionOut *mo = nullptr)
{
    int rc = check_common(stream, H, W, T, order);
    if (rc) return rc;
    if (!std::isfinite(theta) || !(theta > 0.0f) || n_out < 0) return SPK_EINVAL;
    if (n_out == 0) return SPK_OK;
    if (!t_out) return SPK_EINVAL;
    if ((int64_t)n_out * (int64_t)H * (int64_t)W > ((int64_t)1 << 60)) return SPK_EINVAL;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0 || t_out[k] >= T) return SPK_EINVAL;
    if (!out && !wf && !wl && !wn && !mo) return SPK_OK;
    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    TableSlot *slot = nullptr;
    rc = get_tables(dev, T, t_out, n_out, st, &slot);
    if (rc) return rc;
    spk::ReconParams p{};
    p.stream = stream;
    p.fb = (int64_t)spk_frame_bytes(H, W);
    p.T = T;
    p.HW = H * W;
    p.theta = (double)theta;
    p.cnt_le = slot->d_buf;
    p.plane = slot->identity ? nullptr : slot->d_buf + T;
    p.n_out = n_out;
    p.out = out;
    p.win_first = wf;
    p.win_last = wl;
    p.win_n = wn;
    if (mo) {
        p.first_spike = mo->first_spike;
        p.window = mo->window;
        p.mask = mo->mask;
    }
    spk::ChunkPlan cp = spk::plan_chunks(p.HW, T, order, requested_chunks(), requested_warm());
    rc = get_scratch(dev, st, spk::chunk_record_ints(cp, p.HW), &cp.rec);
    if (rc) return rc;
    return spk::launch_recon(p, order, mo ? spk::MODE_MOTION : spk::MODE_RECON, cp, st) ==
                   hipSuccess
               ? SPK_OK
               : SPK_EHIP;
}

}  // namespace

namespace spk {

int g_sur_conv_wg = 0;

int out_tables(int32_t T, const int32_t *t_out, int32_t n_out, hipStream_t stream,
               OutTables *out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    int rc = check_device(&dev);
    if (rc) return rc;
    TableSlot *slot = nullptr;
    rc = get_tables(dev, T, t_out, n_out, stream, &slot);
    if (rc) return rc;
    out->cnt_le = slot->d_buf;
    out->plane = slot->d_buf + T;
    out->t_sorted = slot->d_buf + T + n_out;
    out->identity = slot->identity;
    return SPK_OK;
}

}  // namespace spk

namespace {

// Motion mask (see spk.h): the segment holding t started at a cut less than
// `window` frames back; the reconstruction pass writes it (MODE_MOTION),
// from each pixel's first spike, which tells its first segment.
// Each pixel's first spike frame (-1: none).  One wave per 64-pixel strip
// takes 64 frames at a time (lane j loads frame t0 + j's 8 bytes of the
// strip; the transpose gives each lane its pixel's 64-frame word) until
// every pixel of the strip has spiked or the stream ends.
__global__ __launch_bounds__(64) void first_spike_kernel(const uint8_t *stream, int64_t HW,
                                                         size_t fb, int32_t T, int32_t nstrips,
                                                         int32_t *first)
{
    const int lane = threadIdx.x;
    const int32_t strip = spk::xcd_strip(blockIdx.x, nstrips);
    const int64_t p0 = (int64_t)strip * 64, p = p0 + lane;
    const uint8_t *base = stream + (p0 >> 3);
    const spk::Xpose X(lane);
    int32_t f = -1;
    for (int32_t t0 = 0; t0 < T; t0 += 64) {
        const int32_t fr = t0 + lane;
        uint2 v = make_uint2(0u, 0u);
        if (fr < T) v = *(const uint2 *)(base + (int64_t)fr * fb);
        const uint64_t w = spk::transpose64(v.x, v.y, X, lane);
        if (f < 0 && w) f = t0 + spk::ctz64(w);
        // padding pixels past H*W never spike
        if (__ballot(f < 0 && p < HW) == 0) break;
    }
    if (p < HW) first[p] = f;
}

}  // namespace

// ---- allocation-free reconstruction ---------------------------------------
//
// spk_reconstruct_noalloc takes every device buffer beyond the caller's
// inputs and outputs from `scratch`, a fixed array each GPU holds from
// library load to process exit: the output-time tables first (cnt_le [T],
// plane map [n_out], sorted times [n_out]), then the chunk records of the
// time-chunked walk.  Host code never passes the array's name to a kernel:
// its device address on each GPU comes from hipGetSymbolAddress, taken once
// per device with that device current.  The tables reach the device as
// kernel arguments (no host staging buffer, nothing a capture could replay
// from stale host memory), and cnt_le is built on the device from the
// sorted times.  Every word a kernel reads is written earlier in the same
// call, so nothing needs clearing between calls.

static __device__ __align__(256) int32_t scratch[SPK_NOALLOC_SCRATCH_BYTES / sizeof(int32_t)];

namespace {

constexpr size_t kNoAllocInts = SPK_NOALLOC_SCRATCH_BYTES / sizeof(int32_t);
int32_t *g_scratch_ptr[64];  // device address of `scratch` on each device (NULL: not yet)

int noalloc_scratch(int dev, int32_t **out)
{
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return SPK_EHIP;
        g_scratch_ptr[dev] = (int32_t *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return SPK_OK;
}

// Up to kPutInts table words as a kernel argument (a few KB of kernarg).
constexpr int kPutInts = 960;
struct PutChunk {
    int32_t n;
    int32_t v[kPutInts];
};

__global__ __launch_bounds__(256) void put_kernel(int32_t *dst, PutChunk c)
{
    for (int i = threadIdx.x; i < c.n; i += 256) dst[i] = c.v[i];
}

// cnt_le[t] = number of sorted times <= t, for t < T
__global__ __launch_bounds__(256) void cnt_le_kernel(const int32_t *t_sorted, int32_t n_out,
                                                     int32_t T, int32_t *cnt_le)
{
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= T) return;
    int32_t lo = 0, hi = n_out;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (t_sorted[mid] <= t) lo = mid + 1;
        else hi = mid;
    }
    cnt_le[t] = lo;
}

// Sort keys for the output times (time, then index: a stable order).
constexpr int32_t kNoAllocMaxOut = 1 << 20;
static int64_t g_keys[kNoAllocMaxOut];

hipError_t put_ints(int32_t *dst, const int32_t *src, int32_t n, hipStream_t st)
{
    for (int32_t i = 0; i < n; i += kPutInts) {
        PutChunk c;
        c.n = std::min(kPutInts, n - i);
        std::memcpy(c.v, src + i, (size_t)c.n * sizeof(int32_t));
        hipLaunchKernelGGL(put_kernel, dim3(1), dim3(256), 0, st, dst + i, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t spk_frame_bytes(int32_t H, int32_t W)
{
    if (H <= 0 || W <= 0) return 0;
    return (((size_t)H * (size_t)W + 127) / 128) * 16;
}

const char *spk_strerror(int code)
{
    switch (code) {
    case SPK_OK: return "ok";
    case SPK_EINVAL: return "invalid argument";
    case SPK_ENOMEM: return "out of memory";
    case SPK_EHIP: return "HIP runtime error";
    case SPK_EUNSUPPORTED: return "unsupported device (needs gfx950)";
    case SPK_ERANGE: return "request exceeds the allocation-free entry point's fixed scratch";
    default: return "unknown error";
    }
}

int spk_version(void) { return 100; }

int spk_set_option(int option, int value)
{
    std::lock_guard<std::mutex> lock(g_mu);
    switch (option) {
    case SPK_OPT_TIME_CHUNKS:
        if (value < 0) return SPK_EINVAL;
        g_chunks = value;
        return SPK_OK;
    case SPK_OPT_WARM_TILES:
        if (value < 0) return SPK_EINVAL;
        g_warm = value == 0 ? -1 : value;
        return SPK_OK;
    case SPK_OPT_SUR_CONV_WG:
        if (value < 0) return SPK_EINVAL;
        spk::g_sur_conv_wg = value;
        return SPK_OK;
    case SPK_OPT_PLAN_KGROUP:
    case SPK_OPT_PLAN_WAVES_PER_WG:
    case SPK_OPT_PLAN_WPE:
        return spk::set_plan_option(option, value);
    default:
        return SPK_EINVAL;
    }
}

int spk_get_option(int option)
{
    std::lock_guard<std::mutex> lock(g_mu);
    switch (option) {
    case SPK_OPT_TIME_CHUNKS: return requested_chunks();
    case SPK_OPT_WARM_TILES: return std::max(0, requested_warm());
    case SPK_OPT_SUR_CONV_WG: return spk::g_sur_conv_wg;
    case SPK_OPT_PLAN_KGROUP:
    case SPK_OPT_PLAN_WAVES_PER_WG:
    case SPK_OPT_PLAN_WPE: return spk::get_plan_option(option);
    default: return SPK_EINVAL;
    }
}

int spk_reconstruct(const uint8_t *stream, int32_t H, int32_t W, int32_t T, float theta,
                    const int32_t *t_out, int32_t n_out, float *out, int32_t order,
                    void *hip_stream)
{
    if (n_out > 0 && !out) return SPK_EINVAL;
    return reconstruct_impl(stream, H, W, T, theta, t_out, n_out, out, nullptr, nullptr,
                            nullptr, order, hip_stream);
}

int spk_reconstruct_windows(const uint8_t *stream, int32_t H, int32_t W, int32_t T,
                            float theta, const int32_t *t_out, int32_t n_out, float *out,
                            int32_t *win_first, int32_t *win_last, int32_t *win_n,
                            int32_t order, void *hip_stream)
{
    return reconstruct_impl(stream, H, W, T, theta, t_out, n_out, out, win_first, win_last,
                            win_n, order, hip_stream);
}

int spk_reconstruct_noalloc(const uint8_t *stream, int32_t H, int32_t W, int32_t T, float theta,
                            const int32_t *t_out, int32_t n_out, float *out, int32_t order,
                            void *hip_stream)
{
    int rc = check_common(stream, H, W, T, order);
    if (rc) return rc;
    if (!std::isfinite(theta) || !(theta > 0.0f) || n_out < 0) return SPK_EINVAL;
    if (n_out == 0) return SPK_OK;
    if (!t_out || !out) return SPK_EINVAL;
    if ((int64_t)n_out * (int64_t)H * (int64_t)W > ((int64_t)1 << 60)) return SPK_EINVAL;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0 || t_out[k] >= T) return SPK_EINVAL;
    // the tables must fit in the fixed scratch (records shrink to fit)
    const size_t tab_ints = ((size_t)T + 2 * (size_t)n_out + 63) / 64 * 64;
    if (n_out > kNoAllocMaxOut || tab_ints > kNoAllocInts) return SPK_ERANGE;
    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    rc = check_device(&dev);
    if (rc) return rc;
    int32_t *base = nullptr;
    rc = noalloc_scratch(dev, &base);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    // sorted order of the output times (stable), the plane map and the times
    for (int32_t k = 0; k < n_out; k++) g_keys[k] = ((int64_t)t_out[k] << 32) | k;
    std::sort(g_keys, g_keys + n_out);
    bool identity = true;
    for (int32_t j = 0; j < n_out; j++) {
        if ((int32_t)(g_keys[j] & 0xffffffff) != j) identity = false;
        if (j > 0 && (g_keys[j] >> 32) == (g_keys[j - 1] >> 32)) identity = false;
    }
    int32_t *cnt_le = base, *plane = base + T, *t_sorted = base + T + n_out;
    int32_t buf[kPutInts];
    for (int pass = 0; pass < 2; pass++) {
        if (pass == 0 && identity) continue;  // the plane map is not read
        int32_t *dst = pass == 0 ? plane : t_sorted;
        for (int32_t i = 0; i < n_out; i += kPutInts) {
            const int32_t n = std::min(kPutInts, n_out - i);
            for (int32_t j = 0; j < n; j++)
                buf[j] = pass == 0 ? (int32_t)(g_keys[i + j] & 0xffffffff)
                                   : (int32_t)(g_keys[i + j] >> 32);
            if (put_ints(dst + i, buf, n, st) != hipSuccess) return SPK_EHIP;
        }
    }
    hipLaunchKernelGGL(cnt_le_kernel, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st,
                       t_sorted, n_out, T, cnt_le);
    if (hipGetLastError() != hipSuccess) return SPK_EHIP;
    spk::ReconParams p{};
    p.stream = stream;
    p.fb = (int64_t)spk_frame_bytes(H, W);
    p.T = T;
    p.HW = H * W;
    p.theta = (double)theta;
    p.cnt_le = cnt_le;
    p.plane = identity ? nullptr : plane;
    p.n_out = n_out;
    p.out = out;
    // chunk records in the rest of the scratch: as many chunks as the
    // automatic plan wants, fewer if their records do not fit
    const size_t room = kNoAllocInts - tab_ints;
    spk::ChunkPlan cp = spk::plan_chunks(p.HW, T, order, requested_chunks(), requested_warm());
    for (int c = cp.nchunks; c > 1 && spk::chunk_record_ints(cp, p.HW) > room;)
        cp = spk::plan_chunks(p.HW, T, order, --c, requested_warm());
    if (spk::chunk_record_ints(cp, p.HW) > room) cp = spk::plan_chunks(p.HW, T, order, 1);
    cp.rec = cp.nchunks > 1 ? base + tab_ints : nullptr;
    return spk::launch_recon(p, order, spk::MODE_RECON, cp, st) == hipSuccess ? SPK_OK : SPK_EHIP;
}

int spk_motion(const uint8_t *stream, int32_t H, int32_t W, int32_t T, int32_t order,
               int32_t window, const int32_t *t_out, int32_t n_out, uint8_t *mask,
               void *hip_stream)
{
    int rc = check_common(stream, H, W, T, order);
    if (rc) return rc;
    if (window < 1 || n_out < 0) return SPK_EINVAL;
    if (n_out == 0) return SPK_OK;
    if (!t_out || !mask) return SPK_EINVAL;
    const int64_t HW = (int64_t)H * W;
    if ((int64_t)n_out * HW > ((int64_t)1 << 60)) return SPK_EINVAL;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0 || t_out[k] >= T) return SPK_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    int32_t *first = nullptr;
    if (hipMallocAsync((void **)&first, (size_t)HW * sizeof(int32_t), st) != hipSuccess)
        return SPK_ENOMEM;
    // each pixel's first spike (the start of its first segment), then the
    // reconstruction pass, which writes the mask of each output as it
    // closes the segment holding it
    const int32_t nstrips = (int32_t)((HW + 63) / 64);
    hipLaunchKernelGGL(first_spike_kernel, dim3((unsigned)nstrips), dim3(64), 0, st, stream, HW,
                       spk_frame_bytes(H, W), T, nstrips, first);
    rc = hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
    if (!rc) {
        const MotionOut mo{mask, first, window};
        rc = reconstruct_impl(stream, H, W, T, 1.0f, t_out, n_out, nullptr, nullptr, nullptr,
                              nullptr, order, hip_stream, &mo);
    }
    (void)hipFreeAsync(first, st);
    return rc;
}

}  // extern "C"

namespace {

int segments(const uint8_t *stream, int32_t H, int32_t W, int32_t T, int32_t order, int32_t cap,
             int32_t *seg_first, int32_t *seg_last, int32_t *seg_n, int32_t *seg_rec,
             int32_t *count, hipStream_t st)
{
    int rc = check_common(stream, H, W, T, order);
    if (rc) return rc;
    if (cap < 0 || !count) return SPK_EINVAL;
    if (cap > 0 && !seg_rec && (!seg_first || !seg_last || !seg_n)) return SPK_EINVAL;
    if ((int64_t)cap * (int64_t)H * (int64_t)W > ((int64_t)1 << 60)) return SPK_EINVAL;
    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    rc = check_device(&dev);
    if (rc) return rc;
    spk::ReconParams p{};
    p.stream = stream;
    p.fb = (int64_t)spk_frame_bytes(H, W);
    p.T = T;
    p.HW = H * W;
    p.cap = cap;
    p.seg_first = seg_first;
    p.seg_last = seg_last;
    p.seg_n = seg_n;
    p.seg_rec = seg_rec;
    p.count = count;
    return spk::launch_recon(p, order, spk::MODE_SEGMENTS, spk::ChunkPlan{}, st) == hipSuccess
               ? SPK_OK
               : SPK_EHIP;
}

}  // namespace

extern "C" {

int spk_segments(const uint8_t *stream, int32_t H, int32_t W, int32_t T, int32_t order,
                 int32_t cap, int32_t *seg_first, int32_t *seg_last, int32_t *seg_n,
                 int32_t *count, void *hip_stream)
{
    return segments(stream, H, W, T, order, cap, seg_first, seg_last, seg_n, nullptr, count,
                    (hipStream_t)hip_stream);
}

int spk_segments_packed(const uint8_t *stream, int32_t H, int32_t W, int32_t T, int32_t order,
                        int32_t cap, int32_t *rec, int32_t *count, void *hip_stream)
{
    if (cap > 0 && !rec) return SPK_EINVAL;
    return segments(stream, H, W, T, order, cap, nullptr, nullptr, nullptr, rec, count,
                    (hipStream_t)hip_stream);
}

}  // extern "C"
