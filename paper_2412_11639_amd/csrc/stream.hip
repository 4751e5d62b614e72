// Carry-state reconstruction of a live stream: frames arrive in pieces
// (the paper's hardware processes the camera's frames in 32-frame blocks as
// they arrive, Sec. III-C), and each pixel's running state -- last spike,
// the open segment and its FSR/SSR/third-order state, the first output
// waiting for it -- is kept in device memory between pieces.  Feeding a
// stream in any pieces and finishing gives exactly spk_reconstruct's
// output on the whole stream.
//
// Each piece is one launch: one wave per 64-pixel strip loads its pixels'
// state records, walks the piece's frames with the same per-strip walk as
// the single-pass kernel (transpose, word shortcuts, spike loop, closes),
// writes the outputs of every segment that closes, and stores the state
// back.  Row r of a piece is frame fed + r; the piece's "outputs at or
// before frame" table is built by a small kernel from the sorted output
// times.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "recon_core.h"
#include "spk.h"

namespace spk {
namespace {

// cnt[i] = number of sorted output times <= f0 + i, for i < n
__global__ __launch_bounds__(256) void cnt_range_kernel(const int32_t *t_sorted, int32_t n_out,
                                                        int32_t f0, int32_t n, int32_t *cnt)
{
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t t = f0 + i;
    int32_t lo = 0, hi = n_out;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (t_sorted[mid] <= t) lo = mid + 1;
        else hi = mid;
    }
    cnt[i] = lo;
}

template <int ORDER, bool WIN, int PMAP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
void feed_kernel(ReconParams P, int nblocks, int32_t f0, int32_t *state, int fresh)
{
    __shared__ uint64_t word_s[kGroup][64];
    __shared__ int32_t cnt_s[kGroup][64];
    const int lane = threadIdx.x;
    const int64_t p0 = (int64_t)xcd_strip(blockIdx.x, nblocks) * 64;
    const int64_t p = p0 + lane;
    Emitter<MODE_RECON, WIN, PMAP> em{P, nullptr, p, p < P.HW, 0, 0};
    Run run;
    if (fresh || !em.valid) run.reset(0, 0);
    else load_run<ORDER>(state + p, P.HW, run);
    int32_t cum_base = 0;
    const Xpose X(lane);
    walk<ORDER, false>(P, em, run, P.stream + (p0 >> 3), X, lane, 0, 0, (P.T + 63) / 64, word_s,
                       cnt_s, nullptr, 0, cum_base, f0);
    if (em.valid) save_run<ORDER>(state + p, P.HW, run);
}

template <int ORDER, bool WIN, int PMAP>
__global__ __launch_bounds__(256) void finish_kernel(ReconParams P, const int32_t *state,
                                                     int fresh)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P.HW) return;
    Emitter<MODE_RECON, WIN, PMAP> em{P, nullptr, p, true, 0, 0};
    Run run;
    if (fresh) run.reset(0, 0);
    else load_run<ORDER>(state + p, P.HW, run);
    if (run.cum >= 2)
        em.close(run.first, run.lastspk, (run.cum - 1) - run.first_idx, run.k0, P.n_out);
    else
        em.empty();
}

template <int ORDER, bool WIN, int PMAP>
hipError_t launch_piece(const ReconParams &P, int32_t f0, int32_t *state, bool fresh,
                        bool finish, hipStream_t st)
{
    if (finish) {
        hipLaunchKernelGGL((finish_kernel<ORDER, WIN, PMAP>),
                           dim3((unsigned)((P.HW + 255) / 256)), dim3(256), 0, st, P, state,
                           (int)fresh);
    } else {
        const int nblocks = (P.HW + 63) / 64;
        hipLaunchKernelGGL((feed_kernel<ORDER, WIN, PMAP>), dim3((unsigned)nblocks), dim3(64), 0,
                           st, P, nblocks, f0, state, (int)fresh);
    }
    return hipGetLastError();
}

template <int ORDER>
hipError_t launch_order(const ReconParams &P, bool win, int32_t f0, int32_t *state, bool fresh,
                        bool finish, hipStream_t st)
{
    if (win)
        return P.plane ? launch_piece<ORDER, true, PMAP_GLOBAL>(P, f0, state, fresh, finish, st)
                       : launch_piece<ORDER, true, PMAP_IDENT>(P, f0, state, fresh, finish, st);
    return P.plane ? launch_piece<ORDER, false, PMAP_GLOBAL>(P, f0, state, fresh, finish, st)
                   : launch_piece<ORDER, false, PMAP_IDENT>(P, f0, state, fresh, finish, st);
}

}  // namespace
}  // namespace spk

struct spk_stream_s {
    int dev = -1;
    int32_t H = 0, W = 0, HW = 0, order = SPK_FSR, n_out = 0;
    double theta = 1.0;
    int32_t fed = 0;              // frames fed so far
    bool finished = false;
    bool identity = true;
    float *out = nullptr;
    int32_t *wf = nullptr, *wl = nullptr, *wn = nullptr;
    int32_t *state = nullptr;     // [fields][HW] per-pixel run records
    int32_t *tab = nullptr;       // [n_out] plane map, [n_out] sorted times
    int32_t *cnt = nullptr;       // outputs at or before each frame of a piece
    int32_t cnt_cap = 0;
};

namespace {

bool stream_order_ok(int32_t order)
{
    return order == SPK_FSR || order == SPK_SSR || order == SPK_TFI || order == SPK_TSR;
}

void stream_free(spk_stream_s *s)
{
    if (!s) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (s->dev >= 0) hipSetDevice(s->dev);
    if (s->state) hipFree(s->state);
    if (s->tab) hipFree(s->tab);
    if (s->cnt) hipFree(s->cnt);
    if (have) hipSetDevice(cur);
    delete s;
}

spk::ReconParams stream_params(const spk_stream_s *s)
{
    spk::ReconParams P{};
    P.HW = s->HW;
    P.theta = s->theta;
    P.plane = s->identity ? nullptr : s->tab;
    P.n_out = s->n_out;
    P.out = s->out;
    P.win_first = s->wf;
    P.win_last = s->wl;
    P.win_n = s->wn;
    return P;
}

hipError_t stream_launch(const spk_stream_s *s, const spk::ReconParams &P, bool fresh,
                         bool finish, hipStream_t st)
{
    const bool win = s->wf || s->wl || s->wn || !s->out;
    switch (s->order) {
    case SPK_FSR: return spk::launch_order<1>(P, win, s->fed, s->state, fresh, finish, st);
    case SPK_SSR: return spk::launch_order<2>(P, win, s->fed, s->state, fresh, finish, st);
    case SPK_TFI: return spk::launch_order<3>(P, win, s->fed, s->state, fresh, finish, st);
    default: return spk::launch_order<4>(P, win, s->fed, s->state, fresh, finish, st);
    }
}

}  // namespace

extern "C" {

int spk_stream_create(spk_stream_t *stream, int32_t H, int32_t W, float theta, int32_t order,
                      const int32_t *t_out, int32_t n_out, float *out, int32_t *win_first,
                      int32_t *win_last, int32_t *win_n)
{
    if (!stream) return SPK_EINVAL;
    *stream = nullptr;
    if (H <= 0 || W <= 0 || (int64_t)H * W > (int64_t)INT32_MAX - 128) return SPK_EINVAL;
    if (!std::isfinite(theta) || !(theta > 0.0f) || !stream_order_ok(order)) return SPK_EINVAL;
    if (n_out < 0 || (n_out > 0 && !t_out)) return SPK_EINVAL;
    if ((int64_t)n_out * H * W > ((int64_t)1 << 60)) return SPK_EINVAL;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0) return SPK_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPK_EHIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return SPK_EHIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SPK_EUNSUPPORTED;
    auto *s = new (std::nothrow) spk_stream_s;
    if (!s) return SPK_ENOMEM;
    s->dev = dev;
    s->H = H;
    s->W = W;
    s->HW = H * W;
    s->order = order;
    s->n_out = n_out;
    s->theta = (double)theta;
    s->out = out;
    s->wf = win_first;
    s->wl = win_last;
    s->wn = win_n;
    // sorted output times (stable) and their planes
    std::vector<int32_t> ord(n_out), tab(2 * (size_t)n_out + 1);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int32_t a, int32_t b) { return t_out[a] < t_out[b]; });
    for (int32_t j = 0; j < n_out; j++) {
        tab[j] = ord[j];
        tab[n_out + j] = t_out[ord[j]];
        if (ord[j] != j || (j > 0 && t_out[ord[j]] == t_out[ord[j - 1]])) s->identity = false;
    }
    const size_t state_ints = (size_t)spk::rec_fields_of(order) * (size_t)s->HW;
    s->cnt_cap = 4096;
    if (hipMalloc((void **)&s->state, state_ints * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&s->tab, tab.size() * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&s->cnt, (size_t)s->cnt_cap * sizeof(int32_t)) != hipSuccess) {
        stream_free(s);
        return SPK_ENOMEM;
    }
    if (hipMemcpy(s->tab, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
        hipSuccess) {
        stream_free(s);
        return SPK_EHIP;
    }
    *stream = s;
    return SPK_OK;
}

int spk_stream_feed(spk_stream_t s, const uint8_t *frames, int32_t nframes, void *hip_stream)
{
    if (!s || s->finished || nframes < 0 || (nframes > 0 && !frames)) return SPK_EINVAL;
    if ((uintptr_t)frames & 15u) return SPK_EINVAL;
    if ((int64_t)s->fed + nframes > (int64_t)INT32_MAX - 64) return SPK_EINVAL;
    if (nframes == 0) return SPK_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPK_EHIP;
    if (dev != s->dev) return SPK_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    if (nframes > s->cnt_cap) {
        // a longer piece than any before: the old table may still be read
        if (hipDeviceSynchronize() != hipSuccess) return SPK_EHIP;
        hipFree(s->cnt);
        s->cnt = nullptr;
        const int32_t cap = std::max(nframes, 2 * s->cnt_cap);
        if (hipMalloc((void **)&s->cnt, (size_t)cap * sizeof(int32_t)) != hipSuccess) {
            s->cnt_cap = 0;
            return SPK_ENOMEM;
        }
        s->cnt_cap = cap;
    }
    hipLaunchKernelGGL(spk::cnt_range_kernel, dim3((unsigned)((nframes + 255) / 256)), dim3(256),
                       0, st, s->tab + s->n_out, s->n_out, s->fed, nframes, s->cnt);
    if (hipGetLastError() != hipSuccess) return SPK_EHIP;
    spk::ReconParams P = stream_params(s);
    P.stream = frames;
    P.fb = (int64_t)spk_frame_bytes(s->H, s->W);
    P.T = nframes;
    P.cnt_le = s->cnt;
    if (stream_launch(s, P, s->fed == 0, false, st) != hipSuccess) return SPK_EHIP;
    s->fed += nframes;
    return SPK_OK;
}

int spk_stream_finish(spk_stream_t s, void *hip_stream)
{
    if (!s || s->finished) return SPK_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPK_EHIP;
    if (dev != s->dev) return SPK_EINVAL;
    s->finished = true;
    if (s->n_out == 0 || (!s->out && !s->wf && !s->wl && !s->wn)) return SPK_OK;
    const spk::ReconParams P = stream_params(s);
    return stream_launch(s, P, s->fed == 0, true, (hipStream_t)hip_stream) == hipSuccess
               ? SPK_OK
               : SPK_EHIP;
}

int spk_stream_frames(spk_stream_t s) { return s ? s->fed : SPK_EINVAL; }

int spk_stream_destroy(spk_stream_t s)
{
    if (!s) return SPK_OK;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && s->dev >= 0) {
        hipSetDevice(s->dev);
        hipDeviceSynchronize();
        hipSetDevice(cur);
    }
    stream_free(s);
    return SPK_OK;
}

}  // extern "C"
