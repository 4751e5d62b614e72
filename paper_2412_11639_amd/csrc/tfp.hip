// TFP baseline (Sec. II): spikes counted in a fixed window of frames ending
// at each output frame.  One wave per 64-pixel strip and output: lane j
// loads the strip's 8-byte row of frame f0 + j, the 64x64 bit transpose
// turns the rows into per-pixel time words, and popcount counts the window
// 64 frames at a time.
#include <cmath>

#include "spk.h"
#include "recon_core.h"

namespace spk {
namespace {

__global__ __launch_bounds__(64) void tfp_kernel(const uint8_t *stream, int64_t HW, size_t fb,
                                                 int32_t nstrips, double theta, int32_t window,
                                                 const int32_t *t_sorted, const int32_t *plane,
                                                 float *out)
{
    const int lane = threadIdx.x;
    const int32_t strip = xcd_strip(blockIdx.x % nstrips, nstrips);
    const int32_t j = blockIdx.x / nstrips;
    const int32_t t = t_sorted[j];
    const int32_t f0 = max(0, t - window + 1);
    const int64_t p0 = (int64_t)strip * 64;
    const uint8_t *base = stream + (p0 >> 3);
    const Xpose X(lane);
    int32_t cnt = 0;
    for (int32_t f = f0; f <= t; f += 64) {
        const int32_t fr = f + lane;
        uint2 v = make_uint2(0u, 0u);
        if (fr <= t) v = *(const uint2 *)(base + (int64_t)fr * fb);
        cnt += popc64(transpose64(v.x, v.y, X, lane));
    }
    const int64_t p = p0 + lane;
    if (p < HW)
        out[(int64_t)plane[j] * HW + p] = (float)(theta * (double)cnt / (double)(t - f0 + 1));
}

}  // namespace
}  // namespace spk

extern "C" int spk_tfp(const uint8_t *stream, int32_t H, int32_t W, int32_t T, float theta,
                       int32_t window, const int32_t *t_out, int32_t n_out, float *out,
                       void *hip_stream)
{
    if (!stream || H <= 0 || W <= 0 || T <= 0 || window < 1 || n_out < 0) return SPK_EINVAL;
    if ((uintptr_t)stream & 15u) return SPK_EINVAL;  // frames are read as 8-byte words
    if (!std::isfinite(theta) || !(theta > 0.0f)) return SPK_EINVAL;
    if (n_out == 0) return SPK_OK;
    if (!t_out || !out) return SPK_EINVAL;
    const int64_t HW = (int64_t)H * W;
    if (HW > (int64_t)INT32_MAX - 128 || (int64_t)n_out * HW > ((int64_t)1 << 60))
        return SPK_EINVAL;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0 || t_out[k] >= T) return SPK_EINVAL;
    const int32_t nstrips = (int32_t)((HW + 63) / 64);
    if ((int64_t)nstrips * n_out > INT32_MAX) return SPK_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    spk::OutTables tab;
    const int rc = spk::out_tables(T, t_out, n_out, st, &tab);
    if (rc) return rc;
    hipLaunchKernelGGL(spk::tfp_kernel, dim3((unsigned)(nstrips * n_out)), dim3(64), 0, st,
                       stream, HW, spk_frame_bytes(H, W), nstrips, (double)theta, window,
                       tab.t_sorted, tab.plane, out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPK_OK : SPK_EHIP;
}
