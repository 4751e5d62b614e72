// Decoder of the segment encoding: the intensity at each requested frame
// from a pixel's segment list (first spike, last spike, N intervals) as
// spk_segments writes it, without the stream.  This is the encoder/decoder
// split of the paper's hardware design (Sec. III-C): the segmentation pass
// emits one record per segment, and a second pass expands the records to
// frames.  One lane per pixel walks the requested frames in time order with
// a cursor on its segment list; every store of a frame plane is coalesced
// across the wave.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>
#include <cmath>

#include "spk.h"
#include "spk_internal.h"

namespace spk {
namespace {

constexpr int kDecFrames = 32;  // output frames per LDS tile

// One wave per 64 pixels (lane = pixel).  The requested frames are taken in
// time order, kDecFrames at a time: each lane first advances its cursor
// and writes its values into an LDS tile (its segment loads are prefetched
// one segment ahead, and no global store is pending while it waits for
// them), then the wave stores the tile plane by plane, 256 contiguous
// bytes per plane.
__global__ __launch_bounds__(64) void decode_kernel(const int32_t *seg_first,
                                                    const int32_t *seg_last,
                                                    const int32_t *seg_n, const int32_t *count,
                                                    int32_t cap, int64_t HW, double theta,
                                                    const int32_t *t_sorted,
                                                    const int32_t *plane, int32_t n_out,
                                                    float *out)
{
    __shared__ float tile[kDecFrames][64];
    const int lane = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = p < HW;
    const int32_t S = valid ? count[p] : 0;
    const int32_t stored = S < cap ? S : cap;
    // current segment: index, last spike, value; the next one prefetched
    int32_t s = 0, last = INT_MAX, nf = 0, nl = 0, nn = 0;
    float I = 0.0f;  // S == 0: fewer than two spikes, every output is 0
    auto fetch = [&](int32_t k) {
        const int64_t o = (int64_t)k * HW + p;
        nf = seg_first[o];
        nl = seg_last[o];
        nn = seg_n[o];
    };
    auto take = [&]() {
        if (s < stored) {
            last = nl;
            // Eq. 6 as in the reconstruction pass
            I = (float)(theta * (double)nn / (double)(nl - nf));
        } else {
            // not stored (the list was cut at cap): unknown from here on
            last = INT_MAX;
            I = __builtin_nanf("");
        }
        if (s + 1 < stored) fetch(s + 1);
    };
    if (S > 0) {
        if (stored > 0) fetch(0);
        take();
    }
    for (int32_t j0 = 0; j0 < n_out; j0 += kDecFrames) {
        const int32_t nj = min(kDecFrames, n_out - j0);
        for (int32_t jj = 0; jj < nj; jj++) {
            const int32_t t = t_sorted[j0 + jj];
            // the segment holding the interval in progress at t: advance
            // while the current one ends before t (the last takes later t)
            while (last < t && s + 1 < S) {
                s++;
                take();
            }
            tile[jj][lane] = I;
        }
        for (int32_t jj = 0; jj < nj; jj++)
            if (valid) out[(int64_t)plane[j0 + jj] * HW + p] = tile[jj][lane];
    }
}

}  // namespace
}  // namespace spk

extern "C" int spk_decode(const int32_t *seg_first, const int32_t *seg_last, const int32_t *seg_n,
                          const int32_t *count, int32_t cap, int32_t H, int32_t W, int32_t T,
                          float theta, const int32_t *t_out, int32_t n_out, float *out,
                          void *hip_stream)
{
    if (H <= 0 || W <= 0 || T <= 0 || cap < 0 || n_out < 0 || !count) return SPK_EINVAL;
    if (cap > 0 && (!seg_first || !seg_last || !seg_n)) return SPK_EINVAL;
    if (!std::isfinite(theta) || !(theta > 0.0f)) return SPK_EINVAL;
    const int64_t HW = (int64_t)H * W;
    if (HW > (int64_t)INT32_MAX - 128 || (int64_t)n_out * HW > ((int64_t)1 << 60) ||
        (int64_t)cap * HW > ((int64_t)1 << 60))
        return SPK_EINVAL;
    if (n_out == 0) return SPK_OK;
    if (!t_out || !out) return SPK_EINVAL;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0 || t_out[k] >= T) return SPK_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    spk::OutTables tab;
    const int rc = spk::out_tables(T, t_out, n_out, st, &tab);
    if (rc) return rc;
    hipLaunchKernelGGL(spk::decode_kernel, dim3((unsigned)((HW + 63) / 64)), dim3(64), 0, st,
                       seg_first, seg_last, seg_n, count, cap, HW, (double)theta, tab.t_sorted,
                       tab.plane, n_out, out);
    return hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
}
