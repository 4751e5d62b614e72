// Decoder of the segment encoding: the intensity at each requested frame
// from a pixel's segment list (first spike, last spike, N intervals) as
// spk_segments writes it, without the stream.  This is the encoder/decoder
// split of the paper's hardware design (Sec. III-C): the segmentation pass
// emits one record per segment, and a second pass expands the records to
// frames.  One lane per pixel; the requested frames are taken in time order,
// 32 at a time, and every store of a frame plane is coalesced across the
// wave.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>
#include <cmath>
#include <type_traits>

#include "spk.h"
#include "spk_internal.h"

namespace spk {
namespace {

constexpr int kDecFrames = 32;  // output frames per tile
constexpr int kWin = 8;         // records a lane holds (per-pixel lists)

// One wave per 64 pixels (lane = pixel).  Segment s of a pixel covers the
// requested frames (in time order) from index B(s-1) up to B(s), where
// B(s) = number of requested times <= its last spike (the last stored
// segment of a complete list covers every later frame).  B comes from the
// cumulative count table, or, when the requested times are evenly spaced
// (AP: t0, t0 + dt, ...), from one division, so that a cursor advance needs
// no gather that depends on the record it reads.  The record of the next
// segment is prefetched.
//
// Per tile of 32 frames a lane visits only the segment boundaries inside
// the tile: it writes the value of each piece to its own column of an LDS
// table and sets bit (B - j0) of a mask.  The frames are then expanded with
// one bit extract and one add each (the piece index is the number of mask
// bits at or below the frame) and stored plane by plane, 256 contiguous
// bytes per plane.  A cursor advance -- its loads and its division -- is
// paid once per boundary instead of in every frame the wave visits.
//
// PACKED: the lists are [HW][cap][3] (a pixel's records one after another,
// seg_first pointing at them).  A lane keeps a window of kWin of its records
// in registers and refills it in one burst (kWin consecutive 12-byte
// loads) when the window runs out, so each line of its list is read within
// one refill instead of once per record, about ten tiles apart, by which
// time the line has often left the L2.  The refill is issued at the end of
// the advance that empties the window and the next advance selects from it,
// so the loads have the tile's work to arrive in; the record is selected by
// index rather than shifted down the window, since a register copy would
// wait for the loads in flight.
template <bool IDENT, bool AP, bool PACKED>
__global__ __launch_bounds__(64) void decode_kernel(const int32_t *seg_first,
                                                    const int32_t *seg_last,
                                                    const int32_t *seg_n, const int32_t *count,
                                                    int32_t cap, int64_t HW, int32_t T,
                                                    double theta, const int32_t *cnt_le,
                                                    int32_t t0, int32_t dt,
                                                    const int32_t *plane, int32_t n_out,
                                                    float *out)
{
    // piece k of the current tile for lane l at vals[k][l]: at most one
    // piece per frame
    __shared__ float vals[kDecFrames][64];
    const int lane = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * 64;
    const bool valid = p0 + lane < HW;
    const int32_t S = valid ? count[p0 + lane] : 0;
    const int32_t stored = S < cap ? S : cap;
    // current segment s: value I, first frame index past it B; the record
    // of segment s + 1 prefetched in nf, nl, nn
    int32_t s = -1, nf = 0, nl = 0, nn = 0;
    float I = 0.0f;      // S == 0: fewer than two spikes, every output is 0
    int32_t B = INT_MAX;
    // PACKED: records wbase .. wbase + kWin - 1 (those stored)
    int32_t wb[PACKED ? kWin : 1][3];
    int32_t wbase = 0;
    auto refill = [&](int32_t k) {
        if constexpr (PACKED) {
            const int32_t *r = seg_first + ((p0 + lane) * cap + k) * 3;
#pragma unroll
            for (int j = 0; j < kWin; j++)
                if (k + j < stored) {
                    wb[j][0] = r[3 * j];
                    wb[j][1] = r[3 * j + 1];
                    wb[j][2] = r[3 * j + 2];
                }
            wbase = k;
        }
    };
    auto fetch = [&](int32_t k) {
        if constexpr (PACKED) {
            if (k - wbase >= kWin) refill(k);  // selected at the next advance
        } else {
            const int64_t o = (int64_t)k * HW + p0 + lane;
            nf = seg_first[o];
            nl = seg_last[o];
            nn = seg_n[o];
        }
    };
    auto advance = [&]() {
        s++;
        if (s < stored) {
            if constexpr (PACKED) {
                const int j = s - wbase;
#pragma unroll
                for (int q = 0; q < kWin; q++)
                    if (q == j) {
                        nf = wb[q][0];
                        nl = wb[q][1];
                        nn = wb[q][2];
                    }
            }
            // Eq. 6 as in the reconstruction pass
            I = (float)(theta * (double)nn / (double)((int64_t)nl - nf));
            // requested times <= the segment's last spike: from the
            // cumulative count table, or by one division for t0, t0 + dt, ...
            // (the last segment of the list takes every later time)
            int32_t le;
            if constexpr (AP) {
                const uint32_t q = ((uint32_t)nl - (uint32_t)t0) / (uint32_t)dt + 1u;
                le = nl < t0 ? 0 : (q < (uint32_t)n_out ? (int32_t)q : n_out);
            } else {
                const int32_t c = cnt_le[min(max(nl, 0), T - 1)];
                le = nl < 0 ? 0 : (nl >= T ? n_out : c);
            }
            B = s + 1 >= S ? INT_MAX : le;
            if (s + 1 < stored) fetch(s + 1);
        } else {
            // not stored (the list was cut at cap): unknown from here on
            I = __builtin_nanf("");
            B = INT_MAX;
        }
    };
    if (S > 0) {
        if constexpr (PACKED) {
            if (stored > 0) refill(0);
        } else {
            if (stored > 0) fetch(0);
        }
        advance();
    }
    const uint32_t ulane = (uint32_t)lane;
    for (int32_t j0 = 0; j0 < n_out; j0 += kDecFrames) {
        const int32_t j1 = min(n_out, j0 + kDecFrames);
        // the segment in progress at the tile's first frame
        while (B <= j0) advance();
        uint32_t mask = 0;
        int k = 0;
        vals[0][lane] = I;
        while (B < j1) {
            const int32_t b = B;   // j0 < b < j0 + 32
            mask |= 1u << (b - j0);
            do advance();
            while (B <= b);        // segments that hold no requested frame
            vals[++k][lane] = I;
        }
        // each lane reads back only its own column
        float v[kDecFrames];
        int idx = 0;
#pragma unroll
        for (int jj = 0; jj < kDecFrames; jj++) {
            idx += (mask >> jj) & 1u;
            v[jj] = vals[idx][lane];
        }
        auto put = [&](auto full) {
            float *row = out + (int64_t)j0 * HW + p0;  // plane j0 (in time order)
#pragma unroll
            for (int jj = 0; jj < kDecFrames; jj++) {
                if (decltype(full)::value || j0 + jj < j1) {
                    if constexpr (!IDENT) row = out + (int64_t)plane[j0 + jj] * HW + p0;
                    // streamed past the caches: the frames are not read
                    // back, and the segment records keep the L2
                    __builtin_nontemporal_store(v[jj], &row[ulane]);
                    if constexpr (IDENT) row += HW;
                }
            }
        };
        if (valid) {
            if (j1 - j0 == kDecFrames)
                put(std::true_type{});
            else
                put(std::false_type{});
        }
    }
}

}  // namespace
}  // namespace spk

namespace {

int decode(const int32_t *seg_first, const int32_t *seg_last, const int32_t *seg_n,
           const int32_t *count, int32_t cap, int32_t H, int32_t W, int32_t T, float theta,
           const int32_t *t_out, int32_t n_out, float *out, bool packed, hipStream_t st)
{
    if (H <= 0 || W <= 0 || T <= 0 || cap < 0 || n_out < 0 || !count) return SPK_EINVAL;
    if (cap > 0 && (!seg_first || (!packed && (!seg_last || !seg_n)))) return SPK_EINVAL;
    if (!std::isfinite(theta) || !(theta > 0.0f)) return SPK_EINVAL;
    const int64_t HW = (int64_t)H * W;
    if (HW > (int64_t)INT32_MAX - 128 || (int64_t)n_out * HW > ((int64_t)1 << 60) ||
        (int64_t)cap * HW > ((int64_t)1 << 60))
        return SPK_EINVAL;
    if (n_out == 0) return SPK_OK;
    if (!t_out || !out) return SPK_EINVAL;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0 || t_out[k] >= T) return SPK_EINVAL;
    spk::OutTables tab;
    const int rc = spk::out_tables(T, t_out, n_out, st, &tab);
    if (rc) return rc;
    // evenly spaced requested times (ascending or descending, no repeats):
    // the count of times <= x is one division
    int32_t t0 = 0, dt = 1;
    bool ap = n_out == 1;
    if (n_out >= 2) {
        const int32_t d = t_out[1] - t_out[0];
        ap = d != 0;
        for (int32_t k = 2; ap && k < n_out; k++) ap = t_out[k] - t_out[k - 1] == d;
        if (ap) {
            dt = d > 0 ? d : -d;
            t0 = d > 0 ? t_out[0] : t_out[n_out - 1];
        }
    } else {
        t0 = t_out[0];
    }
    const dim3 grid((unsigned)((HW + 63) / 64)), block(64);
#define SPK_DECODE_LAUNCH(I, A, K)                                                          \
    hipLaunchKernelGGL((spk::decode_kernel<I, A, K>), grid, block, 0, st, seg_first, seg_last, \
                       seg_n, count, cap, HW, T, (double)theta, tab.cnt_le, t0, dt, tab.plane,  \
                       n_out, out)
#define SPK_DECODE_LAYOUT(I, A)          \
    if (packed)                          \
        SPK_DECODE_LAUNCH(I, A, true);   \
    else                                 \
        SPK_DECODE_LAUNCH(I, A, false)
    if (tab.identity && ap) {
        SPK_DECODE_LAYOUT(true, true);
    } else if (tab.identity) {
        SPK_DECODE_LAYOUT(true, false);
    } else if (ap) {
        SPK_DECODE_LAYOUT(false, true);
    } else {
        SPK_DECODE_LAYOUT(false, false);
    }
#undef SPK_DECODE_LAYOUT
#undef SPK_DECODE_LAUNCH
    return hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
}

}  // namespace

extern "C" int spk_decode(const int32_t *seg_first, const int32_t *seg_last, const int32_t *seg_n,
                          const int32_t *count, int32_t cap, int32_t H, int32_t W, int32_t T,
                          float theta, const int32_t *t_out, int32_t n_out, float *out,
                          void *hip_stream)
{
    return decode(seg_first, seg_last, seg_n, count, cap, H, W, T, theta, t_out, n_out, out,
                  false, (hipStream_t)hip_stream);
}

extern "C" int spk_decode_packed(const int32_t *rec, const int32_t *count, int32_t cap, int32_t H,
                                 int32_t W, int32_t T, float theta, const int32_t *t_out,
                                 int32_t n_out, float *out, void *hip_stream)
{
    return decode(rec, nullptr, nullptr, count, cap, H, W, T, theta, t_out, n_out, out, true,
                  (hipStream_t)hip_stream);
}
