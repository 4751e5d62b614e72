// Plain FSR / SSR reconstruction for gfx950.
//
// Method (arXiv 2412.11639): a pixel's inter-spike intervals S1 (Def. 2,
// Eq. 4) are cut wherever they leave zero-order stability (values spanning
// more than 1): first order = FSR; SSR also cuts, inside an FSR segment,
// where the S2 stream of an interval value (gaps between its consecutive
// occurrences, Eq. 5) leaves zero-order stability (Sec. III-B).  A segment's
// intensity is theta * N / (sum of its N intervals) (Eq. 6).
//
// Mapping to the hardware.  One wave owns 64 consecutive pixels (one lane
// per pixel) and walks time in tiles of 64 frames:
//   1. lane j loads the 8-byte word of frame t0 + j covering the wave's 64
//      pixels (frame-major input, one coalesced 512-byte request per wave);
//   2. a 6-stage butterfly over the wave transposes the 64x64 bit block so
//      lane i holds pixel i's 64-frame time word (bit j = frame t0 + j);
//   3. each lane walks its spikes with find-first-set and runs the
//      segmentation state machine (registers only), marking in a 64-bit
//      mask the spikes whose interval opens a new segment;
//   4. a second loop walks that mask, recovers each closed segment's
//      window (first/last spike frame, N by popcount) and writes its
//      intensity to every output time the segment covers.
// Workgroups are single waves; block ids are remapped so consecutive pixel
// strips share an XCD (and its L2), since 16 waves read each 128-byte line.
#include "spk_internal.h"

namespace spk {
namespace {

constexpr int kBig = 1 << 29;

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m)
{
    int lo = __shfl_xor((int)(uint32_t)v, m, 64);
    int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

// 64x64 bit-matrix transpose across a wave: on entry lane j holds row j, on
// exit lane i holds column i (bit j of lane i = bit i of row j).  Stage s
// swaps the off-diagonal s x s blocks between lanes j and j ^ s.
__device__ __forceinline__ uint64_t transpose64(uint64_t a, int lane)
{
    constexpr uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull,
                                   0x00FF00FF00FF00FFull, 0x0F0F0F0F0F0F0F0Full,
                                   0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int i = 0; i < 6; i++) {
        const int s = 32 >> i;
        const uint64_t m = masks[i];  // bit positions with (pos & s) == 0
        const uint64_t y = shfl_xor64(a, s);
        const bool up = (lane & s) != 0;
        const uint64_t sh = up ? (y >> s) : (y << s);
        const uint64_t keep = up ? ~m : m;
        a = (a & keep) | (sh & ~keep);
    }
    return a;
}

__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }
__device__ __forceinline__ int hibit64(uint64_t v) { return 63 - __builtin_clzll(v); }
__device__ __forceinline__ int popc64(uint64_t v) { return __builtin_popcountll(v); }

// Single-wave workgroups are dispatched round-robin over the 8 XCDs; give
// each XCD a contiguous range of pixel strips.
__device__ __forceinline__ int xcd_strip(int b, int nblocks)
{
    const int q = nblocks / 8, r = nblocks % 8;
    const int xcd = b % 8, j = b / 8;
    return xcd < r ? xcd * (q + 1) + j : r * (q + 1) + (xcd - r) * q + j;
}

template <int MODE>
struct Emitter {
    const ReconParams &P;
    int64_t p;
    bool valid;
    int32_t segc;

    // A closed segment spanning spike frames [first, last] with n intervals
    // covers sorted outputs [k0, kend).
    __device__ __forceinline__ void close(int32_t first, int32_t last, int32_t n, int32_t k0,
                                          int32_t kend)
    {
        if (!valid) return;
        if (MODE == MODE_SEGMENTS) {
            if (segc < P.cap) {
                const int64_t o = (int64_t)segc * P.HW + p;
                P.seg_first[o] = first;
                P.seg_last[o] = last;
                P.seg_n[o] = n;
            }
            segc++;
        } else {
            // Eq. 6: theta / ((1/N) sum T0(i)); the N intervals sum to last - first
            const float I = (float)(P.theta * (double)n / (double)(last - first));
            for (int32_t k = k0; k < kend; k++) {
                const int32_t pl = P.plane ? P.plane[k] : k;
                const int64_t o = (int64_t)pl * P.HW + p;
                if (P.out) P.out[o] = I;
                if (P.win_first) P.win_first[o] = first;
                if (P.win_last) P.win_last[o] = last;
                if (P.win_n) P.win_n[o] = n;
            }
        }
    }

    // Fewer than two spikes: no interval, output 0 and window (-1, -1, 0).
    __device__ __forceinline__ void empty()
    {
        if (!valid || MODE == MODE_SEGMENTS) return;
        for (int32_t k = 0; k < P.n_out; k++) {
            const int32_t pl = P.plane ? P.plane[k] : k;
            const int64_t o = (int64_t)pl * P.HW + p;
            if (P.out) P.out[o] = 0.0f;
            if (P.win_first) P.win_first[o] = -1;
            if (P.win_last) P.win_last[o] = -1;
            if (P.win_n) P.win_n[o] = 0;
        }
    }
};

template <int ORDER, int MODE>
__global__ __launch_bounds__(64) void recon_kernel(ReconParams P, int nblocks)
{
    __shared__ int32_t cnt_s[64];
    const int lane = threadIdx.x;
    const int64_t p0 = (int64_t)xcd_strip(blockIdx.x, nblocks) * 64;
    const int64_t p = p0 + lane;
    Emitter<MODE> em{P, p, p < P.HW, 0};
    const uint8_t *base = P.stream + (p0 >> 3);

    // per-pixel state, all in registers
    int32_t lastspk = -1;   // frame of the latest spike
    int32_t cnt_last = 0;   // number of sorted outputs at or before lastspk
    int32_t cum = 0;        // spikes so far
    int32_t first = -1;     // first spike frame of the open segment
    int32_t first_idx = 0;  // its index among the pixel's spikes
    int32_t k0 = 0;         // first sorted output owned by the open segment
    int32_t flo = kBig, fhi = -kBig;  // extremes of the open FSR segment's S1
    // SSR: per interval value (keyed by parity; an FSR segment holds two
    // adjacent values at most) the index of its last occurrence and the
    // extremes of its S2 gaps inside the open segment
    int32_t gidx = 0;
    int32_t l0 = -1, l1 = -1, g0l = kBig, g0h = -kBig, g1l = kBig, g1h = -kBig;

    for (int32_t t0 = 0; t0 < P.T; t0 += 64) {
        const int32_t tr = t0 + lane;
        uint64_t row = 0;
        int32_t c = 0;
        if (tr < P.T) {
            row = *(const uint64_t *)(base + (int64_t)tr * P.fb);
            if (MODE == MODE_RECON) c = P.cnt_le[tr];
        }
        cnt_s[lane] = c;
        uint64_t w = transpose64(row, lane);
        __syncthreads();
        if (w) {
            const uint64_t wfull = w;
            const int32_t cum0 = cum, lastspk0 = lastspk, cnt_last0 = cnt_last;
            int32_t lp;  // position of the previous spike relative to t0
            if (lastspk < 0) {
                // the pixel's first spike opens its first segment
                const int pos = ctz64(w);
                w &= w - 1;
                first = t0 + pos;
                first_idx = 0;
                lp = pos;
            } else {
                lp = lastspk - t0;
            }
            uint64_t B = 0;  // spikes whose interval opens a new segment
            while (w) {
                const int pos = ctz64(w);
                w &= w - 1;
                const int32_t x = pos - lp;  // interval T0 ending at this spike
                lp = pos;
                const int32_t nlo = min(flo, x), nhi = max(fhi, x);
                const bool fcut = nhi - nlo > 1;  // S1 leaves zero-order stability
                bool cut = fcut;
                if (ORDER == 2) {
                    const bool odd = x & 1;
                    const int32_t l = odd ? l1 : l0;
                    const int32_t gl = odd ? g1l : g0l, gh = odd ? g1h : g0h;
                    const int32_t d = gidx - l;  // new element of S2 for value x
                    const int32_t ngl = min(gl, d), ngh = max(gh, d);
                    cut = fcut || (l >= 0 && ngh - ngl > 1);
                    const bool fresh = cut || l < 0;
                    const int32_t ugl = fresh ? kBig : ngl, ugh = fresh ? -kBig : ngh;
                    if (odd) {
                        l1 = gidx; g1l = ugl; g1h = ugh;
                        if (cut) { l0 = -1; g0l = kBig; g0h = -kBig; }
                    } else {
                        l0 = gidx; g0l = ugl; g0h = ugh;
                        if (cut) { l1 = -1; g1l = kBig; g1h = -kBig; }
                    }
                    gidx++;
                }
                flo = fcut ? x : nlo;
                fhi = fcut ? x : nhi;
                B |= (uint64_t)cut << pos;
            }
            // close the segments that ended in this word
            while (B) {
                const int cpos = ctz64(B);
                B &= B - 1;
                const uint64_t below = wfull & ((1ull << cpos) - 1);
                int32_t last, kend;
                if (below) {
                    const int bp = hibit64(below);
                    last = t0 + bp;
                    kend = cnt_s[bp];
                } else {
                    last = lastspk0;
                    kend = cnt_last0;
                }
                const int32_t last_idx = cum0 + popc64(below) - 1;
                em.close(first, last, last_idx - first_idx, k0, kend);
                first = last;
                first_idx = last_idx;
                k0 = kend;
            }
            cum = cum0 + popc64(wfull);
            const int hp = hibit64(wfull);
            lastspk = t0 + hp;
            cnt_last = cnt_s[hp];
        }
        __syncthreads();
    }
    if (cum >= 2)
        em.close(first, lastspk, (cum - 1) - first_idx, k0, P.n_out);
    else
        em.empty();
    if (MODE == MODE_SEGMENTS && em.valid) P.count[p] = em.segc;
}

}  // namespace

hipError_t launch_recon(const ReconParams &p, int order, Mode mode, hipStream_t stream)
{
    const int nblocks = (int)((p.HW + 63) / 64);
    if (nblocks <= 0) return hipSuccess;
    dim3 grid(nblocks), block(64);
    if (order == 1 && mode == MODE_RECON)
        hipLaunchKernelGGL((recon_kernel<1, MODE_RECON>), grid, block, 0, stream, p, nblocks);
    else if (order == 2 && mode == MODE_RECON)
        hipLaunchKernelGGL((recon_kernel<2, MODE_RECON>), grid, block, 0, stream, p, nblocks);
    else if (order == 1)
        hipLaunchKernelGGL((recon_kernel<1, MODE_SEGMENTS>), grid, block, 0, stream, p, nblocks);
    else
        hipLaunchKernelGGL((recon_kernel<2, MODE_SEGMENTS>), grid, block, 0, stream, p, nblocks);
    return hipGetLastError();
}

}  // namespace spk
