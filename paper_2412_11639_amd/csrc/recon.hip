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
// per pixel) and walks time in tiles of 64 frames, grouped by kGroup:
//   1. lane j loads the 8-byte word of frame t0 + j covering the wave's 64
//      pixels (frame-major input); the loads of the next group are issued
//      before the current group is processed, so HBM latency overlaps work
//      and the wave waits on memory once per group;
//   2. a 6-stage butterfly transposes each 64x64 bit block so lane i holds
//      pixel i's 64-frame time word (bit j = frame t0 + j): DPP row moves
//      for distances 1..8, lane-swap permutes for 16 and 32 (no LDS);
//   3. each lane walks its spikes with find-first-set and runs the
//      segmentation state machine (registers only), marking in a mask the
//      spikes whose interval opens a new segment;
//   4. a second loop walks that mask, recovers each closed segment's
//      window (first/last spike frame, N by popcount) and writes its
//      intensity to every output time the segment covers.
// Workgroups are single waves; block ids are remapped so consecutive pixel
// strips share an XCD (and its L2), since 16 waves read each 128-byte line.
#include "spk_internal.h"

namespace spk {
namespace {

constexpr int kBig = 1 << 29;
constexpr int kGroup = 8;          // tiles per prefetch group
constexpr int kMaxLdsPlanes = 8192;  // plane map staged in LDS up to this size

// ---- cross-lane moves ----------------------------------------------------

template <int S>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int lane)
{
    if constexpr (S == 1) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (S == 2) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (S == 4 || S == 8) {
        // within a row of 16 lanes: lanes with bit S clear read lane + S
        // (row_shl), the others lane - S (row_shr)
        const int up = __builtin_amdgcn_update_dpp(0, (int)v, 0x100 + S, 0xF, 0xF, false);
        const int dn = __builtin_amdgcn_update_dpp(0, (int)v, 0x110 + S, 0xF, 0xF, false);
        return (uint32_t)((lane & S) ? dn : up);
    } else {
        static_assert(S == 16, "lane_xor");
        // swap rows 1<->0 and 3<->2 of 16 lanes
        auto r = __builtin_amdgcn_permlane16_swap((int)v, (int)v, false, false);
        return (uint32_t)((lane & 16) ? r[0] : r[1]);
    }
}

// Per-lane constants of the transpose stages s = 16, 8, 4, 2, 1 acting on
// each 32-bit half: the bits a lane keeps and the rotation that brings the
// partner's bits into place.
struct Xpose {
    uint32_t keep[5];
    uint32_t rot[5];
    __device__ __forceinline__ explicit Xpose(int lane)
    {
        constexpr uint32_t m[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u,
                                   0x55555555u};
#pragma unroll
        for (int i = 0; i < 5; i++) {
            const int s = 16 >> i;
            const bool up = (lane & s) != 0;
            keep[i] = up ? ~m[i] : m[i];
            rot[i] = up ? (uint32_t)s : (uint32_t)(32 - s);
        }
    }
};

template <int I>
__device__ __forceinline__ uint32_t xstage(uint32_t v, const Xpose &X, int lane)
{
    constexpr int s = 16 >> I;
    const uint32_t y = lane_xor<s>(v, lane);
    // rotate the partner's word so its swapped block lands in place; bits
    // wrapped around by the rotation fall outside the taken mask
    const uint32_t t = __builtin_amdgcn_alignbit(y, y, X.rot[I]);
    return (v & X.keep[I]) | (t & ~X.keep[I]);
}

// 64x64 bit-matrix transpose across a wave: on entry lane j holds row j as
// (lo, hi), on exit lane i holds column i (bit j of lane i = bit i of row j).
// Stage s swaps the off-diagonal s x s blocks between lanes j and j ^ s.
__device__ __forceinline__ uint64_t transpose64(uint32_t lo, uint32_t hi, const Xpose &X,
                                                int lane)
{
    // s = 32: lanes 32..63 take the partner's high word as their low word,
    // lanes 0..31 the partner's low word as their high word
    auto r = __builtin_amdgcn_permlane32_swap((int)lo, (int)hi, false, false);
    lo = (uint32_t)r[0];
    hi = (uint32_t)r[1];
    lo = xstage<0>(lo, X, lane);
    hi = xstage<0>(hi, X, lane);
    lo = xstage<1>(lo, X, lane);
    hi = xstage<1>(hi, X, lane);
    lo = xstage<2>(lo, X, lane);
    hi = xstage<2>(hi, X, lane);
    lo = xstage<3>(lo, X, lane);
    hi = xstage<3>(hi, X, lane);
    lo = xstage<4>(lo, X, lane);
    hi = xstage<4>(hi, X, lane);
    return ((uint64_t)hi << 32) | lo;
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

// Segmentation state of one pixel (registers).
struct SegState {
    int32_t flo, fhi;  // extremes of the open FSR segment's S1 values
    // SSR: inside the open piece, per interval value (keyed by parity: an
    // FSR segment holds at most two adjacent values) the piece-local index
    // of its latest occurrence (-1: none) and the extremes of its S2 gaps
    int32_t np;        // intervals in the open piece
    int32_t l0, l1, g0l, g0h, g1l, g1h;

    __device__ __forceinline__ void reset()
    {
        flo = kBig;
        fhi = -kBig;
        np = 0;
        l0 = l1 = -1;
        g0l = g1l = kBig;
        g0h = g1h = -kBig;
    }

    // Add interval x; returns true if x opens a new segment (the previous
    // spike then ends the closed one).
    template <int ORDER>
    __device__ __forceinline__ bool step(int32_t x)
    {
        const int32_t nlo = min(flo, x), nhi = max(fhi, x);
        const bool fcut = nhi - nlo > 1;  // S1 leaves zero-order stability
        flo = fcut ? x : nlo;
        fhi = fcut ? x : nhi;
        if constexpr (ORDER == 1) {
            return fcut;
        } else {
            const bool odd = x & 1;
            const int32_t l = odd ? l1 : l0;
            const int32_t gl = odd ? g1l : g0l, gh = odd ? g1h : g0h;
            const int32_t d = np - l;  // next element of S2 for value x
            const int32_t ngl = min(gl, d), ngh = max(gh, d);
            const bool cut = fcut || (l >= 0 && ngh - ngl > 1);
            const bool fresh = cut || l < 0;
            const int32_t ugl = fresh ? kBig : ngl, ugh = fresh ? -kBig : ngh;
            const int32_t idx = cut ? 0 : np;
            if (odd) {
                l1 = idx; g1l = ugl; g1h = ugh;
                l0 = cut ? -1 : l0; g0l = cut ? kBig : g0l; g0h = cut ? -kBig : g0h;
            } else {
                l0 = idx; g0l = ugl; g0h = ugh;
                l1 = cut ? -1 : l1; g1l = cut ? kBig : g1l; g1h = cut ? -kBig : g1h;
            }
            np = idx + 1;
            return cut;
        }
    }
};

// How output k (in time order) maps to its plane: identity, through an LDS
// copy of the map, or through the map in global memory (very large maps).
enum PlaneMap { PMAP_IDENT = 0, PMAP_LDS = 1, PMAP_GLOBAL = 2 };

// Writes of one pixel's closed segments.
template <int MODE, bool WIN, int PMAP>
struct Emitter {
    const ReconParams &P;
    const int32_t *plane_s;  // LDS copy of the plane map (PMAP_LDS)
    int64_t p;
    bool valid;
    int32_t segc;

    __device__ __forceinline__ int32_t plane(int32_t k) const
    {
        if constexpr (PMAP == PMAP_IDENT) return k;
        else if constexpr (PMAP == PMAP_LDS) return plane_s[k];
        else return P.plane[k];
    }

    // A closed segment spanning spike frames [first, last] with n intervals
    // covers sorted outputs [k0, kend).
    __device__ __forceinline__ void close(int32_t first, int32_t last, int32_t n, int32_t k0,
                                          int32_t kend)
    {
        if (!valid) return;
        if constexpr (MODE == MODE_SEGMENTS) {
            if (segc < P.cap) {
                const int64_t o = (int64_t)segc * P.HW + p;
                P.seg_first[o] = first;
                P.seg_last[o] = last;
                P.seg_n[o] = n;
            }
            segc++;
        } else {
            if (k0 >= kend) return;
            // Eq. 6: theta / ((1/N) sum T0(i)); the N intervals sum to last - first
            const float I = (float)(P.theta * (double)n / (double)(last - first));
            for (int32_t k = k0; k < kend; k++) {
                const int64_t o = (int64_t)plane(k) * P.HW + p;
                if constexpr (WIN) {
                    if (P.out) P.out[o] = I;
                    if (P.win_first) P.win_first[o] = first;
                    if (P.win_last) P.win_last[o] = last;
                    if (P.win_n) P.win_n[o] = n;
                } else {
                    P.out[o] = I;
                }
            }
        }
    }

    // Fewer than two spikes: no interval, output 0 and window (-1, -1, 0).
    __device__ __forceinline__ void empty()
    {
        if (!valid || MODE == MODE_SEGMENTS) return;
        for (int32_t k = 0; k < P.n_out; k++) {
            const int64_t o = (int64_t)plane(k) * P.HW + p;
            if constexpr (WIN) {
                if (P.out) P.out[o] = 0.0f;
                if (P.win_first) P.win_first[o] = -1;
                if (P.win_last) P.win_last[o] = -1;
                if (P.win_n) P.win_n[o] = 0;
            } else {
                P.out[o] = 0.0f;
            }
        }
    }
};

template <int ORDER, int MODE, bool WIN, int PMAP>
__global__ __launch_bounds__(64) void recon_kernel(ReconParams P, int nblocks)
{
    __shared__ uint64_t word_s[kGroup][64];
    __shared__ int32_t cnt_s[kGroup][64];
    extern __shared__ int32_t plane_dyn[];
    const int lane = threadIdx.x;
    const int64_t p0 = (int64_t)xcd_strip(blockIdx.x, nblocks) * 64;
    const int64_t p = p0 + lane;
    if constexpr (PMAP == PMAP_LDS)
        for (int32_t k = lane; k < P.n_out; k += 64) plane_dyn[k] = P.plane[k];
    Emitter<MODE, WIN, PMAP> em{P, plane_dyn, p, p < P.HW, 0};
    const uint8_t *base = P.stream + (p0 >> 3);
    const Xpose X(lane);

    // per-pixel state
    int32_t lastspk = -1;   // frame of the latest spike
    int32_t cnt_last = 0;   // number of sorted outputs at or before lastspk
    int32_t cum = 0;        // spikes so far
    int32_t first = -1;     // first spike frame of the open segment
    int32_t first_idx = 0;  // its index among the pixel's spikes
    int32_t k0 = 0;         // first sorted output owned by the open segment
    SegState st;
    st.reset();

    const int32_t ntiles = (P.T + 63) / 64;
    uint32_t rlo[kGroup], rhi[kGroup];
    int32_t rc[kGroup];
    auto fetch = [&](int32_t g) {
#pragma unroll
        for (int i = 0; i < kGroup; i++) {
            const int32_t tr = (g * kGroup + i) * 64 + lane;
            rlo[i] = rhi[i] = 0;
            rc[i] = 0;
            if (tr < P.T) {
                const uint2 v = *(const uint2 *)(base + (int64_t)tr * P.fb);
                rlo[i] = v.x;
                rhi[i] = v.y;
                if (MODE == MODE_RECON) rc[i] = P.cnt_le[tr];
            }
        }
    };
    fetch(0);
    for (int32_t g = 0; g * kGroup < ntiles; g++) {
        // the group's rows are in registers: transpose into LDS, then start
        // fetching the next group
#pragma unroll
        for (int i = 0; i < kGroup; i++) {
            word_s[i][lane] = transpose64(rlo[i], rhi[i], X, lane);
            cnt_s[i][lane] = rc[i];
        }
        fetch(g + 1);
        __syncthreads();
        const int32_t ni = min(kGroup, ntiles - g * kGroup);
        for (int i = 0; i < ni; i++) {
            const int32_t t0 = (g * kGroup + i) * 64;
            uint64_t w = word_s[i][lane];
            if (!w) continue;
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
            // walk the spikes of each 32-bit half; B marks spikes whose
            // interval opens a new segment
            uint32_t Blo = 0, Bhi = 0;
            uint32_t h = (uint32_t)w;
            while (h) {
                const uint32_t nh = h & (h - 1);
                const int pos = __builtin_ctz(h);
                const int32_t x = pos - lp;  // interval T0 ending at this spike
                lp = pos;
                Blo |= st.template step<ORDER>(x) ? (h ^ nh) : 0u;
                h = nh;
            }
            h = (uint32_t)(w >> 32);
            while (h) {
                const uint32_t nh = h & (h - 1);
                const int pos = __builtin_ctz(h) + 32;
                const int32_t x = pos - lp;
                lp = pos;
                Bhi |= st.template step<ORDER>(x) ? (h ^ nh) : 0u;
                h = nh;
            }
            // close the segments that ended in this word
            uint64_t B = ((uint64_t)Bhi << 32) | Blo;
            while (B) {
                const int cpos = ctz64(B);
                B &= B - 1;
                const uint64_t below = wfull & ((1ull << cpos) - 1);
                int32_t last, kend;
                if (below) {
                    const int bp = hibit64(below);
                    last = t0 + bp;
                    kend = cnt_s[i][bp];
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
            cnt_last = cnt_s[i][hp];
        }
        __syncthreads();
    }
    if (cum >= 2)
        em.close(first, lastspk, (cum - 1) - first_idx, k0, P.n_out);
    else
        em.empty();
    if (MODE == MODE_SEGMENTS && em.valid) P.count[p] = em.segc;
}

template <int ORDER, int MODE, bool WIN, int PMAP>
void launch_one(const ReconParams &p, hipStream_t stream)
{
    const int nblocks = (int)((p.HW + 63) / 64);
    const size_t shmem = PMAP == PMAP_LDS ? (size_t)p.n_out * sizeof(int32_t) : 0;
    hipLaunchKernelGGL((recon_kernel<ORDER, MODE, WIN, PMAP>), dim3(nblocks), dim3(64), shmem,
                       stream, p, nblocks);
}

template <int ORDER, int MODE, bool WIN>
void launch_pmap(const ReconParams &p, hipStream_t stream)
{
    if (MODE == MODE_SEGMENTS || !p.plane) launch_one<ORDER, MODE, WIN, PMAP_IDENT>(p, stream);
    else if (p.n_out <= kMaxLdsPlanes) launch_one<ORDER, MODE, WIN, PMAP_LDS>(p, stream);
    else launch_one<ORDER, MODE, WIN, PMAP_GLOBAL>(p, stream);
}

}  // namespace

hipError_t launch_recon(const ReconParams &p, int order, Mode mode, hipStream_t stream)
{
    if (p.HW <= 0) return hipSuccess;
    const bool win = p.win_first || p.win_last || p.win_n || !p.out;
    if (mode == MODE_SEGMENTS) {
        if (order == 1) launch_one<1, MODE_SEGMENTS, false, PMAP_IDENT>(p, stream);
        else launch_one<2, MODE_SEGMENTS, false, PMAP_IDENT>(p, stream);
    } else if (win) {
        if (order == 1) launch_pmap<1, MODE_RECON, true>(p, stream);
        else launch_pmap<2, MODE_RECON, true>(p, stream);
    } else {
        if (order == 1) launch_pmap<1, MODE_RECON, false>(p, stream);
        else launch_pmap<2, MODE_RECON, false>(p, stream);
    }
    return hipGetLastError();
}

}  // namespace spk
