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
constexpr int kTargetWaves = 12288;  // chunk a stream until this many waves run
constexpr int kMinChunkTiles = 16;   // shortest chunk worth a separate wave
constexpr int kWarmTiles = 4;        // speculative warm-up before a chunk
constexpr int kCaptureTiles = 4;     // tiles after a chunk's start that record the
                                     // first segment's window for the fixup pass

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
    int32_t kmin;            // outputs below this belong to an earlier chunk

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
            k0 = max(k0, kmin);
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

// Running state of one pixel.
struct Run {
    int32_t lastspk;    // frame of the latest spike (-1: none yet)
    int32_t cnt_last;   // number of sorted outputs at or before lastspk
    int32_t cum;        // spikes so far
    int32_t first;      // first spike frame of the open segment
    int32_t first_idx;  // its index among the pixel's spikes
    int32_t k0;         // first sorted output owned by the open segment
    int32_t lastb;      // last spike of the latest closed segment (-1: none)
    int32_t cs;         // first frame of the chunk (0 outside chunked runs)
    int32_t fb1, fn1;   // first segment closed at or after cs: last spike, N,
    int32_t fi1;        //   index of that last spike,
    int32_t fwlo, fwhi; //   and its FSR window
    SegState st;

    __device__ __forceinline__ void reset(int32_t k0_, int32_t cs_ = 0)
    {
        lastspk = -1;
        cnt_last = 0;
        cum = 0;
        first = -1;
        first_idx = 0;
        k0 = k0_;
        lastb = -1;
        cs = cs_;
        fb1 = -1;
        fn1 = 0;
        fi1 = 0;
        fwlo = kBig;  // kBig: not captured yet
        fwhi = -kBig;
        st.reset();
    }

    // One interval; while CAPTURE, the FSR window of the first segment that
    // closes at or after the chunk's start is kept for the fixup pass.
    template <int ORDER, bool CAPTURE>
    __device__ __forceinline__ bool step_capture(int32_t x, int32_t tau)
    {
        if constexpr (ORDER == 1 && CAPTURE) {
            const int32_t lo = st.flo, hi = st.fhi;
            const bool cut = st.template step<ORDER>(x);
            if (cut && fwlo == kBig && tau - x >= cs) {
                fwlo = lo;
                fwhi = hi;
            }
            return cut;
        } else {
            return st.template step<ORDER>(x);
        }
    }

    // Process the 64-frame word w starting at frame t0; cnt_row[j] is the
    // number of sorted outputs at or before frame t0 + j.
    template <int ORDER, bool CAPTURE, class EM>
    __device__ __forceinline__ void word(int32_t t0, uint64_t w, const int32_t *cnt_row, EM &em)
    {
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
        // walk the spikes of each 32-bit half; B marks spikes whose interval
        // opens a new segment
        uint32_t Blo = 0, Bhi = 0;
        uint32_t h = (uint32_t)w;
        while (h) {
            const uint32_t nh = h & (h - 1);
            const int pos = __builtin_ctz(h);
            const int32_t x = pos - lp;  // interval T0 ending at this spike
            lp = pos;
            Blo |= step_capture<ORDER, CAPTURE>(x, t0 + pos) ? (h ^ nh) : 0u;
            h = nh;
        }
        h = (uint32_t)(w >> 32);
        while (h) {
            const uint32_t nh = h & (h - 1);
            const int pos = __builtin_ctz(h) + 32;
            const int32_t x = pos - lp;
            lp = pos;
            Bhi |= step_capture<ORDER, CAPTURE>(x, t0 + pos) ? (h ^ nh) : 0u;
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
                kend = cnt_row[bp];
            } else {
                last = lastspk0;
                kend = cnt_last0;
            }
            const int32_t last_idx = cum0 + popc64(below) - 1;
            em.close(first, last, last_idx - first_idx, k0, kend);
            if (fb1 < 0 && last >= cs) {
                fb1 = last;
                fn1 = last_idx - first_idx;
                fi1 = last_idx;
            }
            first = last;
            first_idx = last_idx;
            k0 = kend;
            lastb = last;
        }
        cum = cum0 + popc64(wfull);
        const int hp = hibit64(wfull);
        lastspk = t0 + hp;
        cnt_last = cnt_row[hp];
    }
};

// Per-chunk record of the running state at the chunk's end, [field][chunk][pixel].
enum RecField {
    R_LASTSPK, R_CNTLAST, R_CUM, R_FIRST, R_FIRSTIDX, R_K0, R_LASTB, R_FB1, R_FN1,
    R_FI1, R_FWLO, R_FWHI,
    R_FLO, R_FHI, R_NP, R_L0, R_L1, R_G0L, R_G0H, R_G1L, R_G1H, R_NFIELDS
};
static_assert(R_NFIELDS == kRecFields, "record layout");

// Records of chunk c: the state at the chunk's end (all chunks) and the
// warmed-up speculative state at its start (chunks > 0), each [field][chunk][HW].
__device__ __forceinline__ int32_t *rec_end(const ChunkPlan &cp, int c, int64_t p, int32_t HW)
{
    return cp.rec + (int64_t)c * HW + p;
}
__device__ __forceinline__ int32_t *rec_start(const ChunkPlan &cp, int c, int64_t p, int32_t HW)
{
    return cp.rec + (int64_t)R_NFIELDS * cp.nchunks * HW + (int64_t)c * HW + p;
}

__device__ __forceinline__ void save_run(int32_t *rec, int64_t stride, const Run &r)
{
    const int32_t v[R_NFIELDS] = {r.lastspk, r.cnt_last, r.cum, r.first, r.first_idx, r.k0,
                                  r.lastb, r.fb1, r.fn1, r.fi1, r.fwlo, r.fwhi,
                                  r.st.flo, r.st.fhi, r.st.np,
                                  r.st.l0, r.st.l1,
                                  r.st.g0l, r.st.g0h, r.st.g1l, r.st.g1h};
#pragma unroll
    for (int f = 0; f < R_NFIELDS; f++) rec[f * stride] = v[f];
}

__device__ __forceinline__ void load_run(const int32_t *rec, int64_t stride, Run &r)
{
    int32_t v[R_NFIELDS];
#pragma unroll
    for (int f = 0; f < R_NFIELDS; f++) v[f] = rec[f * stride];
    r.lastspk = v[R_LASTSPK];
    r.cnt_last = v[R_CNTLAST];
    r.cum = v[R_CUM];
    r.first = v[R_FIRST];
    r.first_idx = v[R_FIRSTIDX];
    r.k0 = v[R_K0];
    r.lastb = v[R_LASTB];
    r.fb1 = v[R_FB1];
    r.fn1 = v[R_FN1];
    r.fi1 = v[R_FI1];
    r.fwlo = v[R_FWLO];
    r.fwhi = v[R_FWHI];
    r.cs = 0;
    r.st.flo = v[R_FLO];
    r.st.fhi = v[R_FHI];
    r.st.np = v[R_NP];
    r.st.l0 = v[R_L0];
    r.st.l1 = v[R_L1];
    r.st.g0l = v[R_G0L];
    r.st.g0h = v[R_G0H];
    r.st.g1l = v[R_G1L];
    r.st.g1h = v[R_G1H];
}

// Two states make the same cut decisions for every continuation when their
// FSR extremes agree and, for SSR, each value's S2 gap extremes and the
// distance back to its latest occurrence agree (piece-local indices differ
// by a constant shift, which no decision sees).
template <int ORDER>
__device__ __forceinline__ bool same_decisions(const SegState &a, const SegState &b)
{
    if (a.flo != b.flo || a.fhi != b.fhi) return false;
    if constexpr (ORDER == 1) {
        return true;
    } else {
        const int32_t a0 = a.l0 < 0 ? -1 : a.np - a.l0, b0 = b.l0 < 0 ? -1 : b.np - b.l0;
        const int32_t a1 = a.l1 < 0 ? -1 : a.np - a.l1, b1 = b.l1 < 0 ? -1 : b.np - b.l1;
        return a0 == b0 && a1 == b1 && a.g0l == b.g0l && a.g0h == b.g0h && a.g1l == b.g1l &&
               a.g1h == b.g1h;
    }
}

// Main pass.  With nchunks == 1 a wave walks its strip's whole stream and
// finishes every segment.  With nchunks > 1 the stream is cut into chunks
// of chunk_tiles tiles; chunk 0 runs exactly, every later chunk starts from
// a fresh state at its first spike (speculation), and each wave records its
// state at its chunk's end for the fixup pass, which makes the result exact.
template <int ORDER, int MODE, bool WIN, int PMAP>
__global__ __launch_bounds__(64) void recon_kernel(ReconParams P, int nblocks, ChunkPlan cp)
{
    __shared__ uint64_t word_s[kGroup][64];
    __shared__ int32_t cnt_s[kGroup][64];
    extern __shared__ int32_t plane_dyn[];
    const int lane = threadIdx.x;
    const int L = xcd_strip(blockIdx.x, nblocks * cp.nchunks);
    const int chunk = L / nblocks;
    const int64_t p0 = (int64_t)(L % nblocks) * 64;
    const int64_t p = p0 + lane;
    if constexpr (PMAP == PMAP_LDS)
        for (int32_t k = lane; k < P.n_out; k += 64) plane_dyn[k] = P.plane[k];
    const int32_t ntiles = (P.T + 63) / 64;
    const int32_t tile0 = chunk * cp.chunk_tiles;
    const int32_t tile1 = min(ntiles, tile0 + cp.chunk_tiles);
    // a later chunk first warms its speculative state up on the tail of the
    // previous chunk; it writes no output before its own first frame
    const int32_t tilew = max(0, tile0 - (chunk > 0 ? cp.warm_tiles : 0));
    const int32_t kmin = tile0 > 0 && MODE == MODE_RECON ? P.cnt_le[tile0 * 64 - 1] : 0;
    Emitter<MODE, WIN, PMAP> em{P, plane_dyn, p, p < P.HW, 0, kmin};
    const uint8_t *base = P.stream + (p0 >> 3);
    const Xpose X(lane);
    const int64_t fstride = (int64_t)cp.nchunks * P.HW;

    Run run;
    run.reset(tilew > 0 && MODE == MODE_RECON ? P.cnt_le[tilew * 64 - 1] : 0, tile0 * 64);
    int32_t cum_base = 0;  // spikes seen before tile0

    uint32_t rlo[kGroup], rhi[kGroup];
    int32_t rc[kGroup];
    auto fetch = [&](int32_t tg) {
#pragma unroll
        for (int i = 0; i < kGroup; i++) {
            const int32_t tr = (tg + i) * 64 + lane;
            rlo[i] = rhi[i] = 0;
            rc[i] = 0;
            if (tg + i < tile1 && tr < P.T) {
                const uint2 v = *(const uint2 *)(base + (int64_t)tr * P.fb);
                rlo[i] = v.x;
                rhi[i] = v.y;
                if (MODE == MODE_RECON) rc[i] = P.cnt_le[tr];
            }
        }
    };
    fetch(tilew);
    for (int32_t tg = tilew; tg < tile1; tg += kGroup) {
        // the group's rows are in registers: transpose into LDS, then start
        // fetching the next group
#pragma unroll
        for (int i = 0; i < kGroup; i++) {
            word_s[i][lane] = transpose64(rlo[i], rhi[i], X, lane);
            cnt_s[i][lane] = rc[i];
        }
        fetch(tg + kGroup);
        __syncthreads();
        const int32_t ni = min(kGroup, tile1 - tg);
        for (int i = 0; i < ni; i++) {
            if (tg + i == tile0 && chunk > 0) {
                // the speculative state the fixup pass starts from
                if (em.valid) save_run(rec_start(cp, chunk, p, P.HW), fstride, run);
                cum_base = run.cum;
            }
            const uint64_t w = word_s[i][lane];
            // the first tiles of a later chunk keep what the fixup pass needs
            const int32_t t = tg + i;
            if (ORDER == 1 && chunk > 0 && t >= tile0 && t < tile0 + kCaptureTiles) {
                if (w) run.template word<ORDER, true>(t * 64, w, cnt_s[i], em);
            } else {
                if (w) run.template word<ORDER, false>(t * 64, w, cnt_s[i], em);
            }
        }
        __syncthreads();
    }
    if (cp.nchunks > 1) {
        // end-of-chunk record, spike indices relative to the chunk's start
        run.cum -= cum_base;
        run.first_idx -= cum_base;
        run.fi1 -= cum_base;
        if (em.valid) save_run(rec_end(cp, chunk, p, P.HW), fstride, run);
        return;
    }
    if (run.cum >= 2)
        em.close(run.first, run.lastspk, (run.cum - 1) - run.first_idx, run.k0, P.n_out);
    else
        em.empty();
    if (MODE == MODE_SEGMENTS && em.valid) P.count[p] = em.segc;
}

// Fixup pass for chunked runs (one wave per strip, chunks in order).  The
// true state entering chunk c is known; the wave replays chunk c spike by
// spike with two state machines -- the true one, and the speculative one of
// the main pass (restored from its record at the chunk's start) -- writing
// the true segments it closes.  Once the two make the same decisions the
// rest of the chunk is the main pass's: a lane stops replaying when both
// machines are in equivalent states and either (a) the main pass cut no
// segment after this spike (the open segment then runs to the chunk's end),
// or (b) both have the same open segment (its outputs before the chunk,
// which the main pass does not write, are written here from the main pass's
// record of where it closes).  For FSR a lane also stops when the true
// window contains the speculative one and stays stable up to the main
// pass's next cut (or to the chunk's end if there is none): the true machine
// then cuts exactly there too.  The lane then takes the main pass's
// end-of-chunk record (keeping its own open segment where that segment
// outlives the chunk).  Stopping is exact because cut decisions depend only
// on the state and the intervals that follow.
template <int ORDER, int MODE, bool WIN, int PMAP>
__global__ __launch_bounds__(64) void fixup_kernel(ReconParams P, int nblocks, ChunkPlan cp)
{
    __shared__ int32_t cnt_s[64];
    extern __shared__ int32_t plane_dyn[];
    const int lane = threadIdx.x;
    const int64_t p0 = (int64_t)xcd_strip(blockIdx.x, nblocks) * 64;
    const int64_t p = p0 + lane;
    if constexpr (PMAP == PMAP_LDS)
        for (int32_t k = lane; k < P.n_out; k += 64) plane_dyn[k] = P.plane[k];
    Emitter<MODE, WIN, PMAP> em{P, plane_dyn, p, p < P.HW, 0, 0};
    const uint8_t *base = P.stream + (p0 >> 3);
    const Xpose X(lane);
    const int64_t fstride = (int64_t)cp.nchunks * P.HW;
    const int32_t ntiles = (P.T + 63) / 64;

    Run tr;
    if (em.valid) load_run(rec_end(cp, 0, p, P.HW), fstride, tr);
    else tr.reset(0);
    for (int c = 1; c < cp.nchunks; c++) {
        Run rc, sp;
        if (em.valid) {
            load_run(rec_end(cp, c, p, P.HW), fstride, rc);
            load_run(rec_start(cp, c, p, P.HW), fstride, sp);
        } else {
            rc.reset(0);
            sp.reset(0);
        }
        const int32_t cum_start = tr.cum;
        bool done = rc.cum == 0;  // no spike in this chunk: nothing changes
        const int32_t tile0 = c * cp.chunk_tiles;
        const int32_t tile1 = min(ntiles, tile0 + cp.chunk_tiles);
        const int32_t kmin = P.cnt_le[tile0 * 64 - 1];  // the main pass wrote nothing below
        // rows are fetched one tile ahead
        uint32_t nlo = 0, nhi = 0;
        int32_t ncv = 0;
        auto fetch = [&](int32_t t) {
            const int32_t f = t * 64 + lane;
            nlo = nhi = 0;
            ncv = 0;
            if (t < tile1 && f < P.T) {
                const uint2 v = *(const uint2 *)(base + (int64_t)f * P.fb);
                nlo = v.x;
                nhi = v.y;
                ncv = P.cnt_le[f];
            }
        };
        if (__any(!done)) fetch(tile0);
        for (int32_t t = tile0; t < tile1 && __any(!done); t++) {
            const uint32_t lo = nlo, hi = nhi;
            cnt_s[lane] = ncv;
            fetch(t + 1);
            uint64_t w = transpose64(lo, hi, X, lane);
            __syncthreads();
            while (!done && w) {
                const int pos = ctz64(w);
                w &= w - 1;
                const int32_t tau = t * 64 + pos;
                if (tr.lastspk < 0) {
                    tr.first = tau;
                    tr.first_idx = tr.cum;
                } else if (tr.st.template step<ORDER>(tau - tr.lastspk)) {
                    em.close(tr.first, tr.lastspk, (tr.cum - 1) - tr.first_idx, tr.k0,
                             tr.cnt_last);
                    tr.first = tr.lastspk;
                    tr.first_idx = tr.cum - 1;
                    tr.k0 = tr.cnt_last;
                }
                if (sp.lastspk < 0) {
                    sp.first = tau;
                } else if (sp.st.template step<ORDER>(tau - sp.lastspk)) {
                    sp.first = sp.lastspk;
                    sp.k0 = tr.cnt_last;  // outputs up to the shared previous spike
                }
                tr.lastspk = sp.lastspk = tau;
                tr.cum++;
                tr.cnt_last = cnt_s[pos];
                if (ORDER == 1 && rc.fb1 >= tau && tr.st.flo <= sp.st.flo &&
                    sp.st.fhi <= tr.st.fhi &&
                    max(tr.st.fhi, rc.fwhi) - min(tr.st.flo, rc.fwlo) <= 1) {
                    // FSR: the true window holds the speculative one and stays
                    // stable with every interval up to the main pass's next
                    // cut, so the true machine makes that same cut next and
                    // both restart there: close the true segment at that cut
                    // and take the main pass's record from then on
                    em.close(tr.first, rc.fb1, cum_start + rc.fi1 - tr.first_idx, tr.k0,
                             P.cnt_le[rc.fb1]);
                    tr = rc;
                    tr.cum = cum_start + rc.cum;
                    tr.first_idx = cum_start + rc.first_idx;
                    done = true;
                } else if (ORDER == 1 && rc.lastb < tau && tr.st.flo <= sp.st.flo &&
                    sp.st.fhi <= tr.st.fhi &&
                    max(tr.st.fhi, rc.st.fhi) - min(tr.st.flo, rc.st.flo) <= 1) {
                    // FSR: the main pass makes no cut after this spike, the
                    // true window holds the speculative one, and together
                    // with every interval still to come (the main pass's final
                    // window) it stays stable: no true cut either, and the
                    // true window at the chunk's end is the union
                    const int32_t first = tr.first, first_idx = tr.first_idx, k0 = tr.k0;
                    const int32_t flo = min(tr.st.flo, rc.st.flo), fhi = max(tr.st.fhi, rc.st.fhi);
                    tr = rc;
                    tr.cum = cum_start + rc.cum;
                    tr.first = first;
                    tr.first_idx = first_idx;
                    tr.k0 = k0;
                    tr.st.flo = flo;
                    tr.st.fhi = fhi;
                    done = true;
                } else if (same_decisions<ORDER>(tr.st, sp.st)) {
                    if (rc.lastb < tau) {
                        const int32_t first = tr.first, first_idx = tr.first_idx, k0 = tr.k0;
                        tr = rc;
                        tr.cum = cum_start + rc.cum;
                        tr.first = first;
                        tr.first_idx = first_idx;
                        tr.k0 = k0;
                        done = true;
                    } else if (tr.first == sp.first && tr.k0 >= sp.k0) {
                        // same open segment: the main pass writes its outputs
                        // from the chunk's start on (those it gave it below
                        // tr.k0 were rewritten by this pass); earlier ones
                        // are written here, from the main pass's record of
                        // where this segment closes
                        if (tr.k0 < kmin && rc.fb1 >= 0)
                            em.close(tr.first, rc.fb1, rc.fn1, tr.k0, kmin);
                        tr = rc;
                        tr.cum = cum_start + rc.cum;
                        tr.first_idx = cum_start + rc.first_idx;
                        done = true;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (tr.cum >= 2)
        em.close(tr.first, tr.lastspk, (tr.cum - 1) - tr.first_idx, tr.k0, P.n_out);
    else
        em.empty();
}

template <int ORDER, int MODE, bool WIN, int PMAP>
hipError_t launch_one(const ReconParams &p, const ChunkPlan &cp, hipStream_t stream)
{
    const int nblocks = (int)((p.HW + 63) / 64);
    const size_t shmem = PMAP == PMAP_LDS ? (size_t)p.n_out * sizeof(int32_t) : 0;
    hipLaunchKernelGGL((recon_kernel<ORDER, MODE, WIN, PMAP>), dim3(nblocks * cp.nchunks),
                       dim3(64), shmem, stream, p, nblocks, cp);
    if (cp.nchunks > 1)
        hipLaunchKernelGGL((fixup_kernel<ORDER, MODE, WIN, PMAP>), dim3(nblocks), dim3(64),
                           shmem, stream, p, nblocks, cp);
    return hipGetLastError();
}

template <int ORDER, int MODE, bool WIN>
hipError_t launch_pmap(const ReconParams &p, const ChunkPlan &cp, hipStream_t stream)
{
    if (MODE == MODE_SEGMENTS || !p.plane)
        return launch_one<ORDER, MODE, WIN, PMAP_IDENT>(p, cp, stream);
    if (p.n_out <= kMaxLdsPlanes) return launch_one<ORDER, MODE, WIN, PMAP_LDS>(p, cp, stream);
    return launch_one<ORDER, MODE, WIN, PMAP_GLOBAL>(p, cp, stream);
}

}  // namespace

ChunkPlan plan_chunks(int32_t HW, int32_t T, int requested, int warm)
{
    ChunkPlan cp;
    const int nblocks = (HW + 63) / 64;
    const int ntiles = (T + 63) / 64;
    int c = requested;
    if (c <= 0) {
        c = (kTargetWaves + nblocks - 1) / nblocks;  // enough waves to fill the chip
        c = min(c, ntiles / kMinChunkTiles);          // chunks long enough to pay off
    }
    c = max(1, min(c, ntiles));
    cp.nchunks = c;
    cp.chunk_tiles = (ntiles + c - 1) / c;
    cp.nchunks = (ntiles + cp.chunk_tiles - 1) / cp.chunk_tiles;
    if (cp.nchunks < 1) cp.nchunks = 1;
    cp.warm_tiles = warm >= 0 ? warm : min(kWarmTiles, cp.chunk_tiles / 2);
    return cp;
}

hipError_t launch_recon(const ReconParams &p, int order, Mode mode, const ChunkPlan &cp,
                        hipStream_t stream)
{
    if (p.HW <= 0) return hipSuccess;
    const bool win = p.win_first || p.win_last || p.win_n || !p.out;
    if (mode == MODE_SEGMENTS) {
        ChunkPlan one;
        return order == 1 ? launch_one<1, MODE_SEGMENTS, false, PMAP_IDENT>(p, one, stream)
                          : launch_one<2, MODE_SEGMENTS, false, PMAP_IDENT>(p, one, stream);
    }
    if (win)
        return order == 1 ? launch_pmap<1, MODE_RECON, true>(p, cp, stream)
                          : launch_pmap<2, MODE_RECON, true>(p, cp, stream);
    return order == 1 ? launch_pmap<1, MODE_RECON, false>(p, cp, stream)
                      : launch_pmap<2, MODE_RECON, false>(p, cp, stream);
}

}  // namespace spk
