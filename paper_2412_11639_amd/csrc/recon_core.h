// Device building blocks shared by the reconstruction kernels (plain,
// chunked and batched): the wave-wide 64x64 bit transpose, the per-pixel
// FSR/SSR state machine, the segment writer and the per-word walk.
#pragma once

#include <type_traits>

#include "spk_internal.h"

namespace spk {
namespace {

constexpr int kBig = 1 << 29;
constexpr int kGroup = 8;          // tiles per prefetch group
constexpr int kMaxLdsPlanes = 8192;  // plane map staged in LDS up to this size
constexpr int kTargetWaves = 12288;  // chunk a stream until this many waves run (no occupancy)
constexpr int kMaxAutoChunks = 64;   // largest automatic chunk count
constexpr int kMinChunkTiles = 16;   // shortest chunk worth a separate wave
constexpr int kWarmTiles = 4;        // speculative warm-up before a chunk
constexpr int kCaptureTiles = 4;     // tiles after a chunk's start that record the
                                     // first segment's window for the fixup pass

// Global-memory view of a pointer.  Pointers that reach a kernel through a
// table in device memory (the batched jobs) are generic to the compiler,
// which then emits flat loads and stores; those count against the LDS wait
// counter too, so every LDS wait would also wait for the stream prefetch.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gp(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// ---- cross-lane moves ----------------------------------------------------

// Each DPP move below reads a valid source lane for every lane, so no old
// value is needed (a DPP update with an old value costs an extra move).
template <int S>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int lane)
{
    if constexpr (S == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);  // quad [1,0,3,2]
    } else if constexpr (S == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);  // quad [2,3,0,1]
    } else if constexpr (S == 4) {
        // mirror within 8 lanes (i ^ 7), then within 4 (i ^ 3): i ^ 4
        const int m = __builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true);
        return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, true);
    } else if constexpr (S == 8) {
        // rotate a row of 16 lanes by 8: i ^ 8
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, true);
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
    // keep ? v : t, bit by bit, in one instruction (table index 4v + 2t + keep)
    return __builtin_amdgcn_bitop3_b32(v, t, X.keep[I], 0xE4);
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

// True when every gap between consecutive spikes of the nonzero word w (c
// spikes) is a, or a or a + 1 when plus1; 1 <= a <= 62.  No walk: the c - 1
// gaps sum to the distance from the first spike to the last.  Give each
// spike but the last the spike a frames later if there is one, else (plus1)
// the one a + 1 frames later, and fail if neither exists.  Each chosen gap is
// at least the true one, so the chosen gaps sum to that distance exactly
// when every true gap is a or a + 1; the n1 = popc(w & (w >> a)) gaps of a
// and c - 1 - n1 of a + 1 sum to (c - 1)(a + 1) - n1.
// a * b for 0 <= a, b < 2^24 (here both below 64): one full-rate 24-bit
// multiply.  Written out, because the compiler emits the quarter-rate 32-bit
// multiply when it cannot prove the operands small.
__device__ __forceinline__ int32_t mul_small(int32_t a, int32_t b)
{
    int32_t r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ bool gaps_within(uint64_t w, int a, bool plus1, int32_t c)
{
    const int hi = 63 - __builtin_clzll(w), lo = __builtin_ctzll(w);
    const uint64_t rest = w & ~(1ull << hi);
    const uint64_t s1 = w >> a, s2 = plus1 ? (s1 >> 1) : 0ull;
    const int32_t n1 = __builtin_popcountll(w & s1);
    const int32_t sum = plus1 ? mul_small(c - 1, a + 1) - n1 : mul_small(c - 1, a);
    return !(rest & ~(s1 | s2)) && sum == hi - lo;
}

constexpr int kFastMaxGap = 62;  // word-level shortcut for intervals up to this

// mask ? a : b, bit by bit (mask all ones or all zeros)
__device__ __forceinline__ int32_t bsel(uint32_t mask, int32_t a, int32_t b)
{
    return (int32_t)__builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, mask, 0xE4);
}

// Segmentation state of one pixel (registers).
struct SegState {
    int32_t flo, fhi;  // extremes of the open FSR segment's S1 values
    // SSR: intervals are numbered by ii (running count); the open piece
    // starts at interval ps.  Per interval value (keyed by parity: an FSR
    // segment holds at most two adjacent values) the number of its latest
    // occurrence -- meaningful only when >= ps, so a cut needs no clearing --
    // and the extremes of its S2 gaps inside the piece (reset at the value's
    // first occurrence in a piece, hence valid whenever the occurrence is).
    int32_t ii, ps;
    int32_t l0, l1, g0l, g0h, g1l, g1h;
    // Third order (ORDER 4): the open sub-piece starts at interval p3 (>= ps).
    // S2 elements of each interval value are numbered by c2* (running), and
    // b2* is that count at the value's first occurrence in the sub-piece.
    // Per (value parity, S2-value parity) slot k = 2*odd + dodd: the number
    // of the latest S2 element with that value (meaningful when >= b2 of the
    // value) and the extremes of the S3 gaps between such elements.
    int32_t p3, c20, c21, b20, b21;
    int32_t m0, m1, m2, m3, hl0, hl1, hl2, hl3, hh0, hh1, hh2, hh3;

    __device__ __forceinline__ void reset()
    {
        flo = kBig;
        fhi = -kBig;
        ii = ps = 0;
        l0 = l1 = -1;
        g0l = g1l = kBig;
        g0h = g1h = -kBig;
        p3 = c20 = c21 = b20 = b21 = 0;
        m0 = m1 = m2 = m3 = -1;
        hl0 = hl1 = hl2 = hl3 = kBig;
        hh0 = hh1 = hh2 = hh3 = -kBig;
    }

    // Whole-word shortcut: if none of the word's intervals -- x0 (from the
    // previous word's last spike to the word's first spike) and the gaps
    // inside the nonzero word w, c spikes in all -- opens a new segment,
    // apply them all and return true; otherwise change nothing and return
    // false.  FSR: all intervals in [flo, flo + 1] keep the segment stable.
    // SSR: words whose intervals take the values flo and flo + 1 (see
    // two_values), or all equal one value just below a single-valued
    // segment.  TFI has no shortcut.
    template <int ORDER>
    __device__ __forceinline__ bool fast_word(uint64_t w, int32_t x0, int32_t c)
    {
        if constexpr (ORDER == 3 || ORDER == 4) {
            return false;  // TFI: every interval is cut; third order: no shortcut
        } else if constexpr (ORDER == 1) {
            const int32_t a = flo;
            if (a < 1 || a > kFastMaxGap || x0 < a || x0 > a + 1) return false;
            if (!gaps_within(w, a, true, c)) return false;
            // a gap of a + 1 somewhere (the others are exactly a)
            const bool wide = x0 == a + 1 || popc64(w & (w >> a)) < c - 1;
            fhi = max(fhi, wide ? a + 1 : a);
            return true;
        } else {
            const int32_t v = x0;
            if (v >= flo) {
                // the two-value walk pays off only when most of the wave can
                // take it (a lane left on the spike path keeps the others
                // waiting): vote on its cheap preconditions first
                const int32_t a = flo;
                const bool pre = a >= 1 && a <= kFastMaxGap && fhi <= a + 1 && x0 <= a + 1 &&
                                 gaps_within(w, a, true, c);
                if (popc64(__ballot(pre)) * 4 < popc64(__ballot(1)) * 3) return false;
                return pre && two_values(w, x0, c);
            }
            if (v < 1 || fhi - v > 1) return false;
            // the word opens with a value below the segment's single value:
            // only words of that one value (all S2 gaps inside are 1)
            if (v > kFastMaxGap) return false;
            if (c > 1 && !gaps_within(w, v, false, c)) return false;
            const bool odd = v & 1;
            const int32_t l = odd ? l1 : l0;
            int32_t gl = kBig, gh = -kBig;
            if (l >= ps) {
                gl = min(odd ? g1l : g0l, ii - l);
                gh = max(odd ? g1h : g0h, ii - l);
            }
            if (c > 1) {
                gl = min(gl, 1);
                gh = max(gh, 1);
            }
            if (gh - gl > 1) return false;
            flo = min(flo, v);
            fhi = max(fhi, v);
            // selects rather than stores through a chosen member, which
            // would force the state out of registers
            const int32_t last = ii + c - 1;
            l0 = odd ? l0 : last;
            l1 = odd ? last : l1;
            g0l = odd ? g0l : gl;
            g0h = odd ? g0h : gh;
            g1l = odd ? gl : g1l;
            g1h = odd ? gh : g1h;
            ii += c;
            return true;
        }
    }

    // SSR shortcut for a word whose intervals take the values a = flo and
    // a + 1 (no FSR cut; one of them may be absent), called A and B.  When
    // one value never occurs twice in a row (it is "isolated"; a
    // constant-rate pixel always has one, Lemma 2), every S2 gap of the
    // other value is 1 or 2, so only the
    // isolated value's gaps need a walk -- over its own occurrences, from
    // the frame distances between them (k intervals apart means k*a + 1
    // frames for an isolated B, k*(a+1) - 1 for an isolated A).  All new
    // gaps of both values must keep each value's S2 span within 1 together
    // with the piece's gaps so far; then nothing is cut and the state
    // advances by the whole word.  Otherwise nothing changes (false).
    // Precondition: 1 <= a <= kFastMaxGap, fhi <= a + 1, x0 in {a, a + 1} and
    // every gap inside w is a or a + 1.
    __device__ __forceinline__ bool two_values(uint64_t w, int32_t x0, int32_t c)
    {
        const int32_t a = flo;
        const uint64_t f = w & (~w + 1);             // the word's first spike
        const uint64_t top = 1ull << hibit64(w);     // and its last
        // spikes whose interval is B: every gap inside w is a or a + 1, so
        // those whose predecessor is not a frames back
        uint64_t MB = w & ~(w << a) & ~f;
        if (x0 == a + 1) MB |= f;
        const uint64_t MA = w & ~MB;
        const bool oddA = a & 1;
        const int32_t lA = oddA ? l1 : l0, lB = oddA ? l0 : l1;
        const bool seenA = lA >= ps, seenB = lB >= ps;
        // two B (or two A) in a row, inside the word or across its start
        // (bitwise operators: lane masks, not values)
        const bool BB = ((MB & (MB << (a + 1))) != 0) | (seenB & (lB == ii - 1) & (x0 == a + 1));
        const bool AA = ((MA & (MA << a)) != 0) | (seenA & (lA == ii - 1) & (x0 == a));
        if (BB & AA) return false;
        const bool isoB = !BB;  // the walked (isolated) value is B, else A
        const uint64_t MM = isoB ? MB : MA, MJ = isoB ? MA : MB;
        const int32_t xM = isoB ? a + 1 : a, xJ = isoB ? a : a + 1;
        const int32_t lM = isoB ? lB : lA, lJ = isoB ? lA : lB;
        const bool seenM = isoB ? seenB : seenA, seenJ = isoB ? seenA : seenB;
        const bool oddM = isoB ^ oddA;
        int32_t gMl = oddM ? g1l : g0l, gMh = oddM ? g1h : g0h;
        int32_t gJl = oddM ? g0l : g1l, gJh = oddM ? g0h : g1h;
        if (!seenM) { gMl = kBig; gMh = -kBig; }
        if (!seenJ) { gJl = kBig; gJh = -kBig; }
        int32_t nlM = lM, nlJ = lJ;
        // the other value: gaps 1 (twice in a row) and 2 (around one isolated
        // occurrence) inside the word, and the gap back to its last
        // occurrence.  The isolated value never occurs twice in a row, so at
        // most one of its occurrences precedes the other's first one or
        // follows its last: their interval numbers need no popcount.
        if (MJ) {
            const int32_t first = ii + ((f & MM) != 0);
            if (seenJ) {
                gJl = min(gJl, first - lJ);
                gJh = max(gJh, first - lJ);
            }
            if (MJ & (MJ << xJ)) {
                gJl = min(gJl, 1);
                gJh = max(gJh, 1);
            }
            if (xJ + xM < 64 && (MJ & (MM << xJ) & (MJ << (xJ + xM)))) {
                gJl = min(gJl, 2);
                gJh = max(gJh, 2);
            }
            nlJ = ii + c - 1 - ((top & MM) != 0);
        }
        if (gJh - gJl > 1) return false;
        // the isolated value: a gap of k intervals between two of its
        // occurrences is k*xJ + (xM - xJ) frames.  Its n occurrences in the
        // word have n - 1 gaps summing to K (the difference of their interval
        // numbers); the gaps have span <= 1 only if they lie in {g, g + 1}
        // with g = floor(K / (n - 1)).  Send each occurrence but the last to
        // the nearer of the occurrences g and g + 1 intervals later (one must
        // exist); that gap is at least the true one, and the counts n1, n2 of
        // each choice give n1*g + n2*(g + 1) >= K, equal exactly when every
        // true gap is g or g + 1.  No walk over the occurrences is needed.
        if (MM) {
            const uint64_t fM = MM & (~MM + 1);
            const int32_t first = ii + popc64(w & (fM - 1));
            const int hM = hibit64(MM);
            const int32_t lastM = ii + popc64(w & ((1ull << hM) - 1));
            if (seenM) {
                gMl = min(gMl, first - lM);
                gMh = max(gMh, first - lM);
            }
            const int32_t n = popc64(MM);
            if (n >= 2) {
                const int32_t K = lastM - first;
                // K / (n - 1) with K <= 63: the fraction is a multiple of
                // 1/(n - 1) >= 1/31, far above the reciprocal's error
                const int32_t g = (int32_t)fmaf((float)K, __builtin_amdgcn_rcpf((float)(n - 1)),
                                                1e-3f);
                const int32_t D1 = mul_small(g, xJ) + (xM - xJ), D2 = D1 + xJ;
                const uint64_t s1 = D1 < 64 ? MM >> D1 : 0ull, s2 = D2 < 64 ? MM >> D2 : 0ull;
                const uint64_t rest = MM & ~(1ull << hM);
                if (rest & ~(s1 | s2)) return false;
                const int32_t n1 = popc64(rest & s1), n2 = n - 1 - n1;
                if (mul_small(n1, g) + mul_small(n2, g + 1) != K) return false;
                if (n1) {
                    gMl = min(gMl, g);
                    gMh = max(gMh, g);
                }
                if (n2) {
                    gMl = min(gMl, g + 1);
                    gMh = max(gMh, g + 1);
                }
            }
            nlM = lastM;
        }
        if (gMh - gMl > 1) return false;
        fhi = max(fhi, MB ? a + 1 : a);
        // the isolated value's state goes to its parity's slot
        l0 = oddM ? nlJ : nlM;
        l1 = oddM ? nlM : nlJ;
        g0l = oddM ? gJl : gMl;
        g0h = oddM ? gJh : gMh;
        g1l = oddM ? gMl : gJl;
        g1h = oddM ? gMh : gJh;
        ii += c;
        return true;
    }

    // Add interval x; returns true if x opens a new segment (the previous
    // spike then ends the closed one).  Written as selects so that the wave
    // runs one straight path whatever each lane decides.
    template <int ORDER>
    __device__ __forceinline__ bool step(int32_t x)
    {
        if constexpr (ORDER == 3) {
            // TFI (Sec. II): every interval after the first opens a segment
            const bool cut = flo != kBig;
            flo = fhi = x;
            return cut;
        }
        const int32_t nlo = min(flo, x), nhi = max(fhi, x);
        const bool fcut = nhi - nlo > 1;  // S1 leaves zero-order stability
        flo = fcut ? x : nlo;
        fhi = fcut ? x : nhi;
        if constexpr (ORDER == 1) {
            return fcut;
        } else {
            // the per-value state is selected by x's parity through a mask
            // (all ones for odd x) and bitwise selects: one instruction for
            // the mask, written out so that the compiler does not turn the
            // selects back into a parity test and lane-mask selects
            uint32_t mo;
            asm("v_bfe_i32 %0, %1, 0, 1" : "=v"(mo) : "v"(x));
            const int32_t l = bsel(mo, l1, l0);
            const int32_t d = ii - l;  // next element of S2 for value x
            const int32_t ngl = min(bsel(mo, g1l, g0l), d), ngh = max(bsel(mo, g1h, g0h), d);
            const bool seen = l >= ps;  // x already occurred in the open piece
            const bool cut = fcut || (seen && ngh - ngl > 1);
            const bool keep = seen && !cut;  // the value's gaps continue
            const int32_t ugl = keep ? ngl : kBig, ugh = keep ? ngh : -kBig;
            l0 = bsel(mo, l0, ii);
            l1 = bsel(mo, ii, l1);
            g0l = bsel(mo, g0l, ugl);
            g0h = bsel(mo, g0h, ugh);
            g1l = bsel(mo, ugl, g1l);
            g1h = bsel(mo, ugh, g1h);
            ps = cut ? ii : ps;
            if constexpr (ORDER == 4) {
                // third order: d is the new element of S2(x) if x occurred in
                // the open sub-piece; its S3 gap is the distance (in S2
                // elements) back to the latest element of the same value
                const bool odd = mo != 0u;
                const bool seen3 = l >= p3;
                const bool dodd = d & 1;
                const int32_t c2 = odd ? c21 : c20, b2 = odd ? b21 : b20;
                // bitwise selects on the values: a ?: over the members
                // becomes a load through a selected address, which keeps
                // the whole state in scratch memory
                const uint32_t md = 0u - (uint32_t)dodd;
                const int32_t m = bsel(mo, bsel(md, m3, m2), bsel(md, m1, m0));
                const int32_t hl = bsel(mo, bsel(md, hl3, hl2), bsel(md, hl1, hl0));
                const int32_t hh = bsel(mo, bsel(md, hh3, hh2), bsel(md, hh1, hh0));
                const bool mvalid = seen3 && m >= b2;
                const int32_t e = c2 - m;
                const int32_t nl3 = min(hl, e), nh3 = max(hh, e);
                const bool cut3 = cut || (mvalid && nh3 - nl3 > 1);
                const bool rec = seen3 && !cut3;  // an S2 element inside the sub-piece
                const int32_t ul = mvalid ? nl3 : kBig, uh = mvalid ? nh3 : -kBig;
                const bool w0 = rec && !odd && !dodd, w1 = rec && !odd && dodd;
                const bool w2 = rec && odd && !dodd, w3 = rec && odd && dodd;
                m0 = w0 ? c2 : m0;
                m1 = w1 ? c2 : m1;
                m2 = w2 ? c2 : m2;
                m3 = w3 ? c2 : m3;
                hl0 = w0 ? ul : hl0;
                hl1 = w1 ? ul : hl1;
                hl2 = w2 ? ul : hl2;
                hl3 = w3 ? ul : hl3;
                hh0 = w0 ? uh : hh0;
                hh1 = w1 ? uh : hh1;
                hh2 = w2 ? uh : hh2;
                hh3 = w3 ? uh : hh3;
                const int32_t nc2 = c2 + (rec ? 1 : 0);
                const int32_t nb2 = (!seen3 || cut3) ? c2 : b2;
                c20 = odd ? c20 : nc2;
                c21 = odd ? nc2 : c21;
                b20 = odd ? b20 : nb2;
                b21 = odd ? nb2 : b21;
                p3 = cut3 ? ii : p3;
                ii++;
                return cut3;
            }
            ii++;
            return cut;
        }
    }
};

// Eq. 6 value theta * n / d, computed in double and rounded once to float.
// The quotient takes the steps of the compiler's IEEE double division --
// reciprocal, two Newton-Raphson refinements, the quotient, its residual by
// fma and one correction (Markstein) -- without the exponent scaling and the
// special-case fix-up around them, which only act on operands near the
// exponent limits or non-finite ones.  Here 0 < theta * n < 2^160 and
// 1 <= d < 2^31, so the value is theta * n / d exactly as that division
// gives it (the correctly rounded quotient).
__device__ __forceinline__ float intensity(double theta, int32_t n, int32_t d)
{
    const double x = theta * (double)n, dd = (double)d;
    double y = __builtin_amdgcn_rcp(dd);
    double e = __builtin_fma(-dd, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-dd, y, 1.0);
    y = __builtin_fma(y, e, y);
    const double q = x * y;
    const double r = __builtin_fma(-dd, q, x);
    return (float)__builtin_fma(r, y, q);
}

// How output k (in time order) maps to its plane: identity, through an LDS
// copy of the map, or through the map in global memory (very large maps).
enum PlaneMap { PMAP_IDENT = 0, PMAP_LDS = 1, PMAP_GLOBAL = 2 };

// Writes of one pixel's closed segments.
template <int MODE, bool WIN, int PMAP>
struct Emitter {
    static constexpr int kMode = MODE;
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
        else return gp(P.plane)[k];
    }

    // A closed segment spanning spike frames [first, last] with n intervals
    // covers sorted outputs [k0, kend).
    __device__ __forceinline__ void close(int32_t first, int32_t last, int32_t n, int32_t k0,
                                          int32_t kend)
    {
        if (!valid) return;
        if constexpr (MODE == MODE_SEGMENTS) {
            if (segc < P.cap) {
                if (P.seg_rec) {
                    // a pixel's records one after another: its lane fills
                    // its own lines, which merge in L2 before write-back
                    auto r = gp(P.seg_rec) + ((int64_t)p * P.cap + segc) * 3;
                    r[0] = first;
                    r[1] = last;
                    r[2] = n;
                } else {
                    const int64_t o = (int64_t)segc * P.HW + p;
                    gp(P.seg_first)[o] = first;
                    gp(P.seg_last)[o] = last;
                    gp(P.seg_n)[o] = n;
                }
            }
            segc++;
        } else if constexpr (MODE == MODE_MOTION) {
            k0 = max(k0, kmin);
            if (k0 >= kend) return;
            // 1 where the segment is not the pixel's first and t < first +
            // window: t sorted, so the outputs before kc
            const uint8_t not_first = first != gp(P.first_spike)[p];
            const int64_t tl = (int64_t)first + P.window - 1;
            const int32_t kc = tl >= P.T - 1 ? P.n_out : gp(P.cnt_le)[tl];
            for (int32_t k = k0; k < kend; k++) {
                const int64_t o = (int64_t)(uint64_t)(uint32_t)plane(k) * (uint32_t)P.HW + p;
                gp(P.mask)[o] = k < kc ? not_first : (uint8_t)0;
            }
        } else {
            k0 = max(k0, kmin);
            if (k0 >= kend) return;
            // Eq. 6: theta / ((1/N) sum T0(i)); the N intervals sum to last - first
            const float I = intensity(P.theta, n, last - first);
            if constexpr (PMAP == PMAP_IDENT && !WIN) {
                // planes in time order: step a pointer by one plane per output
                auto q = gp(P.out) + p + (uint64_t)(uint32_t)k0 * (uint32_t)P.HW;
                for (int32_t k = k0; k < kend; k++, q += (uint32_t)P.HW) *q = I;
                return;
            }
            for (int32_t k = k0; k < kend; k++) {
                const int64_t o = (int64_t)(uint64_t)(uint32_t)plane(k) * (uint32_t)P.HW + p;
                if constexpr (WIN) {
                    if (P.out) gp(P.out)[o] = I;
                    if (P.win_first) gp(P.win_first)[o] = first;
                    if (P.win_last) gp(P.win_last)[o] = last;
                    if (P.win_n) gp(P.win_n)[o] = n;
                } else {
                    gp(P.out)[o] = I;
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
            if constexpr (MODE == MODE_MOTION) {
                gp(P.mask)[o] = 0;
            } else if constexpr (WIN) {
                if (P.out) gp(P.out)[o] = 0.0f;
                if (P.win_first) gp(P.win_first)[o] = -1;
                if (P.win_last) gp(P.win_last)[o] = -1;
                if (P.win_n) gp(P.win_n)[o] = 0;
            } else {
                gp(P.out)[o] = 0.0f;
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

    // Whole-word shortcut (SegState::fast_word) for the nonzero word w
    // starting at frame t0: true when no segment ends in it, the run then
    // being advanced past it.
    template <int ORDER>
    __device__ __forceinline__ bool try_fast(int32_t t0, uint64_t w, const int32_t *cnt_row)
    {
        if (lastspk < 0) return false;
        const int32_t c = popc64(w);
        if (!st.template fast_word<ORDER>(w, t0 + ctz64(w) - lastspk, c)) return false;
        cum += c;
        const int hp = hibit64(w);
        lastspk = t0 + hp;
        cnt_last = cnt_row[hp];
        return true;
    }

    // What the closing of a word needs from its start.
    struct WordStart {
        uint64_t wfull;   // the word
        uint64_t rest;    // its spikes that end an interval
        int32_t cum0, lastspk0, cnt_last0;
        int32_t lp;       // previous spike, relative to t0
    };

    // Start of the spike walk over the nonzero word w: a pixel's first spike
    // opens its first segment and ends no interval.
    __device__ __forceinline__ WordStart begin(int32_t t0, uint64_t w)
    {
        WordStart ws{w, w, cum, lastspk, cnt_last, 0};
        if (lastspk < 0) {
            const int pos = ctz64(w);
            ws.rest = w & (w - 1);
            first = t0 + pos;
            first_idx = 0;
            ws.lp = pos;
        } else {
            ws.lp = lastspk - t0;
        }
        return ws;
    }

    // Walk the spikes of rest (the intervals from lp on) through the state
    // machine, one 32-bit half at a time; returns the mask of spikes whose
    // interval opens a new segment.
    template <int ORDER, bool CAPTURE>
    __device__ __forceinline__ uint64_t spikes(int32_t t0, uint64_t rest, int32_t lp)
    {
        // The lowest spike's bit comes from its position and is cleared
        // from h in place.  The clearing is one VALU instruction written
        // out, because the compiler otherwise tests the loop's exit as
        // bit == h on the old value, which keeps both alive and costs a
        // register copy per spike.
        uint32_t Blo = 0, Bhi = 0;
        uint32_t h = (uint32_t)rest;
        while (h) {
            const int pos = __builtin_ctz(h);
            const uint32_t bit = 1u << pos;
            const int32_t x = pos - lp;  // interval T0 ending at this spike
            lp = pos;
            Blo |= step_capture<ORDER, CAPTURE>(x, t0 + pos) ? bit : 0u;
            asm("v_xor_b32 %0, %1, %0" : "+v"(h) : "v"(bit));
        }
        h = (uint32_t)(rest >> 32);
        while (h) {
            const int pos = __builtin_ctz(h);
            const uint32_t bit = 1u << pos;
            const int32_t x = pos + 32 - lp;
            lp = pos + 32;
            Bhi |= step_capture<ORDER, CAPTURE>(x, t0 + 32 + pos) ? bit : 0u;
            asm("v_xor_b32 %0, %1, %0" : "+v"(h) : "v"(bit));
        }
        return ((uint64_t)Bhi << 32) | Blo;
    }

    // Close the segments that ended in the word (B0: the spikes whose
    // interval opened a new one) and advance the run past it.
    // FB1: keep fb1/fn1/fi1 (chunked runs only).
    template <bool FB1, class EM>
    __device__ __forceinline__ void finish(int32_t t0, const WordStart &ws, uint64_t B0,
                                           const int32_t *cnt_row, EM &em)
    {
        // chunked runs keep the first segment closed at or after the chunk's
        // start (for the fixup pass); once every lane that closes a segment
        // in this word has it, the loop runs without that bookkeeping
        auto closes = [&](auto fb1_pending) {
            uint64_t B = B0;
            while (B) {
                const int cpos = ctz64(B);
                B &= B - 1;
                const uint64_t below = ws.wfull & ((1ull << cpos) - 1);
                int32_t last, kend;
                if (below) {
                    const int bp = hibit64(below);
                    last = t0 + bp;
                    kend = cnt_row[bp];
                } else {
                    last = ws.lastspk0;
                    kend = ws.cnt_last0;
                }
                const int32_t last_idx = ws.cum0 + popc64(below) - 1;
                em.close(first, last, last_idx - first_idx, k0, kend);
                if constexpr (decltype(fb1_pending)::value) {
                    if (fb1 < 0 && last >= cs) {
                        fb1 = last;
                        fn1 = last_idx - first_idx;
                        fi1 = last_idx;
                    }
                }
                first = last;
                first_idx = last_idx;
                k0 = kend;
            }
        };
        if (FB1 && __ballot(fb1 < 0 && B0 != 0))
            closes(std::true_type{});
        else
            closes(std::false_type{});
        if (B0) lastb = first;  // the last closed segment's last spike
        cum = ws.cum0 + popc64(ws.wfull);
        const int hp = hibit64(ws.wfull);
        lastspk = t0 + hp;
        cnt_last = cnt_row[hp];
    }

    // TFI (every interval but a pixel's first opens a segment) over the
    // nonzero word w, for outputs at t_out (intensities, windows or the
    // motion mask; not segment lists).  The spike walk would close a
    // segment at nearly every spike, and most of them cover no output.  Here
    // only the segments that cover an output are emitted, with the same
    // arguments as the walk gives them: at most two at the word's start,
    // whose outputs may lie in earlier words, then one per distinct next
    // spike of the output frames in omask (bit j: an output at frame t0 + j,
    // j >= 1).  The run's state then advances past the word as the walk
    // leaves it.  A segment the walk closes and this skips has k0 == kend,
    // so it writes nothing.
    template <class EM>
    __device__ __forceinline__ void word_tfi(int32_t t0, uint64_t w, const int32_t *cnt_row,
                                             uint64_t omask, EM &em)
    {
        const int32_t c = popc64(w);
        const int p1 = ctz64(w), hp = hibit64(w);
        // second and second-to-last spikes when c >= 2 (the extra bit only
        // keeps the count defined for c = 1)
        const int p2 = ctz64((w & (w - 1)) | (1ull << 63));
        const int pl = hibit64((w & ~(1ull << hp)) | 1ull);
        const bool had = lastspk >= 0;
        const int32_t cum0 = cum, lastspk0 = lastspk, cnt_last0 = cnt_last;
        // the word's spikes are numbered 1..c, spike 0 being lastspk; the
        // first one that closes a segment: spike 1, unless the interval it
        // ends is the pixel's first (or it is the pixel's first spike)
        const int i_min = (had ? 1 : 2) + (st.flo == kBig ? 1 : 0);
        if (!had) {
            first = t0 + p1;
            first_idx = 0;
        }
        if (i_min <= c) {
            // the first close: its last spike is spike i_min - 1, and it
            // takes every output from k0 on
            int32_t L, kend;
            if (i_min == 1) {
                L = lastspk0;
                kend = cnt_last0;
            } else {
                const int q = i_min == 2 ? p1 : p2;
                L = t0 + q;
                kend = cnt_row[q];
            }
            const int32_t lidx = cum0 + i_min - 2;
            em.close(first, L, lidx - first_idx, k0, kend);
            // the second, when it ends at spike 1 after lastspk: its outputs
            // may lie before the word
            if (i_min == 1 && c >= 2)
                em.close(lastspk0, t0 + p1, 1, cnt_last0, cnt_row[p1]);
        }
        // later closes end at spikes past lo (spike 1, or 2 when the first
        // close ended there) and before the word's last spike; their outputs
        // lie inside the word
        const int lo = i_min == 3 ? p2 : p1;
        int nx_done = -1;
        uint64_t om = omask;
        while (om) {
            const int o = ctz64(om);
            om &= om - 1;
            // the first spike at or after frame t0 + o (63 when there is none,
            // which the test against hp rejects)
            const int nx = ctz64((w & (~0ull << o)) | (1ull << 63));
            if (nx > lo && nx < hp && nx != nx_done) {
                nx_done = nx;
                const int pv = hibit64(w & ((1ull << nx) - 1));
                em.close(t0 + pv, t0 + nx, 1, cnt_row[pv], cnt_row[nx]);
            }
        }
        // the state the walk leaves
        if (i_min <= c) {
            // the last close ends at spike c - 1
            if (c == 1) {
                first = lastspk0;
                first_idx = cum0 - 1;
                k0 = cnt_last0;
            } else {
                first = t0 + pl;
                first_idx = cum0 + c - 2;
                k0 = cnt_row[pl];
            }
            lastb = first;
        }
        if (c >= 2 || had) {
            const int32_t x = c >= 2 ? hp - pl : t0 + p1 - lastspk0;  // the last interval
            st.flo = x;
            st.fhi = x;
        }
        cum = cum0 + c;
        lastspk = t0 + hp;
        cnt_last = cnt_row[hp];
    }

    // Process the 64-frame word w starting at frame t0; cnt_row[j] is the
    // number of sorted outputs at or before frame t0 + j (omask: the output
    // frames of the word, for TFI with outputs at t_out).
    // FB1: keep fb1/fn1/fi1 (chunked runs only).
    template <int ORDER, bool CAPTURE, bool FB1, class EM>
    __device__ __forceinline__ void word(int32_t t0, uint64_t w, const int32_t *cnt_row, EM &em,
                                         uint64_t omask = 0)
    {
        if constexpr (ORDER == 3 && EM::kMode != MODE_SEGMENTS) {
            // a chunked run keeps its first close at or after the chunk's
            // start for the fixup pass: the walk below does that bookkeeping
            // in the words that may hold it
            if (!(FB1 && fb1 < 0 && t0 + 63 >= cs)) {
                word_tfi(t0, w, cnt_row, omask, em);
                return;
            }
        }
        if (try_fast<ORDER>(t0, w, cnt_row)) return;  // no segment ends in this word
        const WordStart ws = begin(t0, w);
        const uint64_t B0 = spikes<ORDER, CAPTURE>(t0, ws.rest, ws.lp);
        finish<FB1>(t0, ws, B0, cnt_row, em);
    }
};

// Per-chunk record of the running state at the chunk's end, [field][chunk][pixel].
// FSR and TFI runs keep the fields up to R_NFSR, SSR runs all but the FSR
// capture up to R_NSSR, third-order runs all but the capture.
enum RecField {
    R_LASTSPK, R_CNTLAST, R_CUM, R_FIRST, R_FIRSTIDX, R_K0, R_LASTB, R_FB1, R_FN1,
    R_FI1, R_FLO, R_FHI, R_FWLO, R_FWHI, R_NFSR = R_FWHI + 1,
    R_II = R_FWLO, R_PS, R_L0, R_L1, R_G0L, R_G0H, R_G1L, R_G1H, R_NSSR,
    R_P3 = R_NSSR, R_C20, R_C21, R_B20, R_B21, R_M0, R_M1, R_M2, R_M3, R_HL0, R_HL1, R_HL2,
    R_HL3, R_HH0, R_HH1, R_HH2, R_HH3, R_NFIELDS
};
static_assert(R_NFIELDS <= kRecFields, "record layout");

// Fields a run of the given order keeps in its records.
__host__ __device__ constexpr int rec_fields_of(int order)
{
    return order == 2 ? (int)R_NSSR : (order == 4 ? (int)R_NFIELDS : (int)R_NFSR);
}

// Records of chunk c: the state at the chunk's end (all chunks) and the
// warmed-up speculative state at its start (chunks > 0), each [field][chunk][HW].
__device__ __forceinline__ int32_t *rec_end(const ChunkPlan &cp, int c, int64_t p, int32_t HW)
{
    return cp.rec + (int64_t)c * HW + p;
}
__device__ __forceinline__ int32_t *rec_start(const ChunkPlan &cp, int c, int64_t p, int32_t HW)
{
    return cp.rec + (int64_t)cp.fields * cp.nchunks * HW + (int64_t)c * HW + p;
}

template <int ORDER>
__device__ __forceinline__ void save_run(int32_t *rec_, int64_t stride, const Run &r)
{
    const auto rec = gp(rec_);
    rec[R_LASTSPK * stride] = r.lastspk;
    rec[R_CNTLAST * stride] = r.cnt_last;
    rec[R_CUM * stride] = r.cum;
    rec[R_FIRST * stride] = r.first;
    rec[R_FIRSTIDX * stride] = r.first_idx;
    rec[R_K0 * stride] = r.k0;
    rec[R_LASTB * stride] = r.lastb;
    rec[R_FB1 * stride] = r.fb1;
    rec[R_FN1 * stride] = r.fn1;
    rec[R_FI1 * stride] = r.fi1;
    rec[R_FLO * stride] = r.st.flo;
    rec[R_FHI * stride] = r.st.fhi;
    if constexpr (ORDER == 4) {
        const int32_t v[R_NFIELDS - R_P3] = {r.st.p3, r.st.c20, r.st.c21, r.st.b20, r.st.b21,
                                             r.st.m0, r.st.m1, r.st.m2, r.st.m3, r.st.hl0,
                                             r.st.hl1, r.st.hl2, r.st.hl3, r.st.hh0, r.st.hh1,
                                             r.st.hh2, r.st.hh3};
#pragma unroll
        for (int f = 0; f < R_NFIELDS - R_P3; f++) rec[(R_P3 + f) * stride] = v[f];
    }
    if constexpr (ORDER != 2 && ORDER != 4) {
        rec[R_FWLO * stride] = r.fwlo;
        rec[R_FWHI * stride] = r.fwhi;
    } else {
        rec[R_II * stride] = r.st.ii;
        rec[R_PS * stride] = r.st.ps;
        rec[R_L0 * stride] = r.st.l0;
        rec[R_L1 * stride] = r.st.l1;
        rec[R_G0L * stride] = r.st.g0l;
        rec[R_G0H * stride] = r.st.g0h;
        rec[R_G1L * stride] = r.st.g1l;
        rec[R_G1H * stride] = r.st.g1h;
    }
}

template <int ORDER>
__device__ __forceinline__ void load_run(const int32_t *rec_, int64_t stride, Run &r)
{
    const auto rec = gp(rec_);
    r.reset(0);
    r.lastspk = rec[R_LASTSPK * stride];
    r.cnt_last = rec[R_CNTLAST * stride];
    r.cum = rec[R_CUM * stride];
    r.first = rec[R_FIRST * stride];
    r.first_idx = rec[R_FIRSTIDX * stride];
    r.k0 = rec[R_K0 * stride];
    r.lastb = rec[R_LASTB * stride];
    r.fb1 = rec[R_FB1 * stride];
    r.fn1 = rec[R_FN1 * stride];
    r.fi1 = rec[R_FI1 * stride];
    r.st.flo = rec[R_FLO * stride];
    r.st.fhi = rec[R_FHI * stride];
    if constexpr (ORDER == 4) {
        int32_t v[R_NFIELDS - R_P3];
#pragma unroll
        for (int f = 0; f < R_NFIELDS - R_P3; f++) v[f] = rec[(R_P3 + f) * stride];
        r.st.p3 = v[0];
        r.st.c20 = v[1];
        r.st.c21 = v[2];
        r.st.b20 = v[3];
        r.st.b21 = v[4];
        r.st.m0 = v[5];
        r.st.m1 = v[6];
        r.st.m2 = v[7];
        r.st.m3 = v[8];
        r.st.hl0 = v[9];
        r.st.hl1 = v[10];
        r.st.hl2 = v[11];
        r.st.hl3 = v[12];
        r.st.hh0 = v[13];
        r.st.hh1 = v[14];
        r.st.hh2 = v[15];
        r.st.hh3 = v[16];
    }
    if constexpr (ORDER != 2 && ORDER != 4) {
        r.fwlo = rec[R_FWLO * stride];
        r.fwhi = rec[R_FWHI * stride];
    } else {
        r.st.ii = rec[R_II * stride];
        r.st.ps = rec[R_PS * stride];
        r.st.l0 = rec[R_L0 * stride];
        r.st.l1 = rec[R_L1 * stride];
        r.st.g0l = rec[R_G0L * stride];
        r.st.g0h = rec[R_G0H * stride];
        r.st.g1l = rec[R_G1L * stride];
        r.st.g1h = rec[R_G1H * stride];
    }
}

// Two states make the same cut decisions for every continuation when their
// FSR extremes agree and, for SSR, the same values occurred in the open
// piece, at the same distance back, with the same S2 gap extremes (interval
// numbers of the two runs differ by a constant shift, which no decision sees).
template <int ORDER>
__device__ __forceinline__ bool same_decisions(const SegState &a, const SegState &b)
{
    if constexpr (ORDER == 3) return (a.flo == kBig) == (b.flo == kBig);  // TFI
    if (a.flo != b.flo || a.fhi != b.fhi) return false;
    if constexpr (ORDER == 1) {
        return true;
    } else {
        const bool a0 = a.l0 >= a.ps, b0 = b.l0 >= b.ps, a1 = a.l1 >= a.ps, b1 = b.l1 >= b.ps;
        if (a0 != b0 || a1 != b1) return false;
        if (a0 && (a.ii - a.l0 != b.ii - b.l0 || a.g0l != b.g0l || a.g0h != b.g0h))
            return false;
        if (a1 && (a.ii - a.l1 != b.ii - b.l1 || a.g1l != b.g1l || a.g1h != b.g1h))
            return false;
        if constexpr (ORDER == 4) {
            // third order: the same values seen in the sub-piece and, per
            // S2-value slot, the same validity, distance back and S3 extremes
            if ((a.l0 >= a.p3) != (b.l0 >= b.p3) || (a.l1 >= a.p3) != (b.l1 >= b.p3))
                return false;
            auto slot = [](int32_t am, int32_t ab, int32_t ac, int32_t ahl, int32_t ahh,
                           int32_t bm, int32_t bb, int32_t bc, int32_t bhl, int32_t bhh) {
                const bool av = am >= ab, bv = bm >= bb;
                return av == bv && (!av || (ac - am == bc - bm && ahl == bhl && ahh == bhh));
            };
            if (a.l0 >= a.p3 &&
                !(slot(a.m0, a.b20, a.c20, a.hl0, a.hh0, b.m0, b.b20, b.c20, b.hl0, b.hh0) &&
                  slot(a.m1, a.b20, a.c20, a.hl1, a.hh1, b.m1, b.b20, b.c20, b.hl1, b.hh1)))
                return false;
            if (a.l1 >= a.p3 &&
                !(slot(a.m2, a.b21, a.c21, a.hl2, a.hh2, b.m2, b.b21, b.c21, b.hl2, b.hh2) &&
                  slot(a.m3, a.b21, a.c21, a.hl3, a.hh3, b.m3, b.b21, b.c21, b.hl3, b.hh3)))
                return false;
        }
        return true;
    }
}


// One wave walks tiles [tilew, tile1) of its 64-pixel strip starting at
// p0, prefetching a group of tiles ahead.  Row r of the stream at base (and
// of P.cnt_le) is frame f0 + r.  In a chunked run (CHUNKED) the tiles
// before tile0 only warm the state up, the state at tile0 is saved to
// rec_start, and the first tiles after tile0 keep what the fixup pass needs.
// KG tiles per prefetch group.  The LDS rows (word_s, cnt_s: KG x 64) are
// the wave's own; WAVE_SYNC orders their writes and reads with wave-scope
// fences instead of a workgroup barrier, for workgroups of several waves
// that each walk their own strips (a wave's LDS accesses complete in
// order, so a compiler fence is all a lane needs to see its neighbours').
template <bool WAVE_SYNC>
__device__ __forceinline__ void tile_sync()
{
    if constexpr (WAVE_SYNC) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int ORDER, bool CHUNKED, int KG = kGroup, bool WAVE_SYNC = false, class EM>
__device__ __forceinline__ void walk(const ReconParams &P, EM &em, Run &run,
                                     const uint8_t *base, const Xpose &X, int lane,
                                     int32_t tilew, int32_t tile0, int32_t tile1,
                                     uint64_t (*word_s)[64], int32_t (*cnt_s)[64],
                                     int32_t *rec_start, int64_t fstride, int32_t &cum_base,
                                     int32_t f0 = 0)
{
    uint32_t rlo[KG], rhi[KG];
    int32_t rc[KG];
    // row r = 64 t + lane of tile t: the tile's first row is the same for
    // the whole wave and the lane's byte offset lane * fb is fixed, so each
    // load is a wave-uniform base plus that offset (a 64-bit add, no per-lane
    // multiply)
    const int64_t lane_off = (int64_t)lane * P.fb;
    auto fetch = [&](int32_t tg) {
#pragma unroll
        for (int i = 0; i < KG; i++) {
            const int32_t t = tg + i;
            const int32_t tr = t * 64 + lane;
            rlo[i] = rhi[i] = 0;
            rc[i] = 0;
            if (t < tile1 && tr < P.T) {
                const uint8_t *row0 = base + (int64_t)t * 64 * P.fb;
                const uint64_t v = *gp((const uint64_t *)(row0 + lane_off));
                rlo[i] = (uint32_t)v;
                rhi[i] = (uint32_t)(v >> 32);
                if (P.cnt_le) rc[i] = (gp(P.cnt_le) + t * 64)[lane];
            }
        }
    };
    fetch(tilew);
    for (int32_t tg = tilew; tg < tile1; tg += KG) {
        // the group's rows are in registers: transpose into LDS, then start
        // fetching the next group
#pragma unroll
        for (int i = 0; i < KG; i++) {
            word_s[i][lane] = transpose64(rlo[i], rhi[i], X, lane);
            cnt_s[i][lane] = rc[i];
        }
        fetch(tg + KG);
        tile_sync<WAVE_SYNC>();
        const int32_t ni = min(KG, tile1 - tg);
        for (int i = 0; i < ni; i++) {
            const int32_t t = tg + i;
            const uint64_t w = word_s[i][lane];
            // TFI with outputs at t_out: the frames of this tile that hold
            // an output (the same for every pixel)
            uint64_t omask = 0;
            if constexpr (ORDER == 3 && EM::kMode != MODE_SEGMENTS)
                omask = __ballot(lane > 0 && cnt_s[i][lane] > cnt_s[i][lane > 0 ? lane - 1 : 0]);
            if constexpr (CHUNKED) {
                if (t == tile0 && rec_start) {
                    // the speculative state the fixup pass starts from
                    if (em.valid) save_run<ORDER>(rec_start, fstride, run);
                    cum_base = run.cum;
                }
                // the first tiles of a later chunk keep what the fixup needs
                if (ORDER == 1 && rec_start && t >= tile0 && t < tile0 + kCaptureTiles) {
                    if (w) run.template word<ORDER, true, CHUNKED>(f0 + t * 64, w, cnt_s[i], em);
                    continue;
                }
            }
            if (w) run.template word<ORDER, false, CHUNKED>(f0 + t * 64, w, cnt_s[i], em, omask);
        }
        tile_sync<WAVE_SYNC>();
    }
}

}  // namespace
}  // namespace spk
