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
#include <cmath>

#include "recon_core.h"

namespace spk {
namespace {

// Tiles per prefetch group of the main pass.  Four keep the SSR state
// machine and the prefetched rows within 128 VGPRs (124, no scratch; eight
// needed 128 plus 28 bytes of scratch per lane), and four tiles of loads in
// flight are far ahead of memory latency at this kernel's integer work per
// tile (measured on 250x400x20000: FSR 1.35 -> 1.33 ms, SSR unchanged,
// third order 3.76 -> 3.69 ms).
constexpr int kReconGroup = 4;

// Main pass.  With nchunks == 1 a wave walks its strip's whole stream and
// finishes every segment.  With nchunks > 1 the stream is cut into chunks
// of chunk_tiles tiles; chunk 0 runs exactly, every later chunk starts from
// a fresh state at its first spike (speculation), and each wave records its
// state at its chunk's end for the fixup pass, which makes the result exact.
template <int ORDER, int MODE, bool WIN, int PMAP>
// Four waves per SIMD (at most 128 VGPRs) for every order: the walk is
// bound by VALU issue, which the fourth wave keeps fuller.  The third
// order's larger state spills (a few hundred bytes) and still gains: 3.78
// ms against 4.26 at two waves (180 VGPRs, no spill) on a 250x400x20000
// stream.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
void recon_kernel(ReconParams P, int nblocks, ChunkPlan cp)
{
    __shared__ uint64_t word_s[kReconGroup][64];
    __shared__ int32_t cnt_s[kReconGroup][64];
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
    const int32_t kmin = tile0 > 0 && MODE != MODE_SEGMENTS ? P.cnt_le[tile0 * 64 - 1] : 0;
    Emitter<MODE, WIN, PMAP> em{P, plane_dyn, p, p < P.HW, 0, kmin};
    const uint8_t *base = P.stream + (p0 >> 3);
    const Xpose X(lane);
    const int64_t fstride = (int64_t)cp.nchunks * P.HW;

    Run run;
    run.reset(tilew > 0 && MODE != MODE_SEGMENTS ? P.cnt_le[tilew * 64 - 1] : 0, tile0 * 64);
    int32_t cum_base = 0;  // spikes seen before tile0
    if (cp.nchunks > 1)
        walk<ORDER, true, kReconGroup>(P, em, run, base, X, lane, tilew, tile0, tile1, word_s,
                                       cnt_s, chunk > 0 ? rec_start(cp, chunk, p, P.HW) : nullptr,
                                       fstride, cum_base);
    else
        walk<ORDER, false, kReconGroup>(P, em, run, base, X, lane, tilew, tile0, tile1, word_s,
                                        cnt_s, nullptr, fstride, cum_base);
    if (cp.nchunks > 1) {
        // end-of-chunk record, spike indices relative to the chunk's start
        run.cum -= cum_base;
        run.first_idx -= cum_base;
        run.fi1 -= cum_base;
        if (em.valid) save_run<ORDER>(rec_end(cp, chunk, p, P.HW), fstride, run);
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
// then cuts exactly there too.  The window up to that next cut is known only
// when the main pass recorded it (its first cut fell in the chunk's first
// capture tiles); without it the rule needs the two windows equal (the
// true machine then decides as the speculative one does).  The lane then takes the main pass's
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
    if (em.valid) load_run<ORDER>(rec_end(cp, 0, p, P.HW), fstride, tr);
    else tr.reset(0);
    for (int c = 1; c < cp.nchunks; c++) {
        Run rc, sp;
        if (em.valid) {
            load_run<ORDER>(rec_end(cp, c, p, P.HW), fstride, rc);
            load_run<ORDER>(rec_start(cp, c, p, P.HW), fstride, sp);
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
        // The stopping rules, tried after the true and the speculative
        // machines have both taken the spike at tau (see above).
        auto stop_checks = [&](int32_t tau) {
            if (ORDER == 1 && rc.fb1 >= tau &&
                ((tr.st.flo == sp.st.flo && tr.st.fhi == sp.st.fhi) ||
                 (rc.fwlo <= rc.fwhi && tr.st.flo <= sp.st.flo && sp.st.fhi <= tr.st.fhi &&
                  max(tr.st.fhi, rc.fwhi) - min(tr.st.flo, rc.fwlo) <= 1))) {
                // FSR: the true window equals the speculative one, or holds
                // it and stays stable with every interval up to the main
                // pass's next cut (the window the main pass recorded), so
                // the true machine makes that same cut next and both
                // restart there: close the true segment at that cut and
                // take the main pass's record from then on
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
        };
        if (__any(!done)) fetch(tile0);
        for (int32_t t = tile0; t < tile1 && __any(!done); t++) {
            const uint32_t lo = nlo, hi = nhi;
            cnt_s[lane] = ncv;
            fetch(t + 1);
            uint64_t w = transpose64(lo, hi, X, lane);
            __syncthreads();
            // A word that cuts neither machine is taken whole by both with
            // the main pass's word shortcut; the stopping rules are then
            // tried at its last spike.  Without it a chunk whose speculative
            // state never becomes equivalent to the true one (constant
            // light: the true S2 extremes hold gaps the warm-up never saw)
            // would be replayed spike by spike to its end.
            if (!done && w && tr.lastspk >= 0 && tr.lastspk == sp.lastspk) {
                const int32_t c = popc64(w);
                const int32_t x0 = t * 64 + ctz64(w) - tr.lastspk;
                SegState a = tr.st, b = sp.st;
                if (a.template fast_word<ORDER>(w, x0, c) &&
                    b.template fast_word<ORDER>(w, x0, c)) {
                    tr.st = a;
                    sp.st = b;
                    const int hp = hibit64(w);
                    const int32_t tau = t * 64 + hp;
                    tr.lastspk = sp.lastspk = tau;
                    tr.cum += c;
                    tr.cnt_last = cnt_s[hp];
                    w = 0;
                    stop_checks(tau);
                }
            }
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
                stop_checks(tau);
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

namespace {

// Waves of the main pass of the given order that fit on the current device
// at once (occupancy x CUs), or 0 if unknown.
int resident_waves(int order)
{
    constexpr int kMaxDev = 64;
    static int cache[kMaxDev][5] = {};
    int dev = 0, cus = 0, per_cu = 0;
    if (order < 1 || order > 4 || hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev)
        return 0;
    if (cache[dev][order]) return cache[dev][order];
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) {
        switch (order) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, recon_kernel<1, MODE_RECON, false, PMAP_IDENT>, 64, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, recon_kernel<2, MODE_RECON, false, PMAP_IDENT>, 64, 0); break;
        case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, recon_kernel<3, MODE_RECON, false, PMAP_IDENT>, 64, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     &per_cu, recon_kernel<4, MODE_RECON, false, PMAP_IDENT>, 64, 0); break;
        }
    }
    if (e != hipSuccess || cus <= 0 || per_cu <= 0) {
        (void)hipGetLastError();
        return 0;
    }
    return cache[dev][order] = cus * per_cu;
}

}  // namespace

// Automatic chunk count.  More chunks give more waves, but each chunk after
// the first re-walks its warm-up tiles and adds fixup work (about one more
// tile).  The waves of equal length run in rounds of R (the resident
// waves), and a last partial round leaves the chip part idle, so the model
// minimises (1 + (c - 1) (warm + 1) / tiles) * sqrt(ceil(r) / r), r = waves
// / R.  (Measured at 250x400 x 20000 frames, where waves alternate between
// just above and just below whole rounds as c grows, this puts SSR within
// 1.2% and FSR at the fastest of the counts 3..14.)
ChunkPlan plan_chunks(int32_t HW, int32_t T, int order, int requested, int warm)
{
    ChunkPlan cp;
    cp.fields = rec_fields_of(order);
    const int nblocks = (HW + 63) / 64;
    const int ntiles = (T + 63) / 64;
    int c = requested;
    if (c <= 0) {
        const int cmax = max(1, ntiles / kMinChunkTiles);  // chunks long enough to pay off
        const int R = resident_waves(order);
        if (R <= 0) {
            c = min((kTargetWaves + nblocks - 1) / nblocks, cmax);  // enough waves to fill the chip
        } else {
            double best = 0.0;
            for (int k = 1; k <= min(cmax, kMaxAutoChunks); k++) {
                const int chunk_tiles = (ntiles + k - 1) / k;
                const int w = warm >= 0 ? warm : min(kWarmTiles, chunk_tiles / 2);
                const double r = (double)nblocks * k / R;
                const double cost = (1.0 + (double)(k - 1) * (w + 1) / ntiles) *
                                    std::sqrt(std::ceil(r) / r);
                if (k == 1 || cost < best) {
                    best = cost;
                    c = k;
                }
            }
        }
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
        switch (order) {
        case 1: return launch_one<1, MODE_SEGMENTS, false, PMAP_IDENT>(p, one, stream);
        case 2: return launch_one<2, MODE_SEGMENTS, false, PMAP_IDENT>(p, one, stream);
        case 3: return launch_one<3, MODE_SEGMENTS, false, PMAP_IDENT>(p, one, stream);
        default: return launch_one<4, MODE_SEGMENTS, false, PMAP_IDENT>(p, one, stream);
        }
    }
    if (mode == MODE_MOTION) {
        switch (order) {
        case 1: return launch_pmap<1, MODE_MOTION, false>(p, cp, stream);
        case 2: return launch_pmap<2, MODE_MOTION, false>(p, cp, stream);
        case 3: return launch_pmap<3, MODE_MOTION, false>(p, cp, stream);
        default: return launch_pmap<4, MODE_MOTION, false>(p, cp, stream);
        }
    }
    switch (order) {
    case 1: return win ? launch_pmap<1, MODE_RECON, true>(p, cp, stream)
                       : launch_pmap<1, MODE_RECON, false>(p, cp, stream);
    case 2: return win ? launch_pmap<2, MODE_RECON, true>(p, cp, stream)
                       : launch_pmap<2, MODE_RECON, false>(p, cp, stream);
    case 3: return win ? launch_pmap<3, MODE_RECON, true>(p, cp, stream)
                       : launch_pmap<3, MODE_RECON, false>(p, cp, stream);
    default: return win ? launch_pmap<4, MODE_RECON, true>(p, cp, stream)
                        : launch_pmap<4, MODE_RECON, false>(p, cp, stream);
    }
}

}  // namespace spk
