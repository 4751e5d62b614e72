// The persistent kernel of the batched plans (spk_plan_*), templated on its
// launch shape, and the per-shape launchers.  Each batch_k<KG>.hip file
// instantiates the shapes of one group size, so the shapes compile in
// parallel.
//
// Work items are 64-pixel strips of every job, each walked over the job's
// whole stream by one wave (the same per-strip walk as the plain kernel).
// The items are split into 8 contiguous ranges, one per XCD, each with its
// own counter: a wave first takes items from its own XCD's range (so the
// 16 strips that share each 128-byte line of a frame stay in one L2), then
// helps the other ranges.  Every wave leaves once all counters are past
// their range's end; nothing waits on another wave.
//
// Launch shape (chosen by the plan's autotuner; every shape gives the same
// output bit for bit):
//   KG   tiles of 64 frames per prefetch group (4, 8, 16): registers and LDS
//        per wave against how far ahead the loads run;
//   WPG  waves per workgroup (1, 2, 4; runtime): each wave takes its own
//        items and keeps its own LDS rows, synchronised at wave scope;
//   WPE  the waves-per-SIMD target the compiler allocates registers for
//        (variant 0: 4, at most 128 VGPRs, where every order's state fits;
//        variant 1: 5, at most 102, more waves to hide latency but some
//        state in scratch for the SSR and third-order machines).
#pragma once

#include "recon_core.h"

namespace spk {

constexpr int kXcds = 8;
constexpr int kMaxWavesPerWG = 4;

struct JobDesc {
    const uint8_t *stream;
    int64_t fb;
    int32_t T, HW;
    double theta;
    const int32_t *cnt_le;
    const int32_t *plane;  // NULL: identity
    int32_t n_out;
    float *out;
    int32_t strip0;        // first item of this job
    int32_t nstrips;
};

struct Ranges {
    int32_t begin[kXcds + 1];  // item range of each XCD
};

// What one launch needs besides its shape.
struct BatchLaunch {
    const JobDesc *jobs;
    int n_jobs;
    Ranges ranges;
    int32_t *counters;
    int order;
    bool identity;
    int grid, grab, waves_per_wg, wpe_variant;
};

__host__ __device__ constexpr int wpe_of(int order, int variant)
{
    return order > 0 && variant == 1 ? 5 : 4;
}

namespace {

__device__ __forceinline__ int find_job(const JobDesc *jobs, int n_jobs, int32_t item)
{
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].strip0 <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int ORDER, int PMAP, int KG, int WPE>
__global__ __launch_bounds__(64 * kMaxWavesPerWG) __attribute__((amdgpu_waves_per_eu(WPE)))
void batch_kernel(const JobDesc *jobs, int n_jobs, Ranges R, int grab, int32_t *counters)
{
    extern __shared__ __attribute__((aligned(16))) uint64_t lds_dyn[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // this wave's LDS rows: KG words, then KG counts, per lane
    uint64_t(*word_s)[64] = (uint64_t(*)[64])(lds_dyn + (size_t)wave * KG * 96);
    int32_t(*cnt_s)[64] = (int32_t(*)[64])(lds_dyn + (size_t)wave * KG * 96 + KG * 64);
    const Xpose X(lane);
    const int home = blockIdx.x % kXcds;
    for (int k = 0; k < kXcds; k++) {
        const int x = (home + k) % kXcds;
        const int32_t n = R.begin[x + 1] - R.begin[x];
        while (true) {
            int32_t i0 = 0;
            if (lane == 0) i0 = atomicAdd(&counters[x], grab);
            i0 = __shfl(i0, 0, 64);
            if (i0 >= n) break;
            const int32_t i1 = min(n, i0 + grab);
            for (int32_t i = i0; i < i1; i++) {
                const int32_t item = R.begin[x] + i;
                const JobDesc &J = jobs[find_job(jobs, n_jobs, item)];
                ReconParams P{};
                P.stream = J.stream;
                P.fb = J.fb;
                P.T = J.T;
                P.HW = J.HW;
                P.theta = J.theta;
                P.cnt_le = J.cnt_le;
                P.plane = J.plane;
                P.n_out = J.n_out;
                P.out = J.out;
                const int64_t p0 = (int64_t)(item - J.strip0) * 64;
                const int64_t p = p0 + lane;
                Emitter<MODE_RECON, false, PMAP> em{P, nullptr, p, p < P.HW, 0, 0};
                Run run;
                run.reset(0, 0);
                int32_t cum_base = 0;
                walk<ORDER, false, KG, true>(P, em, run, P.stream + (p0 >> 3), X, lane, 0, 0,
                                             (P.T + 63) / 64, word_s, cnt_s, nullptr, 0,
                                             cum_base);
                if (run.cum >= 2)
                    em.close(run.first, run.lastspk, (run.cum - 1) - run.first_idx, run.k0,
                             P.n_out);
                else
                    em.empty();
            }
        }
    }
}

// LDS bytes of one wave at group size KG (KG words and KG counts per lane).
constexpr size_t lds_per_wave(int KG) { return (size_t)KG * 64 * 12; }

template <int ORDER, int KG, int WPE>
hipError_t launch_shape(const BatchLaunch &b, hipStream_t st)
{
    const size_t lds = lds_per_wave(KG) * b.waves_per_wg;
    if (b.identity)
        hipLaunchKernelGGL((batch_kernel<ORDER, PMAP_IDENT, KG, WPE>), dim3(b.grid),
                           dim3(64 * b.waves_per_wg), lds, st, b.jobs, b.n_jobs, b.ranges, b.grab,
                           b.counters);
    else
        hipLaunchKernelGGL((batch_kernel<ORDER, PMAP_GLOBAL, KG, WPE>), dim3(b.grid),
                           dim3(64 * b.waves_per_wg), lds, st, b.jobs, b.n_jobs, b.ranges, b.grab,
                           b.counters);
    return hipGetLastError();
}

template <int ORDER, int KG>
hipError_t launch_order_kg(const BatchLaunch &b, hipStream_t st)
{
    return b.wpe_variant == 0 ? launch_shape<ORDER, KG, wpe_of(ORDER, 0)>(b, st)
                              : launch_shape<ORDER, KG, wpe_of(ORDER, 1)>(b, st);
}

template <int KG>
hipError_t launch_kg(const BatchLaunch &b, hipStream_t st)
{
    switch (b.order) {
    case 1: return launch_order_kg<1, KG>(b, st);
    case 2: return launch_order_kg<2, KG>(b, st);
    case 3: return launch_order_kg<3, KG>(b, st);
    default: return launch_order_kg<4, KG>(b, st);
    }
}

}  // namespace

// Defined in batch_k4.hip, batch_k8.hip and batch_k16.hip.
hipError_t launch_batch_k4(const BatchLaunch &b, hipStream_t st);
hipError_t launch_batch_k8(const BatchLaunch &b, hipStream_t st);
hipError_t launch_batch_k16(const BatchLaunch &b, hipStream_t st);

}  // namespace spk
