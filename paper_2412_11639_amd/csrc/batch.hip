// Batched reconstruction: many streams of uneven size in one persistent
// kernel, captured once in a HIP graph, with launch shapes chosen by a
// small autotuner.
//
// Work items are 64-pixel strips of every job, each walked over the job's
// whole stream by one wave (the same per-strip walk as the plain kernel).
// The items are split into 8 contiguous ranges, one per XCD, each with its
// own counter: a wave first takes items from its own XCD's range (so the
// 16 strips that share each 128-byte line of a frame stay in one L2), then
// helps the other ranges.  Every wave leaves once all counters are past
// their range's end; nothing waits on another wave.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "recon_core.h"
#include "spk.h"

namespace spk {
namespace {

constexpr int kXcds = 8;

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

__global__ void reset_counters(int32_t *counters)
{
    if (threadIdx.x < kXcds) counters[threadIdx.x] = 0;
}

template <int ORDER, int PMAP>
__global__ __launch_bounds__(64) void batch_kernel(const JobDesc *jobs, int n_jobs, Ranges R,
                                                   int grab, int32_t *counters)
{
    __shared__ uint64_t word_s[kGroup][64];
    __shared__ int32_t cnt_s[kGroup][64];
    const int lane = threadIdx.x;
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
                walk<ORDER, false>(P, em, run, P.stream + (p0 >> 3), X, lane, 0, 0,
                                   (P.T + 63) / 64, word_s, cnt_s, nullptr, 0, cum_base);
                if (run.cum >= 2)
                    em.close(run.first, run.lastspk, (run.cum - 1) - run.first_idx, run.k0,
                             P.n_out);
                else
                    em.empty();
            }
        }
    }
}

}  // namespace
}  // namespace spk

using spk::JobDesc;

struct spk_plan_s {
    int dev = -1;
    int order = SPK_FSR;
    int n_jobs = 0;
    int32_t total_items = 0;
    bool identity = true;
    int grid = 0, grab = 1;
    bool use_graph = true;
    JobDesc *d_jobs = nullptr;
    int32_t *d_tables = nullptr;
    int32_t *d_counters = nullptr;
    spk::Ranges ranges{};
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string signature;
};

namespace {

std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;  // signature -> (grid, grab)
bool g_tune_loaded = false;

const char *tune_path() { return std::getenv("SPK_TUNE_CACHE"); }

// The tuning cache is a flat JSON object {"signature": [grid, grab], ...}.
void tune_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = tune_path();
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    size_t pos = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
        const size_t end = text.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = text.substr(pos + 1, end - pos - 1);
        int grid = 0, grab = 0;
        if (std::sscanf(text.c_str() + end + 1, " : [ %d , %d ]", &grid, &grab) == 2 && grid > 0 &&
            grab > 0)
            g_tune[key] = {grid, grab};
        pos = end + 1;
    }
}

void tune_store()
{
    const char *path = tune_path();
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : g_tune)
        std::fprintf(f, "  \"%s\": [%d, %d]%s\n", kv.first.c_str(), kv.second.first,
                     kv.second.second, ++i < g_tune.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

hipError_t launch_batch(const spk_plan_s *pl, int grid, int grab, hipStream_t st)
{
    hipLaunchKernelGGL(spk::reset_counters, dim3(1), dim3(64), 0, st, pl->d_counters);
#define SPK_BATCH_LAUNCH(O)                                                                  \
    if (pl->identity)                                                                          \
        hipLaunchKernelGGL((spk::batch_kernel<O, spk::PMAP_IDENT>), dim3(grid), dim3(64), 0,   \
                           st, pl->d_jobs, pl->n_jobs, pl->ranges, grab, pl->d_counters);      \
    else                                                                                       \
        hipLaunchKernelGGL((spk::batch_kernel<O, spk::PMAP_GLOBAL>), dim3(grid), dim3(64), 0,  \
                           st, pl->d_jobs, pl->n_jobs, pl->ranges, grab, pl->d_counters);
    switch (pl->order) {
    case SPK_FSR: SPK_BATCH_LAUNCH(1) break;
    case SPK_SSR: SPK_BATCH_LAUNCH(2) break;
    case SPK_TFI: SPK_BATCH_LAUNCH(3) break;
    default: SPK_BATCH_LAUNCH(4) break;
    }
#undef SPK_BATCH_LAUNCH
    return hipGetLastError();
}

// Time each candidate launch shape twice (the second run counts) and keep
// the fastest.  Every shape gives the same output.
int autotune(spk_plan_s *pl, hipStream_t st)
{
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, pl->dev) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    const int grids[] = {cus * 4, cus * 8, cus * 16, cus * 32};
    const int grabs[] = {1, 4};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SPK_EHIP;
    float best = 1e30f;
    for (int g : grids) {
        for (int b : grabs) {
            float ms = 0.0f;
            for (int rep = 0; rep < 2; rep++) {
                hipEventRecord(e0, st);
                if (launch_batch(pl, g, b, st) != hipSuccess) return SPK_EHIP;
                hipEventRecord(e1, st);
                if (hipEventSynchronize(e1) != hipSuccess) return SPK_EHIP;
                hipEventElapsedTime(&ms, e0, e1);
            }
            if (ms < best) {
                best = ms;
                pl->grid = g;
                pl->grab = b;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return SPK_OK;
}

void plan_free(spk_plan_s *pl)
{
    if (pl->exec) hipGraphExecDestroy(pl->exec);
    if (pl->graph) hipGraphDestroy(pl->graph);
    if (pl->capture_stream) hipStreamDestroy(pl->capture_stream);
    if (pl->d_jobs) hipFree(pl->d_jobs);
    if (pl->d_tables) hipFree(pl->d_tables);
    if (pl->d_counters) hipFree(pl->d_counters);
    delete pl;
}

}  // namespace

extern "C" {

int spk_plan_create(spk_plan_t *plan, const spk_job *jobs, int32_t n_jobs, int32_t order,
                    int32_t flags)
{
    if (!plan) return SPK_EINVAL;
    *plan = nullptr;
    if (!jobs || n_jobs <= 0 || order < SPK_FSR || order > SPK_TSR) return SPK_EINVAL;
    if (flags & ~(SPK_PLAN_AUTOTUNE | SPK_PLAN_NO_GRAPH)) return SPK_EINVAL;
    // validate every job before touching the device
    int64_t items = 0;
    size_t table_ints = 0;
    for (int32_t j = 0; j < n_jobs; j++) {
        const spk_job &J = jobs[j];
        if (!J.stream || !J.out || J.H <= 0 || J.W <= 0 || J.T <= 0 || J.n_out <= 0 ||
            !J.t_out || !std::isfinite(J.theta) || !(J.theta > 0.0f))
            return SPK_EINVAL;
        if ((uintptr_t)J.stream & 15u) return SPK_EINVAL;  // frames are read as words
        if ((int64_t)J.H * J.W > (int64_t)INT32_MAX - 128) return SPK_EINVAL;
        if ((int64_t)J.n_out * J.H * J.W > ((int64_t)1 << 60)) return SPK_EINVAL;
        for (int32_t k = 0; k < J.n_out; k++)
            if (J.t_out[k] < 0 || J.t_out[k] >= J.T) return SPK_EINVAL;
        items += ((int64_t)J.H * J.W + 63) / 64;
        table_ints += (size_t)J.T + (size_t)J.n_out;
    }
    if (items > INT32_MAX / 2) return SPK_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPK_EHIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return SPK_EHIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SPK_EUNSUPPORTED;

    spk_plan_s *pl = new spk_plan_s();
    pl->dev = dev;
    pl->order = order;
    pl->n_jobs = n_jobs;
    pl->total_items = (int32_t)items;
    pl->use_graph = !(flags & SPK_PLAN_NO_GRAPH);

    // host images of the job table and of the sorted output-time tables
    std::vector<int32_t> tables(table_ints);
    std::vector<JobDesc> desc(n_jobs);
    std::vector<size_t> toff(n_jobs);
    size_t off = 0;
    int32_t strip = 0;
    char sig[64];
    static const char *const names[] = {"", "fsr", "ssr", "tfi", "tsr"};
    pl->signature = names[order];
    for (int32_t j = 0; j < n_jobs; j++) {
        const spk_job &J = jobs[j];
        std::vector<int32_t> ord(J.n_out);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int32_t a, int32_t b) { return J.t_out[a] < J.t_out[b]; });
        bool ident = true;
        for (int32_t k = 0; k < J.n_out; k++)
            if (ord[k] != k || (k > 0 && J.t_out[ord[k]] == J.t_out[ord[k - 1]])) ident = false;
        int32_t *cnt = tables.data() + off, *plane = cnt + J.T;
        int32_t k = 0;
        for (int32_t t = 0; t < J.T; t++) {
            while (k < J.n_out && J.t_out[ord[k]] <= t) k++;
            cnt[t] = k;
        }
        for (int32_t q = 0; q < J.n_out; q++) plane[q] = ord[q];
        toff[j] = off;
        off += (size_t)J.T + J.n_out;
        JobDesc &D = desc[j];
        D.stream = J.stream;
        D.fb = (int64_t)spk_frame_bytes(J.H, J.W);
        D.T = J.T;
        D.HW = J.H * J.W;
        D.theta = (double)J.theta;
        D.n_out = J.n_out;
        D.out = J.out;
        D.strip0 = strip;
        D.nstrips = (D.HW + 63) / 64;
        strip += D.nstrips;
        pl->identity = pl->identity && ident;
        D.plane = nullptr;  // set to the device copy below when any job needs a map
        std::snprintf(sig, sizeof sig, ":%dx%dx%d/%d", J.H, J.W, J.T, J.n_out);
        pl->signature += sig;
    }
    int rc = SPK_OK;
    if (hipMalloc((void **)&pl->d_tables, table_ints * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void **)&pl->d_jobs, n_jobs * sizeof(JobDesc)) != hipSuccess ||
        hipMalloc((void **)&pl->d_counters, spk::kXcds * sizeof(int32_t)) != hipSuccess) {
        plan_free(pl);
        return SPK_ENOMEM;
    }
    for (int32_t j = 0; j < n_jobs; j++) {
        desc[j].cnt_le = pl->d_tables + toff[j];
        if (!pl->identity) desc[j].plane = pl->d_tables + toff[j] + desc[j].T;
    }
    // per-XCD contiguous ranges of items
    for (int x = 0; x <= spk::kXcds; x++)
        pl->ranges.begin[x] = (int32_t)((int64_t)pl->total_items * x / spk::kXcds);
    if (hipMemcpy(pl->d_tables, tables.data(), table_ints * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(pl->d_jobs, desc.data(), n_jobs * sizeof(JobDesc), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipStreamCreateWithFlags(&pl->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        plan_free(pl);
        return SPK_EHIP;
    }
    // launch shape: tuned once per signature (cached across plans and, with
    // SPK_TUNE_CACHE set, across processes), else a fixed default
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_load();
        auto it = g_tune.find(pl->signature);
        if (it != g_tune.end()) {
            pl->grid = it->second.first;
            pl->grab = it->second.second;
        } else if (flags & SPK_PLAN_AUTOTUNE) {
            rc = autotune(pl, pl->capture_stream);
            if (rc == SPK_OK) {
                g_tune[pl->signature] = {pl->grid, pl->grab};
                tune_store();
            }
        } else {
            pl->grid = prop.multiProcessorCount * 16;
            pl->grab = 1;
        }
    }
    if (rc != SPK_OK) {
        plan_free(pl);
        return rc;
    }
    if (pl->use_graph) {
        if (hipStreamBeginCapture(pl->capture_stream, hipStreamCaptureModeThreadLocal) !=
                hipSuccess ||
            launch_batch(pl, pl->grid, pl->grab, pl->capture_stream) != hipSuccess ||
            hipStreamEndCapture(pl->capture_stream, &pl->graph) != hipSuccess ||
            hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess) {
            plan_free(pl);
            return SPK_EHIP;
        }
    }
    if (hipStreamSynchronize(pl->capture_stream) != hipSuccess) {
        plan_free(pl);
        return SPK_EHIP;
    }
    *plan = pl;
    return SPK_OK;
}

int spk_plan_execute(spk_plan_t plan, void *hip_stream)
{
    if (!plan) return SPK_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    if (plan->use_graph)
        return hipGraphLaunch(plan->exec, st) == hipSuccess ? SPK_OK : SPK_EHIP;
    return launch_batch(plan, plan->grid, plan->grab, st) == hipSuccess ? SPK_OK : SPK_EHIP;
}

int spk_plan_info(spk_plan_t plan, int32_t *grid, int32_t *grab, int32_t *items)
{
    if (!plan) return SPK_EINVAL;
    if (grid) *grid = plan->grid;
    if (grab) *grab = plan->grab;
    if (items) *items = plan->total_items;
    return SPK_OK;
}

int spk_plan_destroy(spk_plan_t plan)
{
    if (!plan) return SPK_OK;
    // the plan may still be executing on any stream of its device
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(plan->dev);
    hipError_t e = hipDeviceSynchronize();
    plan_free(plan);
    hipSetDevice(cur);
    return e == hipSuccess ? SPK_OK : SPK_EHIP;
}

}  // extern "C"
