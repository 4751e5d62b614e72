// Batched reconstruction: many streams of uneven size in one persistent
// kernel (batch_kernels.h), captured once in a HIP graph, with the launch
// shape -- total waves, strips per counter grab, tiles per prefetch group,
// waves per workgroup and the waves-per-SIMD register target -- chosen by a
// small autotuner that times candidate shapes on the plan's own jobs.
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

#include "batch_kernels.h"

using spk::JobDesc;

// A launch shape (see batch_kernels.h).  grid counts workgroups.
struct Shape {
    int grid = 0, grab = 1, kg = 8, wpg = 1, wpe = 0;
};

struct spk_plan_s {
    int dev = -1;
    int order = SPK_FSR;
    int n_jobs = 0;
    int32_t total_items = 0;
    bool identity = true;
    Shape shape;
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

__global__ void reset_counters(int32_t *counters)
{
    if (threadIdx.x < spk::kXcds) counters[threadIdx.x] = 0;
}

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tune;  // signature -> shape
bool g_tune_loaded = false;

// Shape set by spk_set_option for plans created without autotuning
// (0 = the default of each field).
int g_force_kg = 0, g_force_wpg = 0, g_force_wpe = 0;

const char *tune_path() { return std::getenv("SPK_TUNE_CACHE"); }

bool shape_ok(const Shape &h)
{
    return h.grid > 0 && h.grab > 0 && (h.kg == 4 || h.kg == 8 || h.kg == 16) &&
           (h.wpg == 1 || h.wpg == 2 || h.wpg == 4) && (h.wpe == 0 || h.wpe == 1);
}

// The tuning cache is a flat JSON object
// {"signature": [grid, grab, kgroup, waves_per_wg, wpe_variant], ...}.
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
        Shape h;
        if (std::sscanf(text.c_str() + end + 1, " : [ %d , %d , %d , %d , %d ]", &h.grid, &h.grab,
                        &h.kg, &h.wpg, &h.wpe) == 5 &&
            shape_ok(h))
            g_tune[key] = h;
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
        std::fprintf(f, "  \"%s\": [%d, %d, %d, %d, %d]%s\n", kv.first.c_str(), kv.second.grid,
                     kv.second.grab, kv.second.kg, kv.second.wpg, kv.second.wpe,
                     ++i < g_tune.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

hipError_t launch_batch(const spk_plan_s *pl, const Shape &h, hipStream_t st)
{
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, st, pl->d_counters);
    spk::BatchLaunch b;
    b.jobs = pl->d_jobs;
    b.n_jobs = pl->n_jobs;
    b.ranges = pl->ranges;
    b.counters = pl->d_counters;
    b.order = pl->order;
    b.identity = pl->identity;
    b.grid = h.grid;
    b.grab = h.grab;
    b.waves_per_wg = h.wpg;
    b.wpe_variant = h.wpe;
    switch (h.kg) {
    case 4: return spk::launch_batch_k4(b, st);
    case 16: return spk::launch_batch_k16(b, st);
    default: return spk::launch_batch_k8(b, st);
    }
}

// Time one shape: two runs, the second counts.  Every shape gives the same
// output.
int time_shape(spk_plan_s *pl, const Shape &h, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
               float *ms)
{
    for (int rep = 0; rep < 2; rep++) {
        if (hipEventRecord(e0, st) != hipSuccess) return SPK_EHIP;
        if (launch_batch(pl, h, st) != hipSuccess) return SPK_EHIP;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return SPK_EHIP;
        if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return SPK_EHIP;
    }
    return SPK_OK;
}

// Staged search over the launch shape, each stage keeping the fastest:
// total waves (4, 8, 16, 32 per CU) x strips per grab (1, 4) at 8 tiles
// per group, one wave per workgroup, the order's default register target;
// then the group size (4, 16); the other register target; waves per
// workgroup (2, 4); and the total waves and grab once more at the shape
// found.  About 20 timed shapes.
int autotune(spk_plan_s *pl, hipStream_t st)
{
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, pl->dev) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SPK_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return SPK_EHIP;
    }
    Shape best;
    float best_ms = 1e30f;
    int rc = SPK_OK;
    auto consider = [&](Shape h) {
        if (rc != SPK_OK) return;
        float ms = 0.0f;
        rc = time_shape(pl, h, st, e0, e1, &ms);
        if (rc == SPK_OK && ms < best_ms) {
            best_ms = ms;
            best = h;
        }
    };
    auto waves_grab = [&]() {
        const Shape base = best;
        for (int w : {4, 8, 16, 32})
            for (int b : {1, 4}) {
                Shape h = base;
                h.grid = cus * w / h.wpg;
                h.grab = b;
                consider(h);
            }
    };
    best.grid = cus * 16;
    waves_grab();
    for (int kg : {4, 16}) {
        Shape h = best;
        h.kg = kg;
        consider(h);
    }
    {
        Shape h = best;
        h.wpe = 1 - h.wpe;
        consider(h);
    }
    for (int wpg : {2, 4}) {
        Shape h = best;
        h.grid = best.grid * best.wpg / wpg;
        h.wpg = wpg;
        consider(h);
    }
    waves_grab();
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc == SPK_OK) pl->shape = best;
    return rc;
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

namespace spk {

int set_plan_option(int option, int value)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    switch (option) {
    case SPK_OPT_PLAN_KGROUP:
        if (value != 0 && value != 4 && value != 8 && value != 16) return SPK_EINVAL;
        g_force_kg = value;
        return SPK_OK;
    case SPK_OPT_PLAN_WAVES_PER_WG:
        if (value != 0 && value != 1 && value != 2 && value != 4) return SPK_EINVAL;
        g_force_wpg = value;
        return SPK_OK;
    case SPK_OPT_PLAN_WPE:
        if (value != 0 && value != 1) return SPK_EINVAL;
        g_force_wpe = value;
        return SPK_OK;
    default:
        return SPK_EINVAL;
    }
}

int get_plan_option(int option)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    switch (option) {
    case SPK_OPT_PLAN_KGROUP: return g_force_kg;
    case SPK_OPT_PLAN_WAVES_PER_WG: return g_force_wpg;
    case SPK_OPT_PLAN_WPE: return g_force_wpe;
    default: return SPK_EINVAL;
    }
}

}  // namespace spk

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
        if ((flags & SPK_PLAN_AUTOTUNE) && it != g_tune.end()) {
            pl->shape = it->second;
        } else if (flags & SPK_PLAN_AUTOTUNE) {
            rc = autotune(pl, pl->capture_stream);
            if (rc == SPK_OK) {
                g_tune[pl->signature] = pl->shape;
                tune_store();
            }
        } else {
            Shape h;
            h.kg = g_force_kg ? g_force_kg : 8;
            h.wpg = g_force_wpg ? g_force_wpg : 1;
            h.wpe = g_force_wpe;
            h.grid = prop.multiProcessorCount * 16 / h.wpg;
            h.grab = 1;
            pl->shape = h;
        }
    }
    if (rc != SPK_OK) {
        plan_free(pl);
        return rc;
    }
    if (pl->use_graph) {
        if (hipStreamBeginCapture(pl->capture_stream, hipStreamCaptureModeThreadLocal) !=
                hipSuccess ||
            launch_batch(pl, pl->shape, pl->capture_stream) != hipSuccess ||
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
    return launch_batch(plan, plan->shape, st) == hipSuccess ? SPK_OK : SPK_EHIP;
}

int spk_plan_info(spk_plan_t plan, int32_t *grid, int32_t *grab, int32_t *items)
{
    if (!plan) return SPK_EINVAL;
    if (grid) *grid = plan->shape.grid;
    if (grab) *grab = plan->shape.grab;
    if (items) *items = plan->total_items;
    return SPK_OK;
}

int spk_plan_shape(spk_plan_t plan, int32_t *kgroup, int32_t *waves_per_wg,
                   int32_t *waves_per_simd)
{
    if (!plan) return SPK_EINVAL;
    if (kgroup) *kgroup = plan->shape.kg;
    if (waves_per_wg) *waves_per_wg = plan->shape.wpg;
    if (waves_per_simd) *waves_per_simd = spk::wpe_of(plan->order, plan->shape.wpe);
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
