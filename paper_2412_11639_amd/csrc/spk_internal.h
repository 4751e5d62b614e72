// Internal interface between the C-ABI glue and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spk {

// What one launch of the reconstruction kernel works on.  Device pointers
// unless stated.
struct ReconParams {
    const uint8_t *stream;   // [T][fb] packed frames
    int64_t fb;              // bytes per frame (multiple of 16)
    int32_t T;
    int32_t HW;
    double theta;
    const int32_t *cnt_le;   // [T]: number of sorted output times <= t
    const int32_t *plane;    // [n_out]: sorted output index -> output plane (NULL = identity)
    int32_t n_out;
    float *out;              // [n_out][HW] or NULL
    int32_t *win_first;      // [n_out][HW] or NULL
    int32_t *win_last;
    int32_t *win_n;
    // segment listing mode
    int32_t cap;
    int32_t *seg_first;      // [cap][HW]
    int32_t *seg_last;
    int32_t *seg_n;
    int32_t *seg_rec;        // [HW][cap][3] (first, last, n), used instead when not NULL
    int32_t *count;          // [HW]
    // static / motion mask mode: mask[k][p] = 1 when the segment holding
    // sorted output k is not the pixel's first (its first spike is not
    // first_spike[p]) and starts less than window frames before output k
    const int32_t *first_spike;  // [HW]
    int32_t window;
    uint8_t *mask;           // [n_out][HW]
};

enum Mode { MODE_RECON = 0, MODE_SEGMENTS = 1, MODE_MOTION = 2 };

// Fields of one per-chunk state record (the most any order keeps).
constexpr int kRecFields = 37;

// How a stream is cut into time chunks processed by separate waves.
struct ChunkPlan {
    int nchunks = 1;
    int chunk_tiles = 1 << 30;  // 64-frame tiles per chunk
    int warm_tiles = 0;         // tiles of speculative warm-up before a chunk
    int fields = kRecFields;    // record fields the order keeps
    int32_t *rec = nullptr;     // device [2][fields][nchunks][HW] int32 when nchunks > 1
};

// Number of chunks for a stream of the given order (requested <= 0:
// automatic; warm < 0: automatic warm-up length).
ChunkPlan plan_chunks(int32_t HW, int32_t T, int order, int requested, int warm = -1);

// Ints of device workspace a plan needs.
inline size_t chunk_record_ints(const ChunkPlan &cp, int32_t HW)
{
    return cp.nchunks > 1 ? (size_t)2 * cp.fields * cp.nchunks * (size_t)HW : 0;
}

// Device tables of one output-time list (cached per device; a table stays
// valid for the kernels queued after this call): cnt_le[t] = number of
// output times <= t for t < T, plane[j] = the output slot of the j-th time
// in time order (stable), t_sorted[j] = that time; identity when t_out is
// strictly increasing.  Checks for a gfx950 device.  Returns an SPK code.
struct OutTables {
    const int32_t *cnt_le, *plane, *t_sorted;
    bool identity;
};
int out_tables(int32_t T, const int32_t *t_out, int32_t n_out, hipStream_t stream,
               OutTables *out);

// SPK_OPT_SUR_CONV_WG: workgroup cap of the surrogate convolutions (0: by
// occupancy).
extern int g_sur_conv_wg;

// SPK_OPT_PLAN_*: the launch shape of plans created without autotuning.
int set_plan_option(int option, int value);
int get_plan_option(int option);

// Enqueue the plain FSR/SSR reconstruction (or segment listing) on stream.
hipError_t launch_recon(const ReconParams &p, int order, Mode mode, const ChunkPlan &cp,
                        hipStream_t stream);

}  // namespace spk
