// Learned surrogate for gfx950: a 4-layer 3x3 CNN (33 -> 32 -> 32 -> 32 -> 1,
// ReLU between) that maps a 32-frame spike window plus the plain
// short-window estimate to the long-window reconstruction.  The output is
// residual on the estimate: y = est + CNN(window, est).
//
//   sur_input     per pixel: the 32-frame window as a bit word (a wave
//                 loads 32 frame rows of 64 pixels and transposes them),
//                 the plain estimate on that window (FSR on the window as a
//                 stream of its own, Eq. 6; fixed-window rate below two
//                 spikes) and whether FSR keeps the window as one segment.
//   conv (MFMA)   implicit GEMM per 16-pixel row tile (a workgroup walks
//                 16x16 blocks, prefetching the next halo): M = 16 pixels,
//                 N = 16 output channels per v_mfma_f32_16x16x32_bf16,
//                 K = 32 input channels of one tap per step, 9 taps (plus a
//                 step for the estimate channel in layer 1).  The weights of
//                 a layer are packed once into the B-operand lane layout and
//                 kept in registers by every wave; activations are bfloat16
//                 NHWC, accumulation float32; the epilogue adds the bias,
//                 applies ReLU (forward) or the ReLU mask (backward) and
//                 writes 16-byte rows through LDS.  The input gradient of a
//                 layer is the same GEMM with the taps mirrored and the
//                 channel roles swapped.
//   wgrad (MFMA)  per tap a GEMM with M = output channels, N = input
//                 channels, K = the pixels of a 16x16 tile (both operands
//                 staged channel-major in LDS); workgroups write partial
//                 sums that one more kernel adds in a fixed order
//                 (deterministic).
//   loss, adam, mux  elementwise.
//   training plan  one step (crops from a per-step table, forward, backward,
//                 Adam) captured in a HIP graph and replayed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <vector>

#include "spk.h"
#include "spk_internal.h"

namespace spk {
namespace sur {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int C = 32;
constexpr int kBig = 1 << 29;

// Parameter blob offsets (floats): W1 [32][9][33], b1, W2 [32][9][32], b2,
// W3 [32][9][32], b3, W4 [1][9][32], b4.
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + 32 * 9 * 33;
constexpr int OFF_W2 = OFF_B1 + 32;
constexpr int OFF_B2 = OFF_W2 + 32 * 9 * 32;
constexpr int OFF_W3 = OFF_B2 + 32;
constexpr int OFF_B3 = OFF_W3 + 32 * 9 * 32;
constexpr int OFF_W4 = OFF_B3 + 32;
constexpr int OFF_B4 = OFF_W4 + 9 * 32;
constexpr int NPARAMS = OFF_B4 + 1;
static_assert(NPARAMS == SPK_SUR_NPARAMS, "parameter layout");

// Packed B operands: [step][nblock][lane][8] bf16.
enum PackKind { PK_FIRST = 0, PK_MID2, PK_MID3, PK_LAST, PK_DG3, PK_DG2, PK_DG4, PK_COUNT };
__host__ __device__ constexpr int pack_steps(int k) { return k == PK_FIRST ? 10 : (k == PK_DG4 ? 1 : 9); }
__host__ __device__ constexpr int pack_nb(int k) { return k == PK_LAST ? 1 : 2; }
__host__ __device__ constexpr int pack_elems(int k) { return pack_steps(k) * pack_nb(k) * 64 * 8; }
__host__ __device__ constexpr int pack_offset(int k)
{
    int o = 0;
    for (int i = 0; i < k; i++) o += pack_elems(i);
    return o;
}
constexpr int PACK_TOTAL = pack_offset(PK_COUNT);

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// Value of the packed B operand: step s, block nb, column j (output channel
// within the block), row k (input channel within the step).
__device__ float pack_value(const float *P, int kind, int s, int nb, int j, int k)
{
    const int co = nb * 16 + j;
    switch (kind) {
    case PK_FIRST:  // steps 0..8: tap s, bit channel k; step 9: estimate, tap k
        if (s < 9) return P[OFF_W1 + (co * 9 + s) * 33 + k];
        return k < 9 ? P[OFF_W1 + (co * 9 + k) * 33 + 32] : 0.0f;
    case PK_MID2: return P[OFF_W2 + (co * 9 + s) * 32 + k];
    case PK_MID3: return P[OFF_W3 + (co * 9 + s) * 32 + k];
    case PK_LAST: return j == 0 ? P[OFF_W4 + s * 32 + k] : 0.0f;
    // input gradients: tap mirrored (8 - s), row = output channel of the
    // forward layer, column = its input channel
    case PK_DG3: return P[OFF_W3 + (k * 9 + (8 - s)) * 32 + co];
    case PK_DG2: return P[OFF_W2 + (k * 9 + (8 - s)) * 32 + co];
    case PK_DG4: return k < 9 ? P[OFF_W4 + (8 - k) * 32 + co] : 0.0f;
    }
    return 0.0f;
}

__device__ __forceinline__ void pack_one(const float *params, __bf16 *packed, int idx)
{
    int kind = 0;
    while (kind + 1 < PK_COUNT && idx >= pack_offset(kind + 1)) kind++;
    int r = idx - pack_offset(kind);
    const int e = r % 8;
    r /= 8;
    const int lane = r % 64;
    r /= 64;
    const int nb = r % pack_nb(kind);
    const int s = r / pack_nb(kind);
    const int j = lane % 16, k = (lane / 16) * 8 + e;
    packed[idx] = to_bf16(pack_value(params, kind, s, nb, j, k));
}

__global__ void pack_kernel(const float *params, __bf16 *packed)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < PACK_TOTAL) pack_one(params, packed, idx);
}

// ---------------------------------------------------------------------------
// input: window bits, short-window estimate, stability flag (+ target crop)

struct SampleTab {
    spk_sur_sample s[SPK_SUR_MAX_SAMPLES];
};

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m)
{
    const int lo = __shfl_xor((int)(uint32_t)v, m, 64);
    const int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

// 64x64 bit transpose across the wave (lane j row j -> lane i column i).
__device__ __forceinline__ uint64_t transpose64(uint64_t a, int lane)
{
    constexpr uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull,
                                   0x00FF00FF00FF00FFull, 0x0F0F0F0F0F0F0F0Full,
                                   0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int i = 0; i < 6; i++) {
        const int s = 32 >> i;
        const uint64_t y = shfl_xor64(a, s);
        const bool up = (lane & s) != 0;
        const uint64_t sh = up ? (y >> s) : (y << s);
        const uint64_t keep = up ? ~masks[i] : masks[i];
        a = (a & keep) | (sh & ~keep);
    }
    return a;
}

// FSR on a 32-frame window (bit j = frame t-31+j) valued at its last frame:
// the last segment's theta*N/D; fewer than two spikes: theta*K/32.
__device__ __forceinline__ void window_estimate(uint32_t win, double theta, float &est,
                                                uint8_t &stable)
{
    const int K = __builtin_popcount(win);
    if (K < 2) {
        est = (float)(theta * (double)K / 32.0);
        stable = 0;
        return;
    }
    uint32_t h = win;
    int last = __builtin_ctz(h);
    h &= h - 1;
    int first = last, n = 0, lo = kBig, hi = -kBig, nseg = 1;
    while (h) {
        const int pos = __builtin_ctz(h);
        h &= h - 1;
        const int x = pos - last;
        const int nlo = min(lo, x), nhi = max(hi, x);
        if (nhi - nlo > 1) {  // the interval opens a new segment at `last`
            first = last;
            n = 0;
            lo = hi = x;
            nseg++;
        } else {
            lo = nlo;
            hi = nhi;
        }
        n++;
        last = pos;
    }
    est = (float)(theta * (double)n / (double)(last - first));
    stable = nseg == 1;
}

// One 64-pixel row tile of crop b (sample S): window, estimate, flag and
// optionally the target.
__device__ __forceinline__ void input_tile(const spk_sur_sample &S, int b, int Hc, int Wc,
                                           int xtiles, double theta, uint32_t *win, float *est,
                                           uint8_t *stable, float *target)
{
    const int lane = threadIdx.x;
    const int tile = blockIdx.x;
    const int y = (tile / xtiles) % Hc;
    const int x0 = (tile % xtiles) * 64;
    const int64_t fb = (int64_t)(((int64_t)S.H * S.W + 127) / 128) * 16;
    // frame row of 64 consecutive stream pixels starting at q0 (not aligned)
    const int64_t q0 = (int64_t)(S.oy + y) * S.W + S.ox + x0;
    uint64_t row = 0;
    if (lane < 32) {
        const uint8_t *frame = S.stream + (int64_t)(S.t - 31 + lane) * fb;
        const int64_t wi = q0 >> 6;
        const int sh = (int)(q0 & 63);
        const uint64_t w0 = *(const uint64_t *)(frame + wi * 8);
        uint64_t w1 = 0;
        if (sh && (wi + 1) * 8 < fb) w1 = *(const uint64_t *)(frame + (wi + 1) * 8);
        row = sh ? (w0 >> sh) | (w1 << (64 - sh)) : w0;
    }
    const uint32_t w = (uint32_t)transpose64(row, lane);
    const int x = x0 + lane;
    if (x >= Wc) return;
    const int64_t o = ((int64_t)b * Hc + y) * Wc + x;
    float e;
    uint8_t st;
    window_estimate(w, theta, e, st);
    win[o] = w;
    est[o] = e;
    stable[o] = st;
    if (target && S.target) target[o] = S.target[(int64_t)(S.oy + y) * S.W + S.ox + x];
}

__global__ __launch_bounds__(64) void input_kernel(SampleTab tab, int Hc, int Wc, int xtiles,
                                                   double theta, uint32_t *win, float *est,
                                                   uint8_t *stable, float *target)
{
    const int b = blockIdx.x / (Hc * xtiles);
    input_tile(tab.s[b], b, Hc, Wc, xtiles, theta, win, est, stable, target);
}

// As input_kernel with the crops of training step *kstep taken from a
// device table of B records per step.  The grid also packs the weights
// (as pack_kernel), which saves the training step a launch.
__global__ __launch_bounds__(64) void input_step_kernel(const spk_sur_sample *samples,
                                                        const int32_t *kstep, int B, int Hc,
                                                        int Wc, int xtiles, double theta,
                                                        uint32_t *win, float *est,
                                                        uint8_t *stable, float *target,
                                                        const float *params, __bf16 *packed)
{
    const int64_t nthr = (int64_t)gridDim.x * 64;
    for (int64_t idx = (int64_t)blockIdx.x * 64 + threadIdx.x; idx < PACK_TOTAL; idx += nthr)
        pack_one(params, packed, (int)idx);
    const int b = blockIdx.x / (Hc * xtiles);
    const spk_sur_sample S = samples[(int64_t)*kstep * B + b];
    input_tile(S, b, Hc, Wc, xtiles, theta, win, est, stable, target);
}

// Streaming window update for a full frame: win = (win >> 1) | bit(t) << 31,
// then the estimate and flag of the new window.
__global__ __launch_bounds__(256) void stream_kernel(const uint8_t *frame, int64_t HW,
                                                     double theta, uint32_t *win, float *est,
                                                     uint8_t *stable)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= HW) return;
    const uint32_t bit = (frame[p >> 3] >> (p & 7)) & 1u;
    const uint32_t w = (win[p] >> 1) | (bit << 31);
    float e;
    uint8_t st;
    window_estimate(w, theta, e, st);
    win[p] = w;
    est[p] = e;
    stable[p] = st;
}

// ---------------------------------------------------------------------------
// convolution as implicit GEMM on MFMA

enum ConvKind {
    CK_FIRST = 0,   // bits + estimate -> 32, ReLU
    CK_MID,         // 32 -> 32, ReLU
    CK_LAST,        // 32 -> 1, linear, float32 out
    CK_DGRAD_MID,   // gradient 32 -> 32 through mirrored taps, ReLU mask
    CK_DGRAD_LAST,  // gradient 1 -> 32 through mirrored taps, ReLU mask
};

struct ConvArgs {
    int B, Hc, Wc;
    int bx, by, nblocks;    // 16x16 output blocks per row / column, in all
    const uint32_t *win;    // CK_FIRST
    const float *scalar;    // CK_FIRST, CK_LAST: estimate; CK_DGRAD_LAST: dL/dy
    const __bf16 *act;      // source activations / gradients (NHWC, 32 ch)
    const __bf16 *packed;   // this layer's packed B operand
    const float *bias;      // forward layers
    const __bf16 *mask;     // dgrad: activations whose ReLU mask applies
    __bf16 *out;            // NHWC 32 ch
    float *out_f32;         // CK_LAST
};

template <int KIND>
struct ConvShape {
    static constexpr int steps = KIND == CK_FIRST ? 10 : (KIND == CK_DGRAD_LAST ? 1 : 9);
    static constexpr int nb = KIND == CK_LAST ? 1 : 2;
};

// 8 bfloat16 ones/zeros from 8 bits (bit e -> element e).  Dword k holds
// bits 2k and 2k + 1: spread to bits 0 and 16 and multiplied by 0x3F80
// (bfloat16 1.0), three integer operations a dword.
__device__ __forceinline__ bf16x8 bits_to_bf16(uint32_t bits)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 d;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const uint32_t x = (bits >> (2 * k)) & 3u;
        d[k] = ((x | (x << 15)) & 0x10001u) * 0x3F80u;
    }
    return __builtin_bit_cast(bf16x8, d);
}

// A workgroup computes 16 x 16 blocks of output pixels, all 32 output
// channels; wave w takes block rows 4w .. 4w+3.  The 18 x 18 input halo is
// staged in LDS (NHWC bfloat16, 64 bytes per pixel, so every A fragment --
// 16 pixels x 8 channels -- is one aligned 16-byte read per lane); a scalar
// input channel (estimate, or dL/dy for the last layer's input gradient) is
// staged beside it as float.  A workgroup walks a contiguous range of
// blocks and loads the next block's halo into registers while it computes
// the current one, so the loads' latency hides behind the MFMA work.
template <int KIND>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs A)
{
    using S = ConvShape<KIND>;
    constexpr bool VEC_IN = KIND != CK_DGRAD_LAST;              // 32-channel input
    constexpr bool SCALAR_IN = KIND == CK_FIRST || KIND == CK_DGRAD_LAST;
    constexpr bool BITS_IN = KIND == CK_FIRST;                  // window words
    constexpr int kHalo = 18 * 18;
    // staging items per thread: 16-byte pieces of the 32-channel halo (for
    // the first layer, one byte of a pixel's window word, expanded to 8
    // channels) and scalar pixels; consecutive threads write consecutive
    // 16-byte pieces of LDS
    constexpr int kVecItems = kHalo * 4;
    constexpr int kVecPer = VEC_IN ? (kVecItems + 255) / 256 : 1;
    constexpr int kScPer = SCALAR_IN ? (kHalo + 255) / 256 : 1;
    constexpr int CP = C;  // pixel stride in the halo tile
    // pixel stride of the output staging rows: 40 bfloat16 puts the four
    // lane groups of one 2-byte store on two bank sets instead of one
    constexpr int SP = 40;
    __shared__ __attribute__((aligned(16))) __bf16 tin[VEC_IN ? kHalo * CP : 8];
    __shared__ float tsc[SCALAR_IN ? kHalo : 1];
    // the scalar channel's 9 taps per output pixel as bfloat16 (then 7
    // zeros): the A fragment of its K step is one 16-byte read
    __shared__ __attribute__((aligned(16))) __bf16 tcol[SCALAR_IN ? 256 * 16 : 8];
    __shared__ __attribute__((aligned(16))) __bf16 stage[4][KIND == CK_LAST ? 8 : 16 * SP];
    __shared__ float stagef[4][KIND == CK_LAST ? 64 : 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int i = lane & 15, g = lane >> 4;
    // this layer's weights, resident in registers
    bf16x8 Bop[S::steps][S::nb];
#pragma unroll
    for (int s = 0; s < S::steps; s++)
#pragma unroll
        for (int n = 0; n < S::nb; n++)
            Bop[s][n] = *(const bf16x8 *)(A.packed + ((s * S::nb + n) * 64 + lane) * 8);
    float bias[S::nb];
#pragma unroll
    for (int n = 0; n < S::nb; n++) {
        bias[n] = 0.0f;
        if constexpr (KIND == CK_FIRST || KIND == CK_MID) bias[n] = A.bias[n * 16 + i];
        if constexpr (KIND == CK_LAST) bias[n] = A.bias[0];
    }
    // the halo of the next block, in flight in registers
    uint32_t pw[BITS_IN ? kVecPer : 1];
    bf16x8 pv[VEC_IN && !BITS_IN ? kVecPer : 1];
    float ps[kScPer];
    auto load = [&](int blk) {
        const int b = blk / (A.bx * A.by);
        const int y0 = ((blk / A.bx) % A.by) * 16, x0 = (blk % A.bx) * 16;
        if constexpr (VEC_IN) {
#pragma unroll
            for (int u = 0; u < kVecPer; u++) {
                const int it = tid + 256 * u;
                const int q = it >> 2, part = it & 3;
                const int y = y0 - 1 + q / 18, x = x0 - 1 + q % 18;
                const bool in =
                    it < kVecItems && y >= 0 && y < A.Hc && x >= 0 && x < A.Wc;
                const int64_t pix = ((int64_t)b * A.Hc + y) * A.Wc + x;
                if constexpr (BITS_IN) {
                    pw[u] = in ? A.win[pix] : 0u;
                } else {
                    bf16x8 v;
#pragma unroll
                    for (int e = 0; e < 8; e++) v[e] = (__bf16)0.0f;
                    if (in) v = *(const bf16x8 *)(A.act + pix * C + part * 8);
                    pv[u] = v;
                }
            }
        }
        if constexpr (SCALAR_IN) {
#pragma unroll
            for (int u = 0; u < kScPer; u++) {
                const int q = tid + 256 * u;
                const int y = y0 - 1 + q / 18, x = x0 - 1 + q % 18;
                const bool in = q < kHalo && y >= 0 && y < A.Hc && x >= 0 && x < A.Wc;
                ps[u] = in ? A.scalar[((int64_t)b * A.Hc + y) * A.Wc + x] : 0.0f;
            }
        }
    };
    auto store = [&]() {
        if constexpr (VEC_IN) {
#pragma unroll
            for (int u = 0; u < kVecPer; u++) {
                const int it = tid + 256 * u;
                if (it < kVecItems) {
                    if constexpr (BITS_IN) {
                        *(bf16x8 *)(&tin[(it >> 2) * CP + (it & 3) * 8]) =
                            bits_to_bf16((pw[u] >> (8 * (it & 3))) & 0xFFu);
                    } else {
                        *(bf16x8 *)(&tin[(it >> 2) * CP + (it & 3) * 8]) = pv[u];
                    }
                }
            }
        }
        if constexpr (SCALAR_IN) {
#pragma unroll
            for (int u = 0; u < kScPer; u++) {
                const int q = tid + 256 * u;
                if (q < kHalo) tsc[q] = ps[u];
            }
        }
    };
    const int per = (A.nblocks + (int)gridDim.x - 1) / (int)gridDim.x;
    const int blk0 = (int)blockIdx.x * per, blk1 = min(A.nblocks, blk0 + per);
    if (blk0 >= blk1) return;
    auto build_col = [&]() {
        if constexpr (SCALAR_IN) {
            const int oy = tid >> 4, ox = tid & 15;
            bf16x8 lo, hi;
#pragma unroll
            for (int e = 0; e < 8; e++) {
                lo[e] = (__bf16)tsc[(oy + e / 3) * 18 + ox + e % 3];
                hi[e] = (__bf16)0.0f;
            }
            hi[0] = (__bf16)tsc[(oy + 2) * 18 + ox + 2];
            *(bf16x8 *)(&tcol[tid * 16]) = lo;
            *(bf16x8 *)(&tcol[tid * 16 + 8]) = hi;
        }
    };
    load(blk0);
    store();
    __syncthreads();
    if constexpr (SCALAR_IN) {
        build_col();
        __syncthreads();
    }
    // output staging rows: pixel lane/4, channels 8 (lane%4) .. +7
    const int px = lane >> 2, part = lane & 3;
    for (int blk = blk0; blk < blk1; blk++) {
        const int b = blk / (A.bx * A.by);
        const int y0 = ((blk / A.bx) % A.by) * 16, x0 = (blk % A.bx) * 16;
        // the halo of this block (rows y0-1 .. y0+16, columns x0-1 .. x0+16)
        // is in LDS; fetch the next one while computing
        const bool more = blk + 1 < blk1;
        if (more) load(blk + 1);
        // the last layer's residual: the estimate at this lane's pixel of
        // the wave's rows (row 4w + lane/16, column lane%16)
        float est_l = 0.0f;
        const int ly = y0 + 4 * wave + (lane >> 4), lx = x0 + (lane & 15);
        const bool lin = ly < A.Hc && lx < A.Wc;
        const int64_t lpix = ((int64_t)b * A.Hc + ly) * A.Wc + lx;
        if constexpr (KIND == CK_LAST) {
            if (lin) est_l = A.scalar[lpix];
        }
        // input gradients: the ReLU masks of this block's output rows, loaded
        // here so that they arrive during the MFMA work
        bf16x8 om[KIND == CK_DGRAD_MID || KIND == CK_DGRAD_LAST ? 4 : 1];
        if constexpr (KIND == CK_DGRAD_MID || KIND == CK_DGRAD_LAST) {
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int y = y0 + 4 * wave + r, x = x0 + px;
#pragma unroll
                for (int e = 0; e < 8; e++) om[r][e] = (__bf16)0.0f;
                if (x < A.Wc && y < A.Hc)
                    om[r] = *(const bf16x8 *)(A.mask + (((int64_t)b * A.Hc + y) * A.Wc + x) * C +
                                              part * 8);
            }
        }
        f32x4 acc[4][S::nb];
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int n = 0; n < S::nb; n++) acc[r][n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        // 32-channel taps: the fragment of halo row 4w + iy shifted by dx
        // is read once and serves every output row r with dy = iy - r in
        // 0..2 (tap s = 3 dy + dx), 18 reads for 36 row-taps.  Each
        // accumulator still takes its taps in the order s = 0 .. 8.
        if constexpr (VEC_IN) {
#pragma unroll
            for (int iy = 0; iy < 6; iy++)
#pragma unroll
                for (int dx = 0; dx < 3; dx++) {
                    const bf16x8 a =
                        *(const bf16x8 *)(&tin[((4 * wave + iy) * 18 + i + dx) * CP + 8 * g]);
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int dy = iy - r;
                        if (dy < 0 || dy > 2) continue;
#pragma unroll
                        for (int n = 0; n < S::nb; n++)
                            acc[r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                a, Bop[3 * dy + dx][n], acc[r][n], 0, 0, 0);
                    }
                }
        }
        // the scalar channel's step (last): row k of the K block = tap k
        if constexpr (SCALAR_IN) {
            constexpr int s = S::steps - 1;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int oy = 4 * wave + r;  // block row of the output
                bf16x8 a;
                if (g < 2) {
                    a = *(const bf16x8 *)(&tcol[(oy * 16 + i) * 16 + 8 * g]);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; e++) a[e] = (__bf16)0.0f;
                }
#pragma unroll
                for (int n = 0; n < S::nb; n++)
                    acc[r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, Bop[s][n], acc[r][n], 0, 0, 0);
            }
        }
        // Epilogue, first half: the results into registers in store layout
        // (lane holds D[pixel 4g + e][channel 16n + i] of each block row).
        // Global stores wait until the next halo is in LDS: its loads are
        // then the only memory operations outstanding.
        bf16x8 ov[KIND == CK_LAST ? 1 : 4];
        float of = 0.0f;
        if constexpr (KIND == CK_LAST) {
            if (i == 0) {
#pragma unroll
                for (int r = 0; r < 4; r++)
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        stagef[wave][r * 16 + 4 * g + e] = acc[r][0][e] + bias[0];
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            of = stagef[wave][lane];
        } else {
#pragma unroll
            for (int r = 0; r < 4; r++) {
#pragma unroll
                for (int n = 0; n < S::nb; n++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        float v = acc[r][n][e] + bias[n];
                        if constexpr (KIND == CK_FIRST || KIND == CK_MID) v = fmaxf(v, 0.0f);
                        stage[wave][(4 * g + e) * SP + 16 * n + i] = to_bf16(v);
                    }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                ov[r] = *(const bf16x8 *)(&stage[wave][px * SP + part * 8]);
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        // (more is the same for the whole workgroup, so the barriers are too)
        if (more) {
            __syncthreads();  // every wave is done with this halo
            store();
        }
        if constexpr (SCALAR_IN) {
            if (more) {
                __syncthreads();  // the next halo's scalar channel is in LDS
                build_col();
            }
        }
        // second half: global stores
        if constexpr (KIND == CK_LAST) {
            if (lin) A.out_f32[lpix] = est_l + of;
        } else {
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int y = y0 + 4 * wave + r, x = x0 + px;
                if (x < A.Wc && y < A.Hc) {
                    bf16x8 v = ov[r];
                    if constexpr (KIND == CK_DGRAD_MID || KIND == CK_DGRAD_LAST) {
#pragma unroll
                        for (int e = 0; e < 8; e++)
                            if (!((float)om[r][e] > 0.0f)) v[e] = (__bf16)0.0f;
                    }
                    *(bf16x8 *)(A.out + (((int64_t)b * A.Hc + y) * A.Wc + x) * C + part * 8) = v;
                }
            }
        }
        if (more) __syncthreads();  // the next halo is in LDS
    }
}

// ---------------------------------------------------------------------------
// loss: dL/dy = 2 (y - target) / N, rounded to bfloat16 like every gradient
// the GEMMs consume; per-block partial sums of the squared error

// partial: one sum per block; with kstep, step *kstep's row of a table
// [step][gridDim.x].
__global__ __launch_bounds__(256) void loss_kernel(const float *y, const float *tgt, int64_t n,
                                                   float *dy, float *partial,
                                                   const int32_t *kstep)
{
    __shared__ float red[256];
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float sq = 0.0f;
    if (idx < n) {
        const float d = y[idx] - tgt[idx];
        sq = d * d;
        dy[idx] = (float)to_bf16(2.0f * d / (float)n);
    }
    // tree sum, element t taking t + s for s = 128, 64, ..., 1; the last
    // six halvings within one wave by shuffles (the same additions)
    red[threadIdx.x] = sq;
    __syncthreads();
    if (threadIdx.x < 128) red[threadIdx.x] += red[threadIdx.x + 128];
    __syncthreads();
    if (threadIdx.x < 64) {
        float v = red[threadIdx.x] + red[threadIdx.x + 64];
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) v += __shfl_down(v, s, 64);
        if (threadIdx.x == 0)
            partial[(kstep ? (int64_t)*kstep * gridDim.x : 0) + blockIdx.x] = v;
    }
}

// ---------------------------------------------------------------------------
// weight gradients on MFMA: for each tap, dW[co][tap][ci] = sum_p g[p][co] *
// a[p + off(tap)][ci] is a GEMM with M = output channels, N = input
// channels and K = pixels.  A workgroup walks 16x16-pixel tiles (grid
// stride) and stages per tile, channel-major in LDS, the operand without a
// halo (K contiguous) and the operand with the 18x18 halo once per
// horizontal tap offset, so that every fragment (8 consecutive pixels of
// one channel) is an aligned 16-byte LDS read; each channel row is padded
// by 16 bytes against bank conflicts.  The hidden layers (wgrad_kernel)
// stage the gradients plain and the activations with the halo.  Layers 1
// and 4 index by q = p + off(tap) instead, which moves the halo to the
// gradient: for layer 1 that spares expanding the window bits of three
// halo copies, for layer 4 (one output channel) it gives M = input
// channels.  Accumulators stay in registers across the tiles a workgroup
// walks; bias gradients are column sums of the gradient tile.  Each
// workgroup writes one partial gradient; reduce_kernel adds the partials
// in a fixed order.

enum WgKind { WG_FIRST = 0, WG_MID, WG_LAST };

template <int K>
struct WgShape {
    static constexpr int cout = K == WG_LAST ? 1 : 32;
    static constexpr int cin = K == WG_FIRST ? 33 : 32;
    static constexpr int nw = cout * 9 * cin;       // weights
    static constexpr int np = nw + cout;            // + biases
};

struct WgArgs {
    int B, Hc, Wc, tx, ty;       // tiles per row / column
    int ntiles;
    const __bf16 *g;             // NHWC 32 ch gradients (WG_FIRST, WG_MID)
    const float *gy;             // dL/dy (WG_LAST)
    const __bf16 *a;             // NHWC 32 ch activations (WG_MID, WG_LAST)
    const uint32_t *win;         // WG_FIRST
    const float *est;            // WG_FIRST
    float *partial;              // [gridDim.x][np]
};

// Workgroups of a weight-gradient launch: two per CU are resident (74 KB
// of LDS each), and 512 give each one several tiles to pipeline its loads
// over while halving the partial rows against 1024 (64 x 128 x 128 step:
// 0.548 -> 0.518 ms; 256 workgroups: 0.615 ms).
constexpr int kWgMaxBlocks = 512;

// The hidden layers (32 -> 32).
__global__ __launch_bounds__(256) void wgrad_kernel(WgArgs A)
{
    using S = WgShape<WG_MID>;
    // rows padded by 16 bytes: the 16 lanes of one fragment read sit on
    // distinct banks (unpadded, the 512- and 576-byte strides put every
    // fourth lane, or all of them, on the same banks)
    __shared__ __attribute__((aligned(16))) __bf16 gT[32][256 + 8];
    __shared__ __attribute__((aligned(16))) __bf16 aT[3][32][18 * 16 + 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i = lane & 15, gq = lane >> 4;
    // this wave's blocks
    const int cb = wave >> 1, jb = wave & 1;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; t++) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;  // bias partial of thread tid: channel tid / 8, pixels (tid % 8) * 32 ..

    // A tile's global data goes through registers: the loads of tile k + 1
    // are issued before tile k's MFMAs, and written to LDS (transposed)
    // once those are done, so their latency hides behind the MFMA work.
    // Staging items per thread: the gradient tile as piece tid (4 pixels x
    // 8 channels), the activation halo as (dx, part, r, seg) pieces of 8
    // pixels x 8 channels.
    constexpr int kATotal = 3 * 4 * 18 * 2;
    constexpr int kAItems = (kATotal + 255) / 256;
    uint32_t gr[4][4];
    uint32_t ar[kAItems][8][4];
    auto load_tile = [&](int tile) {
        const int b = tile / (A.tx * A.ty);
        const int ty0 = ((tile / A.tx) % A.ty) * 16, tx0 = (tile % A.tx) * 16;
        {
            const int seg = tid & 63, part = tid >> 6, px0 = 4 * seg;
            const int y = ty0 + px0 / 16;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int x = tx0 + px0 % 16 + j;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (y < A.Hc && x < A.Wc)
                    v = *(const uint4 *)(A.g + (((int64_t)b * A.Hc + y) * A.Wc + x) * C + part * 8);
                gr[j][0] = v.x;
                gr[j][1] = v.y;
                gr[j][2] = v.z;
                gr[j][3] = v.w;
            }
        }
#pragma unroll
        for (int u = 0; u < kAItems; u++) {
            const int it = tid + 256 * u;
            const int seg = it & 1, r = (it >> 1) % 18, rest = (it >> 1) / 18;
            const int part = rest & 3, dx = rest >> 2, cc0 = 8 * seg;
            const int y = ty0 - 1 + r;
            const bool yin = it < kATotal && y >= 0 && y < A.Hc;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int x = tx0 - 1 + cc0 + dx + j;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (yin && x >= 0 && x < A.Wc)
                    v = *(const uint4 *)(A.a + (((int64_t)b * A.Hc + y) * A.Wc + x) * C + part * 8);
                ar[u][j][0] = v.x;
                ar[u][j][1] = v.y;
                ar[u][j][2] = v.z;
                ar[u][j][3] = v.w;
            }
        }
    };
    // the registers of the loaded tile into LDS, channel-major: channel
    // vectors transposed in registers and written as channel rows
    auto commit_tile = [&]() {
        {
            const int seg = tid & 63, part = tid >> 6, px0 = 4 * seg;
#pragma unroll
            for (int e2 = 0; e2 < 4; e2++) {
                uint2 lo, hi;  // channels 2 e2 and 2 e2 + 1, pixels 0 .. 3
                lo.x = (gr[0][e2] & 0xFFFFu) | (gr[1][e2] << 16);
                lo.y = (gr[2][e2] & 0xFFFFu) | (gr[3][e2] << 16);
                hi.x = (gr[0][e2] >> 16) | (gr[1][e2] & 0xFFFF0000u);
                hi.y = (gr[2][e2] >> 16) | (gr[3][e2] & 0xFFFF0000u);
                *(uint2 *)(&gT[part * 8 + 2 * e2][px0]) = lo;
                *(uint2 *)(&gT[part * 8 + 2 * e2 + 1][px0]) = hi;
            }
        }
#pragma unroll
        for (int u = 0; u < kAItems; u++) {
            const int it = tid + 256 * u;
            if (it >= kATotal) continue;
            const int seg = it & 1, r = (it >> 1) % 18, rest = (it >> 1) / 18;
            const int part = rest & 3, dx = rest >> 2, cc0 = 8 * seg;
#pragma unroll
            for (int e2 = 0; e2 < 4; e2++) {
                uint4 lo, hi;  // channels 2 e2 and 2 e2 + 1, pixels 0 .. 7
                lo.x = (ar[u][0][e2] & 0xFFFFu) | (ar[u][1][e2] << 16);
                lo.y = (ar[u][2][e2] & 0xFFFFu) | (ar[u][3][e2] << 16);
                lo.z = (ar[u][4][e2] & 0xFFFFu) | (ar[u][5][e2] << 16);
                lo.w = (ar[u][6][e2] & 0xFFFFu) | (ar[u][7][e2] << 16);
                hi.x = (ar[u][0][e2] >> 16) | (ar[u][1][e2] & 0xFFFF0000u);
                hi.y = (ar[u][2][e2] >> 16) | (ar[u][3][e2] & 0xFFFF0000u);
                hi.z = (ar[u][4][e2] >> 16) | (ar[u][5][e2] & 0xFFFF0000u);
                hi.w = (ar[u][6][e2] >> 16) | (ar[u][7][e2] & 0xFFFF0000u);
                *(uint4 *)(&aT[dx][part * 8 + 2 * e2][r * 16 + cc0]) = lo;
                *(uint4 *)(&aT[dx][part * 8 + 2 * e2 + 1][r * 16 + cc0]) = hi;
            }
        }
    };

    if ((int)blockIdx.x < A.ntiles) load_tile(blockIdx.x);
    for (int tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
        commit_tile();
        __syncthreads();
        if (tile + (int)gridDim.x < A.ntiles) load_tile(tile + gridDim.x);
        // K steps s (32 pixels each) outside, taps inside: one A fragment
        // (gradients of channel cb*16 + i, pixels 32s + 8gq .. +7) at a
        // time, and nine independent accumulators back to back
#pragma unroll
        for (int s = 0; s < 8; s++) {
            const bf16x8 Af = *(const bf16x8 *)(&gT[cb * 16 + i][32 * s + 8 * gq]);
#pragma unroll
            for (int t = 0; t < 9; t++) {
                const int dy = t / 3, dx = t % 3;
                // pixels 32s + 8gq .. +7: tile row 2s + gq/2, columns 8(gq&1) ..
                const int row = 2 * s + (gq >> 1) + dy, col = 8 * (gq & 1);
                const bf16x8 Bf = *(const bf16x8 *)(&aT[dx][jb * 16 + i][row * 16 + col]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Af, Bf, acc[t], 0, 0, 0);
            }
        }
        // bias: column sums of the gradient tile (pixels (tid % 8) * 32 ..
        // +31 of channel tid / 8, in order, four 16-byte reads)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const bf16x8 v = *(const bf16x8 *)(&gT[tid / 8][(tid % 8) * 32 + 8 * q]);
#pragma unroll
            for (int e = 0; e < 8; e++) bsum += (float)v[e];
        }
        __syncthreads();
    }
    // partial gradient of this workgroup, in the parameter blob's order
    float *out = A.partial + (int64_t)blockIdx.x * S::np;
#pragma unroll
    for (int t = 0; t < 9; t++) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            // D[co 4*(lane/16) + r][ci lane%16] of this wave's blocks
            const int co = cb * 16 + 4 * gq + r, ci = jb * 16 + i;
            out[(co * 9 + t) * S::cin + ci] = acc[t][r];
        }
    }
    // bias sums: 8 threads per channel, combined in a fixed order
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) bsum += __shfl_xor(bsum, m, 64);
    if (tid % 8 == 0) out[S::nw + tid / 8] = bsum;
}

// Weight gradient of the first layer.  Written with q = p + off(tap),
// dW[co][tap][ci] = sum_q g[q - off(tap)][co] x[q][ci] is, per tap, a GEMM
// with M = output channels, N = the 32 window-bit channels and K = pixels.
// The input channels then need no halo -- each tile's window bits are
// expanded to bfloat16 once, 8 x 8 bit transposes into channel-major rows
// -- and the 32-channel gradient carries the halo, staged like the hidden
// layers' activations (three copies shifted by the horizontal tap offset,
// so every fragment is an aligned 16-byte read).  Wave w takes output
// block w >> 1 and input block w & 1 for all taps.  The estimate channel
// is one GEMM for all taps, dW[co][tap] = sum_p g[p][co] est[p + off(tap)]
// with N = taps (9 of 16): the gradient's unshifted fragment against the
// estimate's halo, staged in three shifted bfloat16 copies; the waves with
// input block 0 run it.  The next tile's loads are in flight while the
// current one is computed.  Partial row as wgrad_kernel's.
__global__ __launch_bounds__(256) void wgrad_first_kernel(WgArgs A)
{
    using S = WgShape<WG_FIRST>;
    static_assert(S::cout == 32 && S::cin == 33, "first layer");
    __shared__ __attribute__((aligned(16))) __bf16 xT[32][256 + 8];
    __shared__ __attribute__((aligned(16))) __bf16 gH[3][32][18 * 16 + 8];
    // the estimate's 18 x 18 halo as bfloat16, copy d holding columns
    // d .. d + 15
    __shared__ __attribute__((aligned(16))) __bf16 eH[3][18][16];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int i = lane & 15, gq = lane >> 4;
    const int cb = wave >> 1, jb = wave & 1;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; t++) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // the estimate channel (waves with jb == 0): D[co][tap] of block cb
    f32x4 acce = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;  // bias partial of thread tid: channel tid / 8, pixels (tid % 8) * 32 ..
    // registers of the next tile: window words of piece (part, seg) (threads
    // 0 .. 127: 8 pixels, byte `part`), two estimate-halo values, and two
    // gradient-halo pieces (dx, part, r, seg) of 8 pixels x 8 channels
    constexpr int kHTotal = 3 * 4 * 18 * 2;
    constexpr int kHItems = (kHTotal + 255) / 256;
    uint32_t xw[8];
    float xe[2];
    uint32_t hr_[kHItems][8][4];
    auto load_tile = [&](int tile) {
        const int b = tile / (A.tx * A.ty);
        const int ty0 = ((tile / A.tx) % A.ty) * 16, tx0 = (tile % A.tx) * 16;
        {
            const int seg = tid & 31, px0 = 8 * seg;
            const int y = ty0 + px0 / 16;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int x = tx0 + px0 % 16 + j;
                xw[j] = tid < 128 && y < A.Hc && x < A.Wc
                            ? A.win[((int64_t)b * A.Hc + y) * A.Wc + x]
                            : 0u;
            }
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int q = tid + 256 * u;
                const int ye = ty0 - 1 + q / 18, xe_ = tx0 - 1 + q % 18;
                xe[u] = q < 18 * 18 && ye >= 0 && ye < A.Hc && xe_ >= 0 && xe_ < A.Wc
                            ? A.est[((int64_t)b * A.Hc + ye) * A.Wc + xe_]
                            : 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < kHItems; u++) {
            const int it = tid + 256 * u;
            const int seg = it & 1, r = (it >> 1) % 18, rest = (it >> 1) / 18;
            const int part = rest & 3, dx = rest >> 2, cc0 = 8 * seg;
            const int y = ty0 - 1 + r;
            const bool yin = it < kHTotal && y >= 0 && y < A.Hc;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int x = tx0 - 1 + cc0 + dx + j;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (yin && x >= 0 && x < A.Wc)
                    v = *(const uint4 *)(A.g + (((int64_t)b * A.Hc + y) * A.Wc + x) * C + part * 8);
                hr_[u][j][0] = v.x;
                hr_[u][j][1] = v.y;
                hr_[u][j][2] = v.z;
                hr_[u][j][3] = v.w;
            }
        }
    };
    auto commit_tile = [&]() {
        if (tid < 128) {
            // byte `part` of 8 pixels' windows, 8 x 8 bit transposed into the
            // rows of channels part*8 .. +7 (bfloat16 ones and zeros)
            const int seg = tid & 31, part = tid >> 5, px0 = 8 * seg;
            uint64_t m = 0;  // byte j: pixel j's channels part*8 .. +7
#pragma unroll
            for (int j = 0; j < 8; j++) m |= (uint64_t)((xw[j] >> (8 * part)) & 0xFFu) << (8 * j);
            uint64_t t = (m ^ (m >> 7)) & 0x00AA00AA00AA00AAull;
            m ^= t ^ (t << 7);
            t = (m ^ (m >> 14)) & 0x0000CCCC0000CCCCull;
            m ^= t ^ (t << 14);
            t = (m ^ (m >> 28)) & 0x00000000F0F0F0F0ull;
            m ^= t ^ (t << 28);
#pragma unroll
            for (int e = 0; e < 8; e++)
                *(bf16x8 *)(&xT[part * 8 + e][px0]) = bits_to_bf16((uint32_t)(m >> (8 * e)) & 0xFFu);
        }
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int q = tid + 256 * u;
            if (q < 18 * 18) {
                const int hr = q / 18, hc = q % 18;
                const __bf16 v = to_bf16(xe[u]);
#pragma unroll
                for (int d = 0; d < 3; d++)
                    if (hc - d >= 0 && hc - d < 16) eH[d][hr][hc - d] = v;
            }
        }
#pragma unroll
        for (int u = 0; u < kHItems; u++) {
            const int it = tid + 256 * u;
            if (it >= kHTotal) continue;
            const int seg = it & 1, r = (it >> 1) % 18, rest = (it >> 1) / 18;
            const int part = rest & 3, dx = rest >> 2, cc0 = 8 * seg;
#pragma unroll
            for (int e2 = 0; e2 < 4; e2++) {
                uint4 lo, hi;  // channels 2 e2 and 2 e2 + 1, pixels 0 .. 7
                lo.x = (hr_[u][0][e2] & 0xFFFFu) | (hr_[u][1][e2] << 16);
                lo.y = (hr_[u][2][e2] & 0xFFFFu) | (hr_[u][3][e2] << 16);
                lo.z = (hr_[u][4][e2] & 0xFFFFu) | (hr_[u][5][e2] << 16);
                lo.w = (hr_[u][6][e2] & 0xFFFFu) | (hr_[u][7][e2] << 16);
                hi.x = (hr_[u][0][e2] >> 16) | (hr_[u][1][e2] & 0xFFFF0000u);
                hi.y = (hr_[u][2][e2] >> 16) | (hr_[u][3][e2] & 0xFFFF0000u);
                hi.z = (hr_[u][4][e2] >> 16) | (hr_[u][5][e2] & 0xFFFF0000u);
                hi.w = (hr_[u][6][e2] >> 16) | (hr_[u][7][e2] & 0xFFFF0000u);
                *(uint4 *)(&gH[dx][part * 8 + 2 * e2][r * 16 + cc0]) = lo;
                *(uint4 *)(&gH[dx][part * 8 + 2 * e2 + 1][r * 16 + cc0]) = hi;
            }
        }
    };

    if ((int)blockIdx.x < A.ntiles) load_tile(blockIdx.x);
    for (int tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
        commit_tile();
        __syncthreads();
        if (tile + (int)gridDim.x < A.ntiles) load_tile(tile + gridDim.x);
#pragma unroll
        for (int s = 0; s < 8; s++) {
            // pixels q = 32s + 8gq .. +7: tile row 2s + gq/2, columns 8(gq&1) ..
            const int row = 2 * s + (gq >> 1), col = 8 * (gq & 1);
            const bf16x8 Bf = *(const bf16x8 *)(&xT[jb * 16 + i][32 * s + 8 * gq]);
#pragma unroll
            for (int t = 0; t < 9; t++) {
                // the gradient for q at tap (dy, dx) is at halo (row + 2 - dy,
                // col + 2 - dx): copy 2 - dx
                const int dy = t / 3, dx = t % 3;
                const bf16x8 Af =
                    *(const bf16x8 *)(&gH[2 - dx][cb * 16 + i][(row + 2 - dy) * 16 + col]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Af, Bf, acc[t], 0, 0, 0);
                if (t == 4 && jb == 0) {
                    // estimate channel, un-substituted: dW[co][tap] =
                    // sum_p g[p][co] est[p + off(tap)], A = the gradient at
                    // p (tap 4's fragment), B column i = tap i, read at halo
                    // (row + dy', col + dx') of the estimate
                    bf16x8 Be;
#pragma unroll
                    for (int e = 0; e < 8; e++) Be[e] = (__bf16)0.0f;
                    if (i < 9) Be = *(const bf16x8 *)(&eH[i % 3][row + i / 3][col]);
                    acce = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Af, Be, acce, 0, 0, 0);
                }
            }
        }
        // bias: column sums of the tile's gradients (copy 1 holds tile
        // columns 0 .. 15 in halo rows 1 .. 16), the tile's pixels in order
        {
            const int co = tid / 8, prt = tid % 8;
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int hrow = 1 + 2 * prt + h;
#pragma unroll
                for (int q = 0; q < 2; q++) {
                    const bf16x8 v = *(const bf16x8 *)(&gH[1][co][hrow * 16 + 8 * q]);
#pragma unroll
                    for (int e = 0; e < 8; e++) bsum += (float)v[e];
                }
            }
        }
        __syncthreads();
    }
    // partial gradient of this workgroup, in the parameter blob's order
    float *out = A.partial + (int64_t)blockIdx.x * S::np;
#pragma unroll
    for (int t = 0; t < 9; t++) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            // D[co 4*(lane/16) + r][ci lane%16] of this wave's blocks
            const int co = cb * 16 + 4 * gq + r, ci = jb * 16 + i;
            out[(co * 9 + t) * S::cin + ci] = acc[t][r];
        }
    }
    // D[co 4*(lane/16) + r][tap lane%16] of the estimate channel
    if (jb == 0 && i < 9) {
#pragma unroll
        for (int r = 0; r < 4; r++)
            out[((cb * 16 + 4 * gq + r) * 9 + i) * S::cin + 32] = acce[r];
    }
    // bias sums: 8 threads per channel, combined in a fixed order
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) bsum += __shfl_xor(bsum, m, 64);
    if (tid % 8 == 0) out[S::nw + tid / 8] = bsum;
}

// Weight gradient of the output layer (one output channel).  Written with
// q = p + off(tap), dW[tap][ci] = sum_q a[q][ci] gy[q - off(tap)] is a GEMM
// with M = input channels (32), N = taps (9 of 16) and K = pixels: the
// activations need no halo, only the one-channel gradient does.  Per
// 16x16 tile a workgroup stages the activations channel-major and the
// gradient's 18x18 halo as bfloat16 in three copies shifted by the
// horizontal tap offset, so that every fragment is an aligned 16-byte LDS
// read.  Wave w takes K steps 2w and 2w + 1 (64 of the tile's pixels) for
// both channel blocks; the four waves' sums are added at the end.  The
// next tile's loads are in flight while the current one is computed.
// Partial row: dW in the parameter blob's order, then the bias (the sum of
// the bfloat16 gradients).
__global__ __launch_bounds__(256) void wgrad_last_kernel(WgArgs A)
{
    using S = WgShape<WG_LAST>;
    static_assert(S::cout == 1 && S::cin == 32, "output layer");
    __shared__ __attribute__((aligned(16))) __bf16 aT[32][256 + 8];
    __shared__ __attribute__((aligned(16))) __bf16 gH[3][18][16];
    __shared__ float red[4][2][4][64];
    __shared__ float bred[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int i = lane & 15, gq = lane >> 4;
    f32x4 acc[2] = {f32x4{0.0f, 0.0f, 0.0f, 0.0f}, f32x4{0.0f, 0.0f, 0.0f, 0.0f}};
    float bsum = 0.0f;  // this thread's pixel of every tile
    // registers of the next tile: activations (4 pixels x 8 channels,
    // piece tid), two halo values, the thread's own gradient
    uint32_t ar[4][4];
    float hv[2], gc;
    auto load_tile = [&](int tile) {
        const int b = tile / (A.tx * A.ty);
        const int ty0 = ((tile / A.tx) % A.ty) * 16, tx0 = (tile % A.tx) * 16;
        {
            const int seg = tid & 63, part = tid >> 6, px0 = 4 * seg;
            const int y = ty0 + px0 / 16;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int x = tx0 + px0 % 16 + j;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (y < A.Hc && x < A.Wc)
                    v = *(const uint4 *)(A.a + (((int64_t)b * A.Hc + y) * A.Wc + x) * C + part * 8);
                ar[j][0] = v.x;
                ar[j][1] = v.y;
                ar[j][2] = v.z;
                ar[j][3] = v.w;
            }
        }
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int q = tid + 256 * u;
            const int y = ty0 - 1 + q / 18, x = tx0 - 1 + q % 18;
            hv[u] = q < 18 * 18 && y >= 0 && y < A.Hc && x >= 0 && x < A.Wc
                        ? A.gy[((int64_t)b * A.Hc + y) * A.Wc + x]
                        : 0.0f;
        }
        const int y = ty0 + tid / 16, x = tx0 + tid % 16;
        gc = y < A.Hc && x < A.Wc ? A.gy[((int64_t)b * A.Hc + y) * A.Wc + x] : 0.0f;
    };
    auto commit_tile = [&]() {
        const int seg = tid & 63, part = tid >> 6, px0 = 4 * seg;
#pragma unroll
        for (int e2 = 0; e2 < 4; e2++) {
            uint2 lo, hi;  // channels 2 e2 and 2 e2 + 1, pixels 0 .. 3
            lo.x = (ar[0][e2] & 0xFFFFu) | (ar[1][e2] << 16);
            lo.y = (ar[2][e2] & 0xFFFFu) | (ar[3][e2] << 16);
            hi.x = (ar[0][e2] >> 16) | (ar[1][e2] & 0xFFFF0000u);
            hi.y = (ar[2][e2] >> 16) | (ar[3][e2] & 0xFFFF0000u);
            *(uint2 *)(&aT[part * 8 + 2 * e2][px0]) = lo;
            *(uint2 *)(&aT[part * 8 + 2 * e2 + 1][px0]) = hi;
        }
        // halo value (hr, hc) into copy d at column hc - d
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const int q = tid + 256 * u;
            if (q < 18 * 18) {
                const int hr = q / 18, hc = q % 18;
                const __bf16 v = to_bf16(hv[u]);
#pragma unroll
                for (int d = 0; d < 3; d++)
                    if (hc - d >= 0 && hc - d < 16) gH[d][hr][hc - d] = v;
            }
        }
        bsum += (float)to_bf16(gc);
    };

    if ((int)blockIdx.x < A.ntiles) load_tile(blockIdx.x);
    for (int tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
        commit_tile();
        __syncthreads();
        if (tile + (int)gridDim.x < A.ntiles) load_tile(tile + gridDim.x);
#pragma unroll
        for (int ss = 0; ss < 2; ss++) {
            const int s = 2 * wave + ss;
            // pixels 32s + 8gq .. +7: tile row 2s + gq/2, columns 8(gq&1) ..
            const int row = 2 * s + (gq >> 1), col = 8 * (gq & 1);
            // B: column i is tap i = 3 dy + dx, whose gradient for
            // activation pixel q sits at halo (row + 2 - dy, col + 2 - dx)
            bf16x8 Bf;
#pragma unroll
            for (int e = 0; e < 8; e++) Bf[e] = (__bf16)0.0f;
            if (i < 9) {
                const int dy = i / 3, dx = i % 3;
                Bf = *(const bf16x8 *)(&gH[2 - dx][row + 2 - dy][col]);
            }
#pragma unroll
            for (int cb = 0; cb < 2; cb++) {
                const bf16x8 Af = *(const bf16x8 *)(&aT[cb * 16 + i][32 * s + 8 * gq]);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Af, Bf, acc[cb], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // the four waves' sums, in wave order
#pragma unroll
    for (int cb = 0; cb < 2; cb++)
#pragma unroll
        for (int r = 0; r < 4; r++) red[wave][cb][r][lane] = acc[cb][r];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) bsum += __shfl_xor(bsum, m, 64);
    if (lane == 0) bred[wave] = bsum;
    __syncthreads();
    float *out = A.partial + (int64_t)blockIdx.x * S::np;
    if (wave == 0) {
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                // D[ci 4*(lane/16) + r][tap lane%16] of channel block cb
                const float v = ((red[0][cb][r][lane] + red[1][cb][r][lane]) +
                                 red[2][cb][r][lane]) + red[3][cb][r][lane];
                if (i < 9) out[i * S::cin + cb * 16 + 4 * gq + r] = v;
            }
        if (lane == 0) out[S::nw] = ((bred[0] + bred[1]) + bred[2]) + bred[3];
    }
}

// The weight-gradient partials of every layer, reduced by one launch:
// segment s sums partial[blk][j] (nblocks rows of np) into dst[j]; its
// weights start at reduce workgroup blk0.
struct RedSeg {
    const float *partial;
    float *dst;
    int np, blk0;
    int poff;  // parameter index of dst[0]
};
// Training plans: the reduction also takes Adam's step on every weight it
// finishes (learning rate and bias corrections from per-step tables).
// Each workgroup counts the steps in a counter of its own (kblk[workgroup],
// read and advanced by that workgroup alone), and workgroup 0 also advances
// *kstep, the count the step's earlier kernels read: they have finished by
// then, and no workgroup of the reduction reads it.  Every counter starts
// at zero.
struct RedAdam {
    float *p, *m, *v;
    const float *lr, *c1, *c2;
    int32_t *kstep, *kblk;
    float b1, b2, eps;
};
struct RedArgs {
    RedSeg seg[4];
    int nseg, nblocks;
    RedAdam adam;  // adam.p == NULL: reduction only
};

// Adam update of parameter j with gradient gj (c1, c2: the bias
// corrections 1 - beta^t).
__device__ __forceinline__ void adam_value(int j, float *p, float *m, float *v, float gj, float lr,
                                           float b1, float b2, float eps, float c1, float c2)
{
    const float mj = b1 * m[j] + (1.0f - b1) * gj;
    const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    p[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// dst[j] = sum over blocks of partial[blk][j] in a fixed order: 4 threads
// per weight each add every 4th block (in block order), then the 4 sums
// are added in a fixed tree.  A workgroup covers kRedCols consecutive
// weights of one segment, so each wave reads 256 contiguous bytes per
// block.
constexpr int kRedCols = 64, kRedParts = 256 / kRedCols;
// workgroups of the reduction over all four layers
constexpr int kRedBlocks = (WgShape<WG_FIRST>::np + kRedCols - 1) / kRedCols +
                           2 * ((WgShape<WG_MID>::np + kRedCols - 1) / kRedCols) +
                           (WgShape<WG_LAST>::np + kRedCols - 1) / kRedCols;
__global__ __launch_bounds__(256) void reduce_kernel(RedArgs R)
{
    __shared__ float red[kRedParts][kRedCols + 1];
    int si = 0;
    for (int q = 1; q < R.nseg; q++)
        if ((int)blockIdx.x >= R.seg[q].blk0) si = q;
    const RedSeg S = R.seg[si];
    const int np = S.np, nblocks = R.nblocks;
    const float *partial = S.partial;
    float *dst = S.dst;
    const int jl = threadIdx.x % kRedCols, part = threadIdx.x / kRedCols;
    const int j = ((int)blockIdx.x - S.blk0) * kRedCols + jl;
    float acc = 0.0f;
    // one accumulator, rows in order; the unrolled loads overlap
    if (j < np) {
#pragma unroll 8
        for (int k = part; k < nblocks; k += kRedParts) acc += partial[(int64_t)k * np + j];
    }
    red[part][jl] = acc;
    __syncthreads();
    for (int s = kRedParts / 2; s > 0; s >>= 1) {
        if (part < s) red[part][jl] += red[part + s][jl];
        __syncthreads();
    }
    const RedAdam &D = R.adam;
    const int k = D.p ? D.kblk[blockIdx.x] : 0;
    if (part == 0 && j < np) {
        const float gj = red[0][jl];
        dst[j] = gj;
        if (D.p)
            adam_value(S.poff + j, D.p, D.m, D.v, gj, D.lr[k], D.b1, D.b2, D.eps, D.c1[k],
                       D.c2[k]);
    }
    if (D.p) {
        __syncthreads();  // every use of k is behind
        if (threadIdx.x == 0) {
            D.kblk[blockIdx.x] = k + 1;
            if (blockIdx.x == 0) *D.kstep = k + 1;
        }
    }
}

// The weight-gradient kernels produce dW[co][tap][ci] and db[co] per layer,
// already in the parameter blob's order: W block followed by its bias.

// ---------------------------------------------------------------------------

// Adam update of parameter j from g[j].
__device__ __forceinline__ void adam_update(int j, float *p, float *m, float *v, const float *g,
                                            float lr, float b1, float b2, float eps, float c1,
                                            float c2)
{
    adam_value(j, p, m, v, g[j], lr, b1, b2, eps, c1, c2);
}

__global__ void adam_kernel(float *p, float *m, float *v, const float *g, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) adam_update(j, p, m, v, g, lr, b1, b2, eps, c1, c2);
}

__global__ void mux_kernel(const float *y, const float *est, const uint8_t *stable, int64_t n,
                           float *out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[j] = stable[j] ? y[j] : est[j];
}

// ---------------------------------------------------------------------------
// workspace

struct Workspace {
    __bf16 *packed;
    __bf16 *a1, *a2, *a3;   // activations after ReLU
    __bf16 *g1, *g2;        // gradient ping-pong (NHWC 32 ch)
    float *dy;
    float *partial;
    float *loss_partial;
};

__host__ __device__ inline int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

inline int wg_blocks(int B, int Hc, int Wc) { return B * ((Hc + 15) / 16) * ((Wc + 15) / 16); }

// weight-gradient partial columns of all four layers (each layer has its
// own rows, so that one launch reduces them all)
constexpr int kPartialCols =
    WgShape<WG_FIRST>::np + 2 * WgShape<WG_MID>::np + WgShape<WG_LAST>::np;

inline int64_t workspace_bytes(int B, int Hc, int Wc)
{
    const int64_t P = (int64_t)B * Hc * Wc;
    int64_t s = align256((int64_t)PACK_TOTAL * 2);
    s += 5 * align256(P * C * 2);
    s += align256(P * 4);
    s += align256((int64_t)wg_blocks(B, Hc, Wc) * kPartialCols * 4);
    s += align256(((P + 255) / 256) * 4);
    return s;
}

inline Workspace carve(void *ws, int B, int Hc, int Wc)
{
    const int64_t P = (int64_t)B * Hc * Wc;
    char *c = (char *)ws;
    Workspace w;
    w.packed = (__bf16 *)c;
    c += align256((int64_t)PACK_TOTAL * 2);
    __bf16 **acts[5] = {&w.a1, &w.a2, &w.a3, &w.g1, &w.g2};
    for (auto a : acts) {
        *a = (__bf16 *)c;
        c += align256(P * C * 2);
    }
    w.dy = (float *)c;
    c += align256(P * 4);
    w.partial = (float *)c;
    c += align256((int64_t)wg_blocks(B, Hc, Wc) * kPartialCols * 4);
    w.loss_partial = (float *)c;
    return w;
}

ConvArgs conv_args(int B, int Hc, int Wc)
{
    ConvArgs a{};
    a.B = B;
    a.Hc = Hc;
    a.Wc = Wc;
    a.bx = (Wc + 15) / 16;
    a.by = (Hc + 15) / 16;
    a.nblocks = B * a.bx * a.by;
    return a;
}

constexpr int kConvMaxBlocks = 2048;
constexpr int kMaxDevices = 64;

// Workgroups of conv_kernel<KIND> resident on the whole current device at
// once (they walk the blocks in contiguous ranges, prefetching).
template <int KIND>
int conv_resident()
{
    static int cache[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return kConvMaxBlocks;
    if (cache[dev] == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, conv_kernel<KIND>, 256, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            per_cu <= 0 || cus <= 0)
            return kConvMaxBlocks;
        cache[dev] = per_cu * cus;
    }
    return cache[dev];
}

template <int KIND>
void launch_conv(const ConvArgs &a, hipStream_t st)
{
    int cap = conv_resident<KIND>();
    if (spk::g_sur_conv_wg > 0 && spk::g_sur_conv_wg < cap) cap = spk::g_sur_conv_wg;
    const int blocks = a.nblocks < cap ? a.nblocks : cap;
    hipLaunchKernelGGL(conv_kernel<KIND>, dim3(blocks), dim3(256), 0, st, a);
}

// Fill the per-device launch-shape caches (no device work), so that a
// later stream capture makes no occupancy queries.
void warm_launch_caches()
{
    conv_resident<CK_FIRST>();
    conv_resident<CK_MID>();
    conv_resident<CK_LAST>();
    conv_resident<CK_DGRAD_MID>();
    conv_resident<CK_DGRAD_LAST>();
}

// Weight-gradient partials of layer kind K into a.partial (one row per
// workgroup); the reduction into dst is queued as a segment of R.
template <int K>
void launch_wgrad(WgArgs a, float *grad, int poff, RedArgs &R, hipStream_t st)
{
    float *dst = grad + poff;
    a.ntiles = a.B * a.tx * a.ty;
    const int nblk = a.ntiles < kWgMaxBlocks ? a.ntiles : kWgMaxBlocks;
    if constexpr (K == WG_LAST)
        hipLaunchKernelGGL(wgrad_last_kernel, dim3(nblk), dim3(256), 0, st, a);
    else if constexpr (K == WG_FIRST)
        hipLaunchKernelGGL(wgrad_first_kernel, dim3(nblk), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(wgrad_kernel, dim3(nblk), dim3(256), 0, st, a);
    const int np = WgShape<K>::np;
    RedSeg &S = R.seg[R.nseg++];
    S.partial = a.partial;
    S.dst = dst;
    S.np = np;
    S.poff = poff;
    S.blk0 = R.nseg > 1 ? R.seg[R.nseg - 2].blk0 + (R.seg[R.nseg - 2].np + kRedCols - 1) / kRedCols
                        : 0;
    R.nblocks = nblk;
}

void launch_reduce(const RedArgs &R, hipStream_t st)
{
    const RedSeg &L = R.seg[R.nseg - 1];
    // with all four layers' segments this is kRedBlocks, the number of
    // per-workgroup step counters a training plan allocates
    const int grid = L.blk0 + (L.np + kRedCols - 1) / kRedCols;
    hipLaunchKernelGGL(reduce_kernel, dim3(grid), dim3(256), 0, st, R);
}

// Layer by layer (pack = false: the packed weights are already in the
// workspace).
void forward_all(const float *params, const uint32_t *win, const float *est, int B, int Hc,
                 int Wc, float *y, const Workspace &w, hipStream_t st, bool pack = true)
{
    if (pack)
        hipLaunchKernelGGL(pack_kernel, dim3((PACK_TOTAL + 255) / 256), dim3(256), 0, st,
                           params, w.packed);
    ConvArgs a = conv_args(B, Hc, Wc);
    a.win = win;
    a.scalar = est;
    a.packed = w.packed + pack_offset(PK_FIRST);
    a.bias = params + OFF_B1;
    a.out = w.a1;
    launch_conv<CK_FIRST>(a, st);
    a.act = w.a1;
    a.packed = w.packed + pack_offset(PK_MID2);
    a.bias = params + OFF_B2;
    a.out = w.a2;
    launch_conv<CK_MID>(a, st);
    a.act = w.a2;
    a.packed = w.packed + pack_offset(PK_MID3);
    a.bias = params + OFF_B3;
    a.out = w.a3;
    launch_conv<CK_MID>(a, st);
    a.act = w.a3;
    a.scalar = est;
    a.packed = w.packed + pack_offset(PK_LAST);
    a.bias = params + OFF_B4;
    a.out = nullptr;
    a.out_f32 = y;
    launch_conv<CK_LAST>(a, st);
}

// Forward for training (the activations the backward pass reads are kept).
void forward_train(const float *params, const uint32_t *win, const float *est, int B, int Hc,
                   int Wc, float *y, const Workspace &w, hipStream_t st)
{
    forward_all(params, win, est, B, Hc, Wc, y, w, st);
}

// MSE gradient: loss (dL/dy and the loss partial sums, into a per-step row
// of loss_partial when kstep is given), then per layer from the top the
// weight gradient and the input gradient through the ReLU mask.  With adam
// (training plans) the reduction also takes the Adam step.
void backward_all(const float *params, const uint32_t *win, const float *est, int B, int Hc,
                  int Wc, const float *y, const float *target, float *grad, float *loss_partial,
                  const int32_t *kstep, const Workspace &w, hipStream_t st,
                  const RedAdam *adam = nullptr)
{
    const int64_t P = (int64_t)B * Hc * Wc;
    const int lblocks = (int)((P + 255) / 256);
    hipLaunchKernelGGL(loss_kernel, dim3(lblocks), dim3(256), 0, st, y, target, P, w.dy,
                       loss_partial ? loss_partial : w.loss_partial,
                       loss_partial ? kstep : nullptr);
    ConvArgs a = conv_args(B, Hc, Wc);
    // layer 4: weights from dL/dy and a3; gradient into a3's pre-activation
    WgArgs g{};
    g.B = B;
    g.Hc = Hc;
    g.Wc = Wc;
    g.tx = (Wc + 15) / 16;
    g.ty = (Hc + 15) / 16;
    // each layer's partial rows in a region of its own; one reduction at
    // the end
    const int64_t rows = wg_blocks(B, Hc, Wc);
    float *part = w.partial;
    RedArgs R{};
    g.partial = part;
    part += rows * WgShape<WG_LAST>::np;
    g.gy = w.dy;
    g.a = w.a3;
    launch_wgrad<WG_LAST>(g, grad, OFF_W4, R, st);
    a.scalar = w.dy;
    a.packed = w.packed + pack_offset(PK_DG4);
    a.mask = w.a3;
    a.out = w.g1;
    launch_conv<CK_DGRAD_LAST>(a, st);
    // layer 3
    g.g = w.g1;
    g.a = w.a2;
    g.partial = part;
    part += rows * WgShape<WG_MID>::np;
    launch_wgrad<WG_MID>(g, grad, OFF_W3, R, st);
    a.act = w.g1;
    a.packed = w.packed + pack_offset(PK_DG3);
    a.mask = w.a2;
    a.out = w.g2;
    launch_conv<CK_DGRAD_MID>(a, st);
    // layer 2
    g.g = w.g2;
    g.a = w.a1;
    g.partial = part;
    part += rows * WgShape<WG_MID>::np;
    launch_wgrad<WG_MID>(g, grad, OFF_W2, R, st);
    a.act = w.g2;
    a.packed = w.packed + pack_offset(PK_DG2);
    a.mask = w.a1;
    a.out = w.g1;
    launch_conv<CK_DGRAD_MID>(a, st);
    // layer 1
    g.g = w.g1;
    g.win = win;
    g.est = est;
    g.partial = part;
    launch_wgrad<WG_FIRST>(g, grad, OFF_W1, R, st);
    if (adam) R.adam = *adam;
    launch_reduce(R, st);
}

}  // namespace
}  // namespace sur
}  // namespace spk

using namespace spk::sur;

// A training loop captured once in a HIP graph.  Device buffer (one
// allocation): workspace, the batch (win, est, stable, target, y), the
// gradient, the per-step tables (crops, learning rate, bias corrections)
// and the step counter.
struct spk_sur_train_s {
    int dev = -1;
    int32_t steps = 0, done = 0, B = 0, Hc = 0, Wc = 0;
    void *buf = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

size_t spk_sur_workspace_bytes(int32_t B, int32_t Hc, int32_t Wc)
{
    if (B <= 0 || Hc <= 0 || Wc <= 0) return 0;
    return (size_t)workspace_bytes(B, Hc, Wc);
}


static int check_batch(int32_t B, int32_t Hc, int32_t Wc)
{
    if (B <= 0 || Hc <= 0 || Wc <= 0) return SPK_EINVAL;
    if ((int64_t)B * Hc * Wc > ((int64_t)1 << 31) / C) return SPK_EINVAL;
    return SPK_OK;
}

int spk_sur_workspace_layout(int32_t B, int32_t Hc, int32_t Wc, size_t *offsets)
{
    if (!offsets || check_batch(B, Hc, Wc)) return SPK_EINVAL;
    // carve an address range that is never dereferenced
    const uintptr_t base = (uintptr_t)1 << 20;
    const Workspace w = carve((void *)base, B, Hc, Wc);
    const void *views[SPK_SUR_WS_VIEWS] = {w.packed, w.a1, w.a2, w.a3, w.g1, w.g2, w.dy};
    for (int k = 0; k < SPK_SUR_WS_VIEWS; k++)
        offsets[k] = (size_t)((uintptr_t)views[k] - base);
    return SPK_OK;
}

// A crop record is usable for Hc x Wc crops (and has a target if one is
// wanted).
static bool sample_ok(const spk_sur_sample &S, int32_t Hc, int32_t Wc, bool need_target)
{
    if (!S.stream || S.H <= 0 || S.W <= 0 || S.T < 32 || S.t < 31 || S.t >= S.T || S.oy < 0 ||
        S.ox < 0 || S.oy + Hc > S.H || S.ox + Wc > S.W)
        return false;
    if ((int64_t)S.H * S.W > (int64_t)INT32_MAX - 128) return false;
    // frames are read as 8-byte words from 16-byte aligned rows
    if ((uintptr_t)S.stream & 15u) return false;
    return !need_target || S.target;
}

int spk_sur_input(const spk_sur_sample *samples, int32_t B, int32_t Hc, int32_t Wc, float theta,
                  uint32_t *win, float *est, uint8_t *stable, float *target, void *hip_stream)
{
    if (!samples || !win || !est || !stable || B > SPK_SUR_MAX_SAMPLES) return SPK_EINVAL;
    if (check_batch(B, Hc, Wc) || !std::isfinite(theta) || !(theta > 0.0f)) return SPK_EINVAL;
    SampleTab tab{};
    for (int b = 0; b < B; b++) {
        if (!sample_ok(samples[b], Hc, Wc, target != nullptr)) return SPK_EINVAL;
        tab.s[b] = samples[b];
    }
    const int xtiles = (Wc + 63) / 64;
    hipLaunchKernelGGL(input_kernel, dim3(B * Hc * xtiles), dim3(64), 0, (hipStream_t)hip_stream,
                       tab, Hc, Wc, xtiles, (double)theta, win, est, stable, target);
    return hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
}

int spk_sur_stream_step(const uint8_t *frame, int32_t H, int32_t W, float theta, uint32_t *win,
                        float *est, uint8_t *stable, void *hip_stream)
{
    if (!frame || !win || !est || !stable || H <= 0 || W <= 0) return SPK_EINVAL;
    if (!std::isfinite(theta) || !(theta > 0.0f)) return SPK_EINVAL;
    const int64_t HW = (int64_t)H * W;
    if (HW > (int64_t)INT32_MAX - 128) return SPK_EINVAL;
    hipLaunchKernelGGL(stream_kernel, dim3((unsigned)((HW + 255) / 256)), dim3(256), 0,
                       (hipStream_t)hip_stream, frame, HW, (double)theta, win, est, stable);
    return hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
}

int spk_sur_forward(const float *params, const uint32_t *win, const float *est, int32_t B,
                    int32_t Hc, int32_t Wc, float *y, void *workspace, void *hip_stream)
{
    if (!params || !win || !est || !y || !workspace || check_batch(B, Hc, Wc)) return SPK_EINVAL;
    const Workspace w = carve(workspace, B, Hc, Wc);
    forward_train(params, win, est, B, Hc, Wc, y, w, (hipStream_t)hip_stream);
    return hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
}

static int sur_infer(const float *params, const uint32_t *win, const float *est, int32_t B,
                     int32_t Hc, int32_t Wc, float *y, void *workspace, void *hip_stream,
                     bool pack)
{
    if (!params || !win || !est || !y || !workspace || check_batch(B, Hc, Wc)) return SPK_EINVAL;
    const Workspace w = carve(workspace, B, Hc, Wc);
    forward_all(params, win, est, B, Hc, Wc, y, w, (hipStream_t)hip_stream, pack);
    return hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
}

int spk_sur_infer(const float *params, const uint32_t *win, const float *est, int32_t B,
                  int32_t Hc, int32_t Wc, float *y, void *workspace, void *hip_stream)
{
    return sur_infer(params, win, est, B, Hc, Wc, y, workspace, hip_stream, true);
}

int spk_sur_infer_prepacked(const float *params, const uint32_t *win, const float *est,
                            int32_t B, int32_t Hc, int32_t Wc, float *y, void *workspace,
                            void *hip_stream)
{
    return sur_infer(params, win, est, B, Hc, Wc, y, workspace, hip_stream, false);
}

int spk_sur_backward(const float *params, const uint32_t *win, const float *est, int32_t B,
                     int32_t Hc, int32_t Wc, const float *y, const float *target, float *grad,
                     float *loss_partial_out, void *workspace, void *hip_stream)
{
    if (!params || !win || !est || !y || !target || !grad || !workspace ||
        check_batch(B, Hc, Wc))
        return SPK_EINVAL;
    const Workspace w = carve(workspace, B, Hc, Wc);
    backward_all(params, win, est, B, Hc, Wc, y, target, grad, loss_partial_out, nullptr, w,
                 (hipStream_t)hip_stream);
    return hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
}

static bool adam_ok(float beta1, float beta2, float eps)
{
    return beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f;
}

// Adam's bias corrections 1 - beta^t (the same expression for the eager
// step and the per-step tables of a training plan).
static float bias_correction(float beta, int32_t t) { return 1.0f - std::pow(beta, (float)t); }

int spk_sur_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr,
                 float beta1, float beta2, float eps, void *hip_stream)
{
    if (!params || !m || !v || !grad || step < 1 || !(lr > 0.0f) || !adam_ok(beta1, beta2, eps))
        return SPK_EINVAL;
    const float c1 = bias_correction(beta1, step), c2 = bias_correction(beta2, step);
    hipLaunchKernelGGL(adam_kernel, dim3((NPARAMS + 255) / 256), dim3(256), 0,
                       (hipStream_t)hip_stream, params, m, v, grad, NPARAMS, lr, beta1, beta2, eps,
                       c1, c2);
    return hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
}

int spk_sur_mux(const float *y, const float *est, const uint8_t *stable, int64_t n, float *out,
                void *hip_stream)
{
    if (!y || !est || !stable || !out || n < 0) return SPK_EINVAL;
    if (n == 0) return SPK_OK;
    hipLaunchKernelGGL(mux_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)hip_stream, y, est, stable, n, out);
    return hipGetLastError() == hipSuccess ? SPK_OK : SPK_EHIP;
}

static void train_free(spk_sur_train_s *pl)
{
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->buf) (void)hipFree(pl->buf);
    delete pl;
}

int spk_sur_train_create(spk_sur_train_t *plan, float *params, float *m, float *v,
                         const spk_sur_sample *samples, const float *lr, int32_t steps,
                         int32_t B, int32_t Hc, int32_t Wc, float theta, float beta1, float beta2,
                         float eps, int32_t step0, float *loss_partial)
{
    if (!plan) return SPK_EINVAL;
    *plan = nullptr;
    if (!params || !m || !v || !samples || !lr || steps <= 0 || step0 < 1 ||
        B > SPK_SUR_MAX_SAMPLES || check_batch(B, Hc, Wc) || !std::isfinite(theta) ||
        !(theta > 0.0f) || !adam_ok(beta1, beta2, eps))
        return SPK_EINVAL;
    if ((int64_t)step0 + steps > INT32_MAX || (int64_t)steps * B > INT32_MAX) return SPK_EINVAL;
    for (int64_t k = 0; k < (int64_t)steps * B; k++)
        if (!sample_ok(samples[k], Hc, Wc, true)) return SPK_EINVAL;
    for (int32_t k = 0; k < steps; k++)
        if (!(lr[k] > 0.0f) || !std::isfinite(lr[k])) return SPK_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPK_EHIP;
    // host tables: learning rate and bias corrections per step
    std::vector<float> tab((size_t)steps * 3);
    for (int32_t k = 0; k < steps; k++) {
        tab[k] = lr[k];
        tab[(size_t)steps + k] = bias_correction(beta1, step0 + k);
        tab[(size_t)steps * 2 + k] = bias_correction(beta2, step0 + k);
    }
    const int64_t P = (int64_t)B * Hc * Wc;
    const int64_t ws = workspace_bytes(B, Hc, Wc);
    const int64_t o_win = align256(ws), o_est = o_win + align256(P * 4),
                  o_stable = o_est + align256(P * 4), o_target = o_stable + align256(P),
                  o_y = o_target + align256(P * 4), o_grad = o_y + align256(P * 4),
                  o_samples = o_grad + align256((int64_t)NPARAMS * 4),
                  o_tab = o_samples + align256((int64_t)steps * B * sizeof(spk_sur_sample)),
                  o_k = o_tab + align256((int64_t)steps * 3 * 4),
                  total = o_k + align256(4 * (1 + kRedBlocks));
    auto *pl = new spk_sur_train_s;
    pl->dev = dev;
    pl->steps = steps;
    pl->B = B;
    pl->Hc = Hc;
    pl->Wc = Wc;
    if (hipMalloc(&pl->buf, (size_t)total) != hipSuccess) {
        (void)hipGetLastError();
        train_free(pl);
        return SPK_ENOMEM;
    }
    char *c = (char *)pl->buf;
    uint32_t *win = (uint32_t *)(c + o_win);
    float *est = (float *)(c + o_est), *target = (float *)(c + o_target), *y = (float *)(c + o_y);
    float *grad = (float *)(c + o_grad), *dtab = (float *)(c + o_tab);
    uint8_t *stable = (uint8_t *)(c + o_stable);
    spk_sur_sample *dsamples = (spk_sur_sample *)(c + o_samples);
    int32_t *kstep = (int32_t *)(c + o_k);  // then the reduction's own counters
    const std::vector<int32_t> zero(1 + kRedBlocks, 0);
    if (hipMemcpy(dsamples, samples, (size_t)steps * B * sizeof(spk_sur_sample),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dtab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(kstep, zero.data(), zero.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        train_free(pl);
        return SPK_EHIP;
    }
    // capture one step on a private stream
    warm_launch_caches();
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        train_free(pl);
        return SPK_EHIP;
    }
    const Workspace w = carve(pl->buf, B, Hc, Wc);
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const int xtiles = (Wc + 63) / 64;
        // the input kernel also packs the weights; the reduction takes the
        // Adam step and advances kstep
        hipLaunchKernelGGL(input_step_kernel, dim3(B * Hc * xtiles), dim3(64), 0, cs, dsamples,
                           kstep, B, Hc, Wc, xtiles, (double)theta, win, est, stable, target,
                           params, w.packed);
        forward_all(params, win, est, B, Hc, Wc, y, w, cs, false);
        const RedAdam ad{params, m,         v,     dtab,  dtab + steps, dtab + 2 * steps,
                         kstep,  kstep + 1, beta1, beta2, eps};
        backward_all(params, win, est, B, Hc, Wc, y, target, grad, loss_partial, kstep, w, cs,
                     &ad);
        ok = hipStreamEndCapture(cs, &pl->graph) == hipSuccess && pl->graph;
    }
    ok = ok && hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) == hipSuccess;
    (void)hipStreamDestroy(cs);
    if (!ok) {
        (void)hipGetLastError();
        train_free(pl);
        return SPK_EHIP;
    }
    *plan = pl;
    return SPK_OK;
}

int spk_sur_train_run(spk_sur_train_t plan, int32_t n, void *hip_stream)
{
    if (!plan || n < 0 || n > plan->steps - plan->done) return SPK_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->dev) return SPK_EINVAL;
    for (int32_t i = 0; i < n; i++)
        if (hipGraphLaunch(plan->exec, (hipStream_t)hip_stream) != hipSuccess) return SPK_EHIP;
    plan->done += n;
    return SPK_OK;
}

int spk_sur_train_destroy(spk_sur_train_t plan)
{
    if (!plan) return SPK_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(plan->dev);
    (void)hipDeviceSynchronize();
    train_free(plan);
    (void)hipSetDevice(cur);
    return SPK_OK;
}

}  // extern "C"
