/*
 * spk -- spike-camera reconstruction on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library.  Method: "High-speed and High-quality Vision
 * Reconstruction of Spike Camera with Spike Stability Theorem"
 * (arXiv 2412.11639).  Each pixel's binary spike stream S0 (the discrete
 * integrate-and-fire of Eq. 2) is turned into its inter-spike interval
 * stream S1 (Def. 2, Eq. 4); S1 is cut into segments that stay zero-order
 * stable (values span at most 1), at first order (FSR) or additionally at
 * second order (SSR, the S2 streams of Eq. 5), Sec. III-B; each segment's
 * intensity is theta * N / sum of its N intervals (Eq. 6, with the paper's
 * 8-bit scale 255 replaced by theta).
 *
 * Common conventions
 *   stream   device pointer to T packed binary frames, frame-major: frame t
 *            starts at byte t * spk_frame_bytes(H, W); pixel p = y * W + x
 *            is bit (p & 7) of byte (p >> 3), least significant bit first;
 *            padding bits must be zero.  Frames are 16-byte aligned, and the
 *            stream pointer must be too (SPK_EINVAL otherwise).
 *   t_out    host pointer to n_out output frame indices, 0 <= t < T, in any
 *            order, duplicates allowed; output plane k is for t_out[k].
 *   out      device pointer, float32 [n_out][H][W].
 *   order    SPK_FSR or SPK_SSR.
 *   hip_stream  a hipStream_t (NULL = the default stream); all device work is
 *            enqueued on it and the call returns without synchronising.
 *   Output time t uses the segment holding the interval in progress at t:
 *            m(t) = clamp(#spikes at frames < t, 1, K - 1) (1-based), so
 *            frames up to the first spike use the first interval and frames
 *            after the last spike the last one.  A pixel with fewer than two
 *            spikes outputs 0 and the window (-1, -1, 0).
 *   Ownership: the caller owns every buffer it passes.  The library keeps a
 *            small per-device workspace (sorted output times) that lives until
 *            process exit; plans own their device tables until destroyed.
 *            Cached output-time tables are shared by calls on any stream:
 *            a call that reuses tables uploaded on another stream makes its
 *            own stream wait (hipStreamWaitEvent) for that upload, so calls
 *            on different streams never read a table before it has landed.
 *   Errors:  arguments are checked on the host before anything is enqueued;
 *            on error nothing is written and a negative code is returned.
 *            A failed launch returns SPK_EHIP; faults inside kernels surface
 *            at the caller's next synchronisation.  Calls on one device are
 *            safe from one host thread at a time.
 */
#ifndef SPK_H
#define SPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SPK_OK = 0,
    SPK_EINVAL = -1,      /* bad argument                                  */
    SPK_ENOMEM = -2,      /* device or host allocation failed              */
    SPK_EHIP = -3,        /* a HIP runtime call or launch failed           */
    SPK_EUNSUPPORTED = -4, /* no usable gfx950 device                      */
    SPK_ERANGE = -5        /* beyond the fixed scratch of spk_reconstruct_noalloc */
};

/*
 * Segmentation orders: SPK_FSR and SPK_SSR are the paper's first- and
 * second-order stable reconstructions (Sec. III-B).  SPK_TSR takes the
 * n-order rule (Sec. III-A, Eq. 5) one step further: inside each SSR piece
 * it also cuts where an S3 stream (gaps between consecutive positions of an
 * S2 value inside S2) leaves zero-order stability.  SPK_TFI is the TFI
 * baseline the paper compares against (Sec. II: the reciprocal of the
 * interval between the two spikes around the output frame), run as the
 * order that keeps every interval on its own (windows have N = 1).
 */
enum { SPK_FSR = 1, SPK_SSR = 2, SPK_TFI = 3, SPK_TSR = 4 };

/* Bytes per packed frame: ceil(H*W / 128) * 16.  0 if H or W <= 0. */
size_t spk_frame_bytes(int32_t H, int32_t W);

/* Human-readable text for an error code (static storage). */
const char *spk_strerror(int code);

/* Library version as major * 10000 + minor * 100 + patch. */
int spk_version(void);

/*
 * Process-wide tuning options (not part of any result: every setting gives
 * bit-identical output).
 *   SPK_OPT_TIME_CHUNKS  number of time chunks a long stream is split into
 *                        so that more waves run at once; 0 = automatic
 *                        (the default; the SPK_CHUNKS environment variable
 *                        overrides it at first use).  Values above the
 *                        number of 64-frame tiles are clamped.
 *   SPK_OPT_WARM_TILES   64-frame tiles each speculative time chunk is
 *                        warmed up on before its start; 0 = automatic
 *                        (the default: four, at most half a chunk; the
 *                        SPK_WARM environment variable overrides it at
 *                        first use).  The fixup pass makes the result exact
 *                        for any value.
 *   SPK_OPT_SUR_CONV_WG  at most this many workgroups per layer-by-layer
 *                        surrogate convolution, each walking a contiguous
 *                        range of 16 x 16 pixel blocks; 0 (default): as many
 *                        as fit on the device at once.
 *   SPK_OPT_PLAN_KGROUP, SPK_OPT_PLAN_WAVES_PER_WG, SPK_OPT_PLAN_WPE
 *                        the launch shape of batched plans created without
 *                        SPK_PLAN_AUTOTUNE (see spk_plan_shape): 64-frame
 *                        tiles per prefetch group (4, 8, 16), waves per
 *                        workgroup (1, 2, 4), register target variant (0:
 *                        four waves per SIMD, 1: five); 0 = default
 *                        (8, 1, 0).
 * spk_set_option returns SPK_OK or SPK_EINVAL (unknown option, value out of
 * range); spk_get_option returns the value or SPK_EINVAL.
 */
enum {
    SPK_OPT_TIME_CHUNKS = 1,
    SPK_OPT_SUR_CONV_WG = 3,
    SPK_OPT_PLAN_KGROUP = 4,
    SPK_OPT_PLAN_WAVES_PER_WG = 5,
    SPK_OPT_PLAN_WPE = 6,
    SPK_OPT_WARM_TILES = 7
};
int spk_set_option(int option, int value);
int spk_get_option(int option);

/*
 * Reconstruct intensity at the requested frames (Sec. III-B segmentation,
 * Eq. 6 intensity).  theta: finite and > 0 (255 reproduces Eq. 6's 8-bit
 * scale).  The intensity is computed as (double)theta * N / D and rounded
 * once to float.  n_out == 0 is a no-op.
 */
int spk_reconstruct(const uint8_t *stream, int32_t H, int32_t W, int32_t T, float theta,
                    const int32_t *t_out, int32_t n_out, float *out, int32_t order,
                    void *hip_stream);

/*
 * As spk_reconstruct, and also the window of the segment used for each
 * output: first and last spike frame and the number of intervals N (so the
 * duration is last - first).  Each of out, win_first, win_last, win_n is a
 * device pointer [n_out][H][W] or NULL (not written).
 */
int spk_reconstruct_windows(const uint8_t *stream, int32_t H, int32_t W, int32_t T,
                            float theta, const int32_t *t_out, int32_t n_out, float *out,
                            int32_t *win_first, int32_t *win_last, int32_t *win_n,
                            int32_t order, void *hip_stream);

/*
 * For callers that cannot allocate device memory -- code running under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation --
 * spk_reconstruct with no allocation of any kind: every device buffer beyond
 * the caller's stream and out (the output-time tables and the per-chunk
 * records of long streams) lives in a fixed array of
 * SPK_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds from
 * library load until the process ends.  The output times reach the device
 * as kernel arguments (no host staging).  Results are identical to
 * spk_reconstruct's.  Limits: n_out <= 2^20 and T + 2 * n_out <= 2^24 - 64
 * (else SPK_ERANGE, nothing enqueued); a long stream is split into fewer
 * time chunks when their records do not fit the rest of the array (same
 * results, less parallelism).  Every call on a GPU uses that GPU's one
 * array: calls on one GPU whose work overlaps (two host threads, or two
 * streams whose work runs at the same time) race on it and must be
 * serialised by the caller.  Other arguments and errors as spk_reconstruct.
 */
#define SPK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int spk_reconstruct_noalloc(const uint8_t *stream, int32_t H, int32_t W, int32_t T, float theta,
                            const int32_t *t_out, int32_t n_out, float *out, int32_t order,
                            void *hip_stream);

/*
 * Every segment of every pixel (the full segmentation of Sec. III-B).
 * seg_first/seg_last/seg_n: device int32 [cap][H*W]: segment s of pixel p
 * at s * H*W + p (first spike frame, last spike frame, number of intervals).
 * count: device int32 [H*W], the total number of segments of each pixel
 * (segments past cap are counted but not stored).  cap >= 0; with cap == 0
 * the seg_* pointers may be NULL.
 */
int spk_segments(const uint8_t *stream, int32_t H, int32_t W, int32_t T, int32_t order,
                 int32_t cap, int32_t *seg_first, int32_t *seg_last, int32_t *seg_n,
                 int32_t *count, void *hip_stream);

/*
 * TFP baseline (Sec. II): theta * (spikes in the `window` frames ending at
 * t_out[k]) / (window length), the window clipped at the stream's start
 * (length min(window, t + 1)); computed as (double)theta * count / length
 * and rounded once to float.  window >= 1.  out: device float
 * [n_out][H][W].  Arguments and errors as spk_reconstruct.
 */
int spk_tfp(const uint8_t *stream, int32_t H, int32_t W, int32_t T, float theta,
            int32_t window, const int32_t *t_out, int32_t n_out, float *out, void *hip_stream);

/*
 * Static / motion mask (the use of the stability theorem the paper's
 * conclusion names: stable and unstable spike emission tell static from
 * moving parts).  mask[k][p] = 1 when the segment of the given order that
 * holds the interval in progress at t_out[k] begins at a cut less than
 * `window` frames back (its first spike f > t - window and it is not the
 * pixel's first segment), else 0; 0 for pixels with fewer than two spikes.
 * mask: device uint8 [n_out][H][W].  window >= 1; other
 * arguments and errors as spk_reconstruct.  Uses temporary device memory
 * from the stream-ordered allocator.
 */
int spk_motion(const uint8_t *stream, int32_t H, int32_t W, int32_t T, int32_t order,
               int32_t window, const int32_t *t_out, int32_t n_out, uint8_t *mask,
               void *hip_stream);

/*
 * Decoder of the segment encoding (the encoder/decoder split of the
 * paper's hardware design, Sec. III-C): the intensity at each requested
 * frame from segment lists as spk_segments writes them (seg_first,
 * seg_last, seg_n [cap][H*W], count [H*W], all device), without the stream.
 * The output for t is Eq. 6 on the segment holding the interval in progress
 * at t, exactly as spk_reconstruct computes it from the stream the lists
 * came from (same order, same T).  A pixel whose list was cut at cap
 * (count > cap) decodes to NaN from the first frame its stored segments do
 * not reach.  t_out, n_out, out, theta, errors as spk_reconstruct.
 */
int spk_decode(const int32_t *seg_first, const int32_t *seg_last, const int32_t *seg_n,
               const int32_t *count, int32_t cap, int32_t H, int32_t W, int32_t T, float theta,
               const int32_t *t_out, int32_t n_out, float *out, void *hip_stream);

/*
 * The same segment lists kept contiguous per pixel (Sec. III-B
 * segmentation, Sec. III-C encoder/decoder): rec is device int32
 * [H*W][cap][3], segment s of pixel p at rec[(p * cap + s) * 3 + {0, 1, 2}]
 * = (first spike frame, last spike frame, number of intervals), the same
 * values spk_segments stores at s * H*W + p.  Each pixel's list is one run
 * of memory, so the encoder fills whole lines and the decoder reads each
 * line once (with the [cap][H*W] arrays every record load of a wave takes
 * 64 separate lines).  count, cap, the other arguments and errors as
 * spk_segments / spk_decode; with cap == 0 rec may be NULL.
 */
int spk_segments_packed(const uint8_t *stream, int32_t H, int32_t W, int32_t T, int32_t order,
                        int32_t cap, int32_t *rec, int32_t *count, void *hip_stream);
int spk_decode_packed(const int32_t *rec, const int32_t *count, int32_t cap, int32_t H, int32_t W,
                      int32_t T, float theta, const int32_t *t_out, int32_t n_out, float *out,
                      void *hip_stream);

/*
 * Carry-state reconstruction of a live stream (the paper's hardware
 * processes the camera's frames in 32-frame blocks as they arrive,
 * Sec. III-C): frames are fed in pieces of any length, each pixel's state
 * (last spike, the open segment with its FSR / SSR / third-order state, and
 * the first output that waits for it) stays in device memory between
 * pieces, and every output is written as soon as the segment holding it
 * closes.  After spk_stream_finish the outputs equal what spk_reconstruct /
 * spk_reconstruct_windows give on the concatenated stream (bit for bit), as
 * long as every t_out is below the number of frames fed; an output time at
 * or past the end takes the last segment (no later spike was seen).
 *
 * spk_stream_create: H, W, theta, order as spk_reconstruct; t_out (host,
 *   any order, duplicates allowed, t >= 0) is copied; out, win_first,
 *   win_last, win_n: device [n_out][H][W] buffers or NULL, written by the
 *   feeds and the finish (they must stay valid until the finish has run).
 *   Allocates the per-pixel state (at most 37 ints per pixel) on the
 *   current device.  SPK_EINVAL, SPK_ENOMEM, SPK_EHIP, SPK_EUNSUPPORTED.
 * spk_stream_feed: the next nframes packed frames (device, frame-major,
 *   16-byte aligned, layout as spk_reconstruct's stream), enqueued on
 *   hip_stream.  nframes == 0 is a no-op.  The frames must stay valid
 *   until the call's work has run.
 * spk_stream_finish: writes every output still waiting (the open segment
 *   of each pixel; 0 and (-1, -1, 0) for pixels with fewer than two spikes).
 *   No feed is accepted afterwards.
 * spk_stream_frames: frames fed so far (or SPK_EINVAL for NULL).
 * spk_stream_destroy: waits for the device and frees the state (NULL: no-op).
 * All calls on one spk_stream_t must run in order: enqueue them on one HIP
 * stream, or synchronise between them.  A stream object belongs to the
 * device current at its creation.
 */
typedef struct spk_stream_s *spk_stream_t;
int spk_stream_create(spk_stream_t *stream, int32_t H, int32_t W, float theta, int32_t order,
                      const int32_t *t_out, int32_t n_out, float *out, int32_t *win_first,
                      int32_t *win_last, int32_t *win_n);
int spk_stream_feed(spk_stream_t stream, const uint8_t *frames, int32_t nframes,
                    void *hip_stream);
int spk_stream_finish(spk_stream_t stream, void *hip_stream);
int spk_stream_frames(spk_stream_t stream);
int spk_stream_destroy(spk_stream_t stream);

/*
 * Batched plans: many streams of uneven size reconstructed by one
 * persistent kernel (one wave per 64-pixel strip of a stream at a time,
 * strips taken from per-XCD work counters), captured once in a HIP graph.
 *
 * spk_job describes one stream: stream and out are device pointers laid
 * out as for spk_reconstruct; t_out is a host pointer read (and copied)
 * during spk_plan_create only; n_out > 0.
 *
 * spk_plan_create validates every job on the host (SPK_EINVAL on any bad
 * field, nothing allocated), uploads the job table and the sorted output
 * times, chooses the launch shape, captures the graph (unless
 * SPK_PLAN_NO_GRAPH) and synchronises before returning.  The shape is the
 * total waves and workgroups, strips per counter grab, 64-frame tiles per
 * prefetch group, waves per workgroup and the register target (see
 * spk_plan_info, spk_plan_shape).  With SPK_PLAN_AUTOTUNE it is found by
 * timing about 20 candidate shapes on the real jobs in stages (waves x
 * grab, group size, register target, waves per workgroup, waves x grab
 * again), which writes their outputs; the choice is cached per job-size
 * signature in the process and, if the environment variable
 * SPK_TUNE_CACHE names a file, in that JSON file.  Without it the shape is
 * the default or the one set with the SPK_OPT_PLAN_* options.
 * The streams must stay valid and unchanged in place for the plan's life;
 * their contents may change between executions.
 *
 * spk_plan_execute enqueues one execution on hip_stream (NULL = default
 * stream) and returns; executions of one plan must not overlap (they share
 * the plan's work counters).  spk_plan_destroy waits for the plan's device
 * to drain and frees everything the plan owns.  Results are identical to
 * spk_reconstruct of each job, for every launch shape.
 */
typedef struct spk_job {
    const uint8_t *stream;
    int32_t H, W, T;
    float theta;
    const int32_t *t_out;
    int32_t n_out;
    float *out;
} spk_job;

typedef struct spk_plan_s *spk_plan_t;

enum { SPK_PLAN_AUTOTUNE = 1, SPK_PLAN_NO_GRAPH = 2 };

int spk_plan_create(spk_plan_t *plan, const spk_job *jobs, int32_t n_jobs, int32_t order,
                    int32_t flags);
int spk_plan_execute(spk_plan_t plan, void *hip_stream);
/* Launch shape and size: workgroups, strips taken per counter grab, total
 * strips.  Any pointer may be NULL. */
int spk_plan_info(spk_plan_t plan, int32_t *grid, int32_t *grab, int32_t *items);
/* The rest of the launch shape: 64-frame tiles per prefetch group (4, 8 or
 * 16), waves per workgroup (1, 2 or 4, each taking its own strips) and the
 * waves per SIMD the kernel's registers were allocated for (4 or 5).
 * Any pointer may be NULL. */
int spk_plan_shape(spk_plan_t plan, int32_t *kgroup, int32_t *waves_per_wg,
                   int32_t *waves_per_simd);
int spk_plan_destroy(spk_plan_t plan);

/*
 * Learned surrogate (not part of the paper's method: a small CNN that maps
 * a 32-frame spike window plus the plain short-window estimate to the
 * long-window reconstruction; the plain method stays the fallback).
 *
 * Network: four 3x3 convolutions with zero padding, 33 -> 32 -> 32 -> 32 -> 1
 * channels, ReLU after the first three, output added to the estimate
 * (y = est + CNN).  Input channel j < 32 is frame t-31+j of the pixel
 * (0/1), channel 32 the short-window estimate.
 * Parameters: one device float32 vector of SPK_SUR_NPARAMS values,
 * W1 [32][9][33], b1 [32], W2 [32][9][32], b2 [32], W3 [32][9][32], b3 [32],
 * W4 [1][9][32], b4 [1]; tap k = 3*dy + dx reads offset (dy - 1, dx - 1).
 * The kernels compute in bfloat16 on the matrix cores with float32
 * accumulation; weights, inputs, activations and backpropagated gradients
 * are rounded to bfloat16, everything else stays float32.
 *
 * A batch is B images of Hc x Wc pixels, arrays [B][Hc][Wc] (device).
 * workspace: device scratch of spk_sur_workspace_bytes(B, Hc, Wc) bytes,
 * owned by the caller; spk_sur_backward reads the activations that the
 * spk_sur_forward call before it left there (same params, inputs, shape).
 */
#define SPK_SUR_NPARAMS 28321
#define SPK_SUR_MAX_SAMPLES 64

typedef struct spk_sur_sample {
    const uint8_t *stream; /* device: T packed frames of an H x W stream   */
    int32_t H, W, T;
    int32_t oy, ox;        /* crop origin; the crop lies inside the frame */
    int32_t t;             /* output time, 31 <= t < T                    */
    const float *target;   /* device H x W training targets, or NULL      */
} spk_sur_sample;

size_t spk_sur_workspace_bytes(int32_t B, int32_t Hc, int32_t Wc);

/* Where the workspace keeps what the network stored, for inspection (tests
 * check every stored value against a CPU reference).  offsets receives
 * SPK_SUR_WS_VIEWS byte offsets into a workspace for (B, Hc, Wc), in this
 * order: the packed weights; the activations a1, a2, a3 after each ReLU
 * (bfloat16 [B][Hc][Wc][32], written by spk_sur_forward and spk_sur_infer);
 * after spk_sur_backward, the gradients into a1 and a2 after their ReLU
 * masks (bfloat16 [B][Hc][Wc][32]; the gradient into a3 is not kept) and
 * dL/dy (float32 [B][Hc][Wc], values of bfloat16).  SPK_EINVAL on a bad
 * shape or NULL offsets. */
#define SPK_SUR_WS_VIEWS 7
int spk_sur_workspace_layout(int32_t B, int32_t Hc, int32_t Wc, size_t *offsets);

/* Window, short-window estimate and stability flag for B <= 64 crops
 * (samples is a host array).  win[b][y][x] bit j = frame t-31+j; est = the
 * plain method (FSR, Eq. 6) on the window as a stream of its own at its last
 * frame, theta*K/32 below two spikes; stable = FSR keeps the window as one
 * segment.  target (may be NULL) receives the crops of the samples' target
 * frames, which must then all be given. */
int spk_sur_input(const spk_sur_sample *samples, int32_t B, int32_t Hc, int32_t Wc, float theta,
                  uint32_t *win, float *est, uint8_t *stable, float *target, void *hip_stream);

/* Streaming update for a whole H x W frame: win = (win >> 1) | frame << 31,
 * then est and stable of the new window (frame: one packed frame). */
int spk_sur_stream_step(const uint8_t *frame, int32_t H, int32_t W, float theta, uint32_t *win,
                        float *est, uint8_t *stable, void *hip_stream);

/* y = network(win, est), float32 [B][Hc][Wc]. */
int spk_sur_forward(const float *params, const uint32_t *win, const float *est, int32_t B,
                    int32_t Hc, int32_t Wc, float *y, void *workspace, void *hip_stream);

/* As spk_sur_forward for inference only; y is identical (the activations
 * are still written to the workspace). */
int spk_sur_infer(const float *params, const uint32_t *win, const float *est, int32_t B,
                  int32_t Hc, int32_t Wc, float *y, void *workspace, void *hip_stream);

/* As spk_sur_infer without re-packing the weights: the convolutions take
 * them in the MFMA operand layout that the last spk_sur_forward or
 * spk_sur_infer call on this workspace left at its start (it must have had
 * the same params; the packed block does not depend on B, Hc, Wc, so a
 * workspace sized for the largest batch serves them all).  params is
 * still read for the biases.  For serving loops that run one model on
 * every frame; y is identical to spk_sur_infer's. */
int spk_sur_infer_prepacked(const float *params, const uint32_t *win, const float *est,
                            int32_t B, int32_t Hc, int32_t Wc, float *y, void *workspace,
                            void *hip_stream);

/* Gradient of the mean squared error between y and target over all B*Hc*Wc
 * pixels with respect to the parameters (grad: float32 [SPK_SUR_NPARAMS],
 * overwritten).  loss_partial (may be NULL): ceil(B*Hc*Wc / 256) partial
 * sums of squared errors, in block order. */
int spk_sur_backward(const float *params, const uint32_t *win, const float *est, int32_t B,
                     int32_t Hc, int32_t Wc, const float *y, const float *target, float *grad,
                     float *loss_partial, void *workspace, void *hip_stream);

/* One Adam step (with bias correction, step >= 1) on params in place;
 * m and v are the caller's float32 moment buffers. */
int spk_sur_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr,
                 float beta1, float beta2, float eps, void *hip_stream);

/* Training loop replayed from a HIP graph, for callers whose step is bound
 * by host launch overhead.  Each step is spk_sur_input (with targets),
 * spk_sur_forward, spk_sur_backward and spk_sur_adam, with results
 * identical bit for bit to those calls.  samples: host array of steps * B
 * crop records, step k's at [k * B, k * B + B); lr: host, steps learning
 * rates (> 0); both are copied to the device.  Adam's step number of the
 * plan's first step is step0 (>= 1); beta1, beta2, eps as spk_sur_adam.
 * params, m, v: the caller's device buffers, updated in place by every
 * step.  loss_partial (device, may be NULL): row k (ceil(B*Hc*Wc/256)
 * partial sums of squared errors) is written by step k.  The sample
 * streams and targets must stay valid while steps run.  The plan belongs
 * to the current device and owns its buffers and graph.
 * Errors: SPK_EINVAL (arguments, any record), SPK_ENOMEM, SPK_EHIP. */
typedef struct spk_sur_train_s *spk_sur_train_t;
int spk_sur_train_create(spk_sur_train_t *plan, float *params, float *m, float *v,
                         const spk_sur_sample *samples, const float *lr, int32_t steps,
                         int32_t B, int32_t Hc, int32_t Wc, float theta, float beta1, float beta2,
                         float eps, int32_t step0, float *loss_partial);
/* Enqueue the plan's next n steps on hip_stream (SPK_EINVAL if fewer than
 * n remain, or from another device). */
int spk_sur_train_run(spk_sur_train_t plan, int32_t n, void *hip_stream);
/* Waits for the device, then frees the plan (NULL: no-op). */
int spk_sur_train_destroy(spk_sur_train_t plan);

/* Fallback: out = stable ? y : est, over n values. */
int spk_sur_mux(const float *y, const float *est, const uint8_t *stable, int64_t n, float *out,
                void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SPK_H */
