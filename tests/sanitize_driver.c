/*
 * Host-only exercise of the C generator and the C oracle under the address
 * and undefined-behaviour sanitizers (built by tests/test_sanitize.py with
 * gcc; no GPU code).  Every entry point runs on small and ragged shapes,
 * with the edge cases of its arguments; the sanitizers abort on the first
 * out-of-bounds access, leak, overflow or misaligned access.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* generator (spkgen/gen.c) */
size_t spkgen_frame_bytes(int32_t H, int32_t W);
int spkgen_from_increments(uint8_t *out, int32_t H, int32_t W, int32_t T, const int64_t *inc,
                           int32_t per_frame, const int64_t *v0, int64_t theta, int32_t nthreads);
int spkgen_blocks(uint8_t *out, int32_t H, int32_t W, int32_t T, uint64_t seed, int32_t block,
                  double qmin, double qmax, double vx, double vy, int32_t nthreads);
int spkgen_blocks_truth(float *out, int32_t H, int32_t W, const int32_t *frames,
                        int32_t n_frames, uint64_t seed, int32_t block, double qmin, double qmax,
                        double vx, double vy);
int spkgen_gratings(uint8_t *out, int32_t H, int32_t W, int32_t T, uint64_t seed, double phi,
                    int32_t nthreads);
int spkgen_gratings_truth(float *out, int32_t H, int32_t W, const int32_t *frames,
                          int32_t n_frames, uint64_t seed, double phi);

/* oracle (oracle/oracle.c) */
int32_t spk_oracle_segment_intervals(const int32_t *x, int32_t n, int32_t order, int32_t *start);
int32_t spk_oracle_reconstruct(const uint8_t *stream, int32_t H, int32_t W, int32_t T,
                               double theta, const int32_t *t_out, int32_t n_out, int32_t order,
                               double *out, int32_t *win_first, int32_t *win_last,
                               int32_t *win_n, int32_t nthreads);
int32_t spk_oracle_reconstruct_causal(const uint8_t *stream, int32_t H, int32_t W, int32_t T,
                                      double theta, const int32_t *t_out, int32_t n_out,
                                      int32_t order, double *out, int32_t *win_first,
                                      int32_t *win_last, int32_t *win_n, int32_t nthreads);
int32_t spk_oracle_segments(const uint8_t *stream, int32_t H, int32_t W, int32_t T,
                            int32_t order, int32_t cap, int32_t *seg_first, int32_t *seg_last,
                            int32_t *seg_n, int32_t *count, int32_t nthreads);
int32_t spk_oracle_window(const uint8_t *stream, int32_t H, int32_t W, int32_t T, double theta,
                          int32_t t, double *est, uint8_t *stable);
int32_t spk_oracle_tfp(const uint8_t *stream, int32_t H, int32_t W, int32_t T, double theta,
                       int32_t window, const int32_t *t_out, int32_t n_out, double *out);
typedef struct spk_oracle_stream spk_oracle_stream;
spk_oracle_stream *spk_oracle_stream_create(int32_t H, int32_t W, double theta, int32_t order,
                                            const int32_t *t_out, int32_t n_out, double *out,
                                            int32_t *win_first, int32_t *win_last,
                                            int32_t *win_n);
int32_t spk_oracle_stream_feed(spk_oracle_stream *s, const uint8_t *frames, int32_t nframes);
int32_t spk_oracle_stream_finish(spk_oracle_stream *s);
void spk_oracle_stream_destroy(spk_oracle_stream *s);

#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                  \
        }                                                              \
    } while (0)

static int run_shape(int32_t H, int32_t W, int32_t T, int kind)
{
    const size_t fb = spkgen_frame_bytes(H, W);
    uint8_t *s = (uint8_t *)calloc((size_t)T * fb, 1);
    const int64_t hw = (int64_t)H * W;
    CHECK(s);
    if (kind == 0) {
        CHECK(spkgen_blocks(s, H, W, T, 7, 4, 0.02, 1.0, 0.7, -0.3, 3) == 0);
    } else if (kind == 1) {
        CHECK(spkgen_gratings(s, H, W, T, 8, 1000.0, 2) == 0);
    } else {
        int64_t *inc = (int64_t *)malloc(sizeof(int64_t) * (size_t)hw);
        int64_t *v0 = (int64_t *)malloc(sizeof(int64_t) * (size_t)hw);
        CHECK(inc && v0);
        for (int64_t p = 0; p < hw; p++) {
            inc[p] = 1 + (p * 37) % 64;
            v0[p] = (p * 11) % 64;
        }
        CHECK(spkgen_from_increments(s, H, W, T, inc, 0, v0, 64, 2) == 0);
        free(inc);
        free(v0);
    }
    int32_t frames[3] = {0, T / 2, T - 1};
    float *truth = (float *)malloc(sizeof(float) * 3 * (size_t)hw);
    CHECK(truth);
    CHECK(spkgen_blocks_truth(truth, H, W, frames, 3, 7, 4, 0.02, 1.0, 0.7, -0.3) == 0);
    CHECK(spkgen_gratings_truth(truth, H, W, frames, 3, 8, 1000.0) == 0);
    free(truth);
    int32_t t_out[6] = {T - 1, 0, T / 3, T / 3, T - 1, T / 2};
    const int32_t n_out = 6;
    double *out = (double *)malloc(sizeof(double) * n_out * (size_t)hw);
    double *out2 = (double *)malloc(sizeof(double) * n_out * (size_t)hw);
    int32_t *wf = (int32_t *)malloc(sizeof(int32_t) * n_out * (size_t)hw);
    int32_t *wl = (int32_t *)malloc(sizeof(int32_t) * n_out * (size_t)hw);
    int32_t *wn = (int32_t *)malloc(sizeof(int32_t) * n_out * (size_t)hw);
    CHECK(out && out2 && wf && wl && wn);
    for (int32_t order = 1; order <= 4; order++) {
        CHECK(spk_oracle_reconstruct(s, H, W, T, 1.0, t_out, n_out, order, out, wf, wl, wn, 3) ==
              0);
        CHECK(spk_oracle_reconstruct_causal(s, H, W, T, 1.0, t_out, n_out, order, out2, NULL,
                                            NULL, NULL, 2) == 0);
        const int32_t cap = 3;
        int32_t *sf = (int32_t *)malloc(sizeof(int32_t) * cap * (size_t)hw);
        int32_t *sl = (int32_t *)malloc(sizeof(int32_t) * cap * (size_t)hw);
        int32_t *sn = (int32_t *)malloc(sizeof(int32_t) * cap * (size_t)hw);
        int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)hw);
        CHECK(sf && sl && sn && cnt);
        CHECK(spk_oracle_segments(s, H, W, T, order, cap, sf, sl, sn, cnt, 4) == 0);
        CHECK(spk_oracle_segments(s, H, W, T, order, 0, NULL, NULL, NULL, cnt, 1) == 0);
        free(sf);
        free(sl);
        free(sn);
        free(cnt);
        /* the carry-state form, fed in ragged pieces, equals the single pass */
        spk_oracle_stream *st =
            spk_oracle_stream_create(H, W, 1.0, order, t_out, n_out, out2, NULL, NULL, NULL);
        CHECK(st);
        for (int32_t a = 0; a < T;) {
            const int32_t n = a % 3 == 0 ? 1 : 17;
            const int32_t m = a + n > T ? T - a : n;
            CHECK(spk_oracle_stream_feed(st, s + (size_t)a * fb, m) == 0);
            a += m;
        }
        CHECK(spk_oracle_stream_feed(st, s, 0) == 0);
        CHECK(spk_oracle_stream_finish(st) == 0);
        spk_oracle_stream_destroy(st);
        CHECK(memcmp(out, out2, sizeof(double) * n_out * (size_t)hw) == 0);
    }
    if (T >= 32) {
        double *est = (double *)malloc(sizeof(double) * (size_t)hw);
        uint8_t *stable = (uint8_t *)malloc((size_t)hw);
        CHECK(est && stable);
        CHECK(spk_oracle_window(s, H, W, T, 1.0, 31, est, stable) == 0);
        CHECK(spk_oracle_window(s, H, W, T, 1.0, T - 1, est, stable) == 0);
        free(est);
        free(stable);
    }
    CHECK(spk_oracle_tfp(s, H, W, T, 1.0, 32, t_out, n_out, out) == 0);
    CHECK(spk_oracle_tfp(s, H, W, T, 1.0, 1, t_out, n_out, out) == 0);
    free(out);
    free(out2);
    free(wf);
    free(wl);
    free(wn);
    free(s);
    return 0;
}

int main(void)
{
    /* interval lists directly: empty, one, alternating, a long constant run */
    int32_t x[200], start[200];
    for (int i = 0; i < 200; i++) x[i] = i < 100 ? 3 + (i % 2) : 7 + (i % 5 == 0);
    for (int32_t order = 1; order <= 4; order++) {
        CHECK(spk_oracle_segment_intervals(x, 0, order, start) == 0);
        CHECK(spk_oracle_segment_intervals(x, 1, order, start) == 1);
        CHECK(spk_oracle_segment_intervals(x, 200, order, start) >= 1);
    }
    CHECK(spk_oracle_segment_intervals(x, 5, 9, start) == -1);
    const int32_t shapes[][3] = {{1, 1, 1}, {1, 7, 40}, {3, 5, 64}, {9, 13, 200}, {16, 16, 333}};
    for (int k = 0; k < 5; k++)
        for (int kind = 0; kind < 3; kind++)
            if (run_shape(shapes[k][0], shapes[k][1], shapes[k][2], kind)) return 1;
    printf("sanitized run ok\n");
    return 0;
}
