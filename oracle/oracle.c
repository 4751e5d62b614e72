/*
 * Reference oracle for spike-stream reconstruction -- TEST INFRASTRUCTURE.
 *
 * A plain, slow, obviously correct CPU implementation of what the GPU
 * library computes, in double precision.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may build, load or call it; the product
 * path never does.  It shares no code with the GPU library.
 *
 * Paper: "High-speed and High-quality Vision Reconstruction of Spike Camera
 * with Spike Stability Theorem" (arXiv 2412.11639).  Notation follows it:
 * S0 is a pixel's binary stream, S1 = {T0(1), T0(2), ...} its inter-spike
 * intervals (Def. 2, Eq. 4), S2 the interval streams of S1 (Eq. 5).
 *
 * Steps per pixel (each function cites the passage it follows):
 *   O-1 spikes        frames whose bit is set                     (Eq. 2)
 *   O-2 intervals     T0(i) = tau(i+1) - tau(i)                   (Def. 2, Eq. 4)
 *   O-3 FSR           greedy cut where S1 leaves zero-order stability
 *                                                    (Sec. III-B; Sec. III-C module)
 *   O-4 SSR           inside each FSR segment, cut where the S2 stream of
 *                     either interval value leaves zero-order stability
 *                                                    (Sec. III-B, Fig. 1 caption)
 *   O-6 output time   the segment holding the interval in progress at t
 *   O-7 intensity     I = theta * N / sum_i T0(i)                 (Eq. 6)
 *   third order       inside each SSR piece, cut where an S3 stream (gaps of
 *                     an S2 value inside S2) leaves zero-order stability
 *                                                    (Sec. III-A, Eq. 5)
 * Baselines the paper compares against (Sec. II): TFI (every interval its
 * own segment, so I = theta / T0) as a further order, and TFP (spike count
 * over a fixed window).
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - zero-order stable == the values span at most 1 (max - min <= 1);
 *   - a violating interval closes the open segment and starts the next one;
 *   - SSR is a second stage applied inside each FSR segment; its S2 state
 *     starts empty at every FSR or SSR cut; an empty S2 is stable;
 *   - fewer than two spikes: output 0, window (-1, -1, 0);
 *   - output time t uses interval m(t) = clamp(#{spikes at frames < t}, 1, K-1)
 *     (1-based), i.e. the interval whose integration covers frame t; frames
 *     before the first spike use the first interval, after the last spike
 *     the last one;
 *   - theta scales Eq. 6 (theta = 255 gives the paper's 8-bit scale).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_FSR 1
#define ORACLE_SSR 2
#define ORACLE_TFI 3
#define ORACLE_TSR 4
#define ORACLE_ORDER_OK(o) \
    ((o) == ORACLE_FSR || (o) == ORACLE_SSR || (o) == ORACLE_TFI || (o) == ORACLE_TSR)

/* ---- O-1: spike frames of pixel p (Eq. 2: P(n) = 1 marks a spike) ------ */
static int32_t spikes_of_pixel(const uint8_t *stream, size_t fb, int32_t T, int64_t p,
                               int32_t *tau)
{
    int32_t K = 0;
    for (int32_t t = 0; t < T; t++) {
        uint8_t byte = stream[(size_t)t * fb + (size_t)(p >> 3)];
        if ((byte >> (p & 7)) & 1) tau[K++] = t;
    }
    return K;
}

/* ---- zero-order stability of a value set given by its extremes (Def. 2):
 * one value, or two values that differ by exactly 1 -------------------- */
static int zero_order_stable(int32_t lo, int32_t hi)
{
    return hi - lo <= 1;
}

/* ---- O-3: FSR (Sec. III-B "break the S1 when its elements violate the
 * zero-order stability rule"; Sec. III-C stability module: a new element that
 * keeps (e1, e2) stable is appended, one that violates pops the segment and
 * resets (e1, e2) and the sum with itself).
 * x[0..n-1] is S1; writes the first interval index of every segment to
 * start[], returns the number of segments. */
static int32_t fsr_segments(const int32_t *x, int32_t n, int32_t *start)
{
    if (n <= 0) return 0;
    int32_t nseg = 0;
    start[nseg++] = 0;
    int32_t lo = x[0], hi = x[0];
    for (int32_t m = 1; m < n; m++) {
        int32_t nlo = x[m] < lo ? x[m] : lo;
        int32_t nhi = x[m] > hi ? x[m] : hi;
        if (zero_order_stable(nlo, nhi)) {
            lo = nlo;
            hi = nhi;
        } else {
            start[nseg++] = m;
            lo = hi = x[m];
        }
    }
    return nseg;
}

/* S2 bookkeeping for one interval value inside the current SSR piece: the
 * index of its latest occurrence and the extremes of the gaps between its
 * consecutive occurrences (that gap list is S2 for this value, Eq. 5). */
typedef struct {
    int32_t value;
    int32_t last;
    int32_t gap_lo, gap_hi;
    int32_t has_gap;
} s2_track;

/* ---- O-4: SSR inside one FSR segment [s, e] (Sec. III-B: compute S2 of the
 * segmented S1 for both firing-value choices and break where they violate the
 * zero-order rule).  Appends piece starts to start[], returns the count. */
static int32_t ssr_refine(const int32_t *x, int32_t s, int32_t e, int32_t *start)
{
    int32_t nseg = 0;
    s2_track tr[2];
    int32_t ntr = 0;
    start[nseg++] = s;
    for (int32_t m = s; m <= e; m++) {
        int32_t v = x[m];
        int32_t j = -1;
        for (int32_t k = 0; k < ntr; k++)
            if (tr[k].value == v) j = k;
        if (j >= 0) {
            int32_t d = m - tr[j].last; /* a new element of S2 for value v */
            int32_t glo = tr[j].has_gap && tr[j].gap_lo < d ? tr[j].gap_lo : d;
            int32_t ghi = tr[j].has_gap && tr[j].gap_hi > d ? tr[j].gap_hi : d;
            if (!zero_order_stable(glo, ghi)) {
                /* cut before interval m: it opens the next piece, whose S2
                 * state starts empty */
                start[nseg++] = m;
                ntr = 0;
                tr[ntr++] = (s2_track){v, m, 0, 0, 0};
                continue;
            }
            tr[j].gap_lo = glo;
            tr[j].gap_hi = ghi;
            tr[j].has_gap = 1;
            tr[j].last = m;
        } else {
            /* inside an FSR segment there are at most two distinct values */
            if (ntr >= 2) abort();
            tr[ntr++] = (s2_track){v, m, 0, 0, 0};
        }
    }
    return nseg;
}

/* ---- third order: inside one SSR piece [s, e], the next stage of the
 * n-order rule (Sec. III-A, Eq. 5 applied once more; Sec. III-B: the
 * judgement extends to S3 at O(2^(n-1)) streams).  For each interval value
 * v of the open sub-piece, S2(v) is the list of gaps between its
 * consecutive occurrences; for each value g of S2(v), S3(v, g) is the list
 * of gaps between consecutive positions of g in S2(v).  The sub-piece is
 * cut before the interval whose new S2 element makes some S3(v, g) leave
 * zero-order stability; the cut opens a sub-piece whose S2 and S3 start
 * empty.  Appends sub-piece starts to start[], returns the count. */
typedef struct {
    int32_t value;   /* an element value g of S2(v) */
    int32_t last;    /* index in S2(v) of its latest occurrence */
    int32_t gap_lo, gap_hi, has_gap;
} s3_track;

typedef struct {
    int32_t value;   /* interval value v */
    int32_t last;    /* interval index of its latest occurrence */
    int32_t n2;      /* elements of S2(v) so far */
    s3_track t3[2];
    int32_t nt3;
} v_track;

static int32_t tsr_refine(const int32_t *x, int32_t s, int32_t e, int32_t *start)
{
    int32_t nseg = 0;
    v_track tr[2];
    int32_t ntr = 0;
    start[nseg++] = s;
    for (int32_t m = s; m <= e; m++) {
        int32_t v = x[m];
        int32_t j = -1;
        for (int32_t k = 0; k < ntr; k++)
            if (tr[k].value == v) j = k;
        if (j < 0) {
            /* an SSR piece holds at most two interval values */
            if (ntr >= 2) abort();
            tr[ntr].value = v;
            tr[ntr].last = m;
            tr[ntr].n2 = 0;
            tr[ntr].nt3 = 0;
            ntr++;
            continue;
        }
        v_track *t = &tr[j];
        int32_t d = m - t->last;   /* new element of S2(v), at index n2 */
        int32_t q = -1;
        for (int32_t k = 0; k < t->nt3; k++)
            if (t->t3[k].value == d) q = k;
        if (q >= 0) {
            s3_track *u = &t->t3[q];
            int32_t g = t->n2 - u->last;   /* new element of S3(v, d) */
            int32_t glo = u->has_gap && u->gap_lo < g ? u->gap_lo : g;
            int32_t ghi = u->has_gap && u->gap_hi > g ? u->gap_hi : g;
            if (!zero_order_stable(glo, ghi)) {
                start[nseg++] = m;
                ntr = 0;
                tr[ntr].value = v;
                tr[ntr].last = m;
                tr[ntr].n2 = 0;
                tr[ntr].nt3 = 0;
                ntr++;
                continue;
            }
            u->gap_lo = glo;
            u->gap_hi = ghi;
            u->has_gap = 1;
            u->last = t->n2;
        } else {
            /* S2(v) is zero-order stable inside an SSR piece: two values */
            if (t->nt3 >= 2) abort();
            t->t3[t->nt3++] = (s3_track){d, t->n2, 0, 0, 0};
        }
        t->n2++;
        t->last = m;
    }
    return nseg;
}

/* Segment S1 (n intervals) by the given order; writes segment starts,
 * returns the number of segments. work[] holds n ints. */
static int32_t segment_intervals(const int32_t *x, int32_t n, int32_t order, int32_t *start,
                                 int32_t *work)
{
    if (order == ORACLE_TFI) {
        /* TFI (Sec. II): every interval on its own, intensity theta / T0(i) */
        for (int32_t i = 0; i < n; i++) start[i] = i;
        return n;
    }
    int32_t nf = fsr_segments(x, n, order == ORACLE_FSR ? start : work);
    if (order == ORACLE_FSR) return nf;
    /* third order refines the SSR pieces, which then go to a buffer of
     * their own */
    int32_t *ssr = start;
    if (order == ORACLE_TSR) {
        ssr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        if (!ssr) abort();
    }
    int32_t ns = 0;
    for (int32_t i = 0; i < nf; i++) {
        int32_t s = work[i];
        int32_t e = (i + 1 < nf ? work[i + 1] : n) - 1;
        ns += ssr_refine(x, s, e, ssr + ns);
    }
    if (order != ORACLE_TSR) return ns;
    int32_t nt = 0;
    for (int32_t i = 0; i < ns; i++) {
        int32_t s = ssr[i];
        int32_t e = (i + 1 < ns ? ssr[i + 1] : n) - 1;
        nt += tsr_refine(x, s, e, start + nt);
    }
    free(ssr);
    return nt;
}

/* Exported: segment an interval list directly (tests). */
int32_t spk_oracle_segment_intervals(const int32_t *x, int32_t n, int32_t order,
                                     int32_t *start)
{
    if (n < 0 || (n > 0 && (!x || !start)) || !ORACLE_ORDER_OK(order))
        return -1;
    int32_t *work = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!work) return -2;
    int32_t r = segment_intervals(x, n, order, start, work);
    free(work);
    return r;
}

/* ---- per-pixel driver --------------------------------------------------- */

typedef struct {
    int32_t *tau, *x, *start, *work, *seg_of;
} scratch_t;

typedef struct {
    const uint8_t *stream;
    int32_t H, W, T;
    size_t fb;
    double theta;
    const int32_t *t_out;
    int32_t n_out;
    int32_t order;
    double *out;
    int32_t *win_first, *win_last, *win_n;
    /* segments mode */
    int32_t cap;
    int32_t *seg_first, *seg_last, *seg_n, *count;
    /* causal mode: output at t from frames 0 .. t only */
    int32_t causal;
    int64_t p0, p1;
} task_t;

/* number of spikes at frames < t (tau ascending) */
static int32_t spikes_before(const int32_t *tau, int32_t K, int32_t t)
{
    int32_t lo = 0, hi = K;
    while (lo < hi) {
        int32_t mid = (lo + hi) / 2;
        if (tau[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

static void pixel_task(const task_t *tk, scratch_t *sc, int64_t p)
{
    int64_t hw = (int64_t)tk->H * tk->W;
    int32_t K = spikes_of_pixel(tk->stream, tk->fb, tk->T, p, sc->tau); /* O-1 */
    int32_t n = K >= 2 ? K - 1 : 0;
    for (int32_t i = 0; i < n; i++) sc->x[i] = sc->tau[i + 1] - sc->tau[i]; /* O-2 */
    int32_t nseg = segment_intervals(sc->x, n, tk->order, sc->start, sc->work); /* O-3/4 */

    if (tk->count) {
        tk->count[p] = nseg;
        for (int32_t s = 0; s < nseg && s < tk->cap; s++) {
            int32_t a = sc->start[s];
            int32_t b = (s + 1 < nseg ? sc->start[s + 1] : n) - 1;
            tk->seg_first[(int64_t)s * hw + p] = sc->tau[a];
            tk->seg_last[(int64_t)s * hw + p] = sc->tau[b + 1];
            tk->seg_n[(int64_t)s * hw + p] = b - a + 1;
        }
        return;
    }

    for (int32_t s = 0; s < nseg; s++) {
        int32_t b = (s + 1 < nseg ? sc->start[s + 1] : n);
        for (int32_t i = sc->start[s]; i < b; i++) sc->seg_of[i] = s;
    }
    for (int32_t k = 0; k < tk->n_out; k++) {
        double I = 0.0;
        int32_t first = -1, last = -1, cnt = 0;
        if (tk->causal) {
            /* The method run on frames 0 .. t alone, valued at its last frame.
             * That stream holds the Kt = #{spikes at frames <= t} first spikes,
             * so its S1 is the first Kt-1 intervals of the whole stream's S1.
             * FSR and SSR decide every cut from the intervals up to the cut,
             * so its segments are the whole stream's segments cut off after
             * interval Kt-1; O-6 on it picks that last interval (t lies at or
             * after its last spike).  Result: the segment holding interval
             * Kt-1, truncated there. */
            int32_t Kt = spikes_before(sc->tau, K, tk->t_out[k] + 1);
            if (Kt >= 2) {
                int32_t i = Kt - 2;               /* 0-based index of interval Kt-1 */
                int32_t a = sc->start[sc->seg_of[i]];
                first = sc->tau[a];
                last = sc->tau[i + 1];
                cnt = i - a + 1;
                I = tk->theta * (double)cnt / (double)(last - first);
            }
        } else if (K >= 2) {
            /* O-6: interval in progress at t (1-based m, clamped to [1, K-1]) */
            int32_t m = spikes_before(sc->tau, K, tk->t_out[k]);
            if (m < 1) m = 1;
            if (m > K - 1) m = K - 1;
            int32_t s = sc->seg_of[m - 1];
            int32_t a = sc->start[s];
            int32_t b = (s + 1 < nseg ? sc->start[s + 1] : n) - 1;
            first = sc->tau[a];
            last = sc->tau[b + 1];
            cnt = b - a + 1;
            /* O-7, Eq. 6: 255 / ((1/N) sum T0(i)) with 255 -> theta; the
             * intervals of the segment sum to last - first */
            I = (tk->theta * (double)cnt) / (double)(last - first);
        }
        int64_t o = (int64_t)k * hw + p;
        if (tk->out) tk->out[o] = I;
        if (tk->win_first) tk->win_first[o] = first;
        if (tk->win_last) tk->win_last[o] = last;
        if (tk->win_n) tk->win_n[o] = cnt;
    }
}

static void *task_run(void *arg)
{
    task_t *tk = (task_t *)arg;
    size_t T1 = (size_t)tk->T + 1;
    scratch_t sc;
    sc.tau = (int32_t *)malloc(sizeof(int32_t) * T1);
    sc.x = (int32_t *)malloc(sizeof(int32_t) * T1);
    sc.start = (int32_t *)malloc(sizeof(int32_t) * T1);
    sc.work = (int32_t *)malloc(sizeof(int32_t) * T1);
    sc.seg_of = (int32_t *)malloc(sizeof(int32_t) * T1);
    if (sc.tau && sc.x && sc.start && sc.work && sc.seg_of)
        for (int64_t p = tk->p0; p < tk->p1; p++) pixel_task(tk, &sc, p);
    else
        abort();
    free(sc.tau);
    free(sc.x);
    free(sc.start);
    free(sc.work);
    free(sc.seg_of);
    return NULL;
}

static void run_all(task_t *base, int32_t nthreads)
{
    int64_t hw = (int64_t)base->H * base->W;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > hw) nthreads = (int32_t)hw;
    task_t tasks[256];
    pthread_t th[256];
    for (int32_t i = 0; i < nthreads; i++) {
        tasks[i] = *base;
        tasks[i].p0 = hw * i / nthreads;
        tasks[i].p1 = hw * (i + 1) / nthreads;
    }
    for (int32_t i = 1; i < nthreads; i++) pthread_create(&th[i], NULL, task_run, &tasks[i]);
    task_run(&tasks[0]);
    for (int32_t i = 1; i < nthreads; i++) pthread_join(th[i], NULL);
}

static size_t frame_bytes(int32_t H, int32_t W)
{
    return (((size_t)H * (size_t)W + 127) / 128) * 16;
}

/* Intensity (and window) per output time per pixel.  out/win_* are
 * [n_out][H*W]; any may be NULL.  Returns 0, or -1 on a bad argument. */
int32_t spk_oracle_reconstruct(const uint8_t *stream, int32_t H, int32_t W, int32_t T,
                               double theta, const int32_t *t_out, int32_t n_out,
                               int32_t order, double *out, int32_t *win_first,
                               int32_t *win_last, int32_t *win_n, int32_t nthreads)
{
    if (!stream || H <= 0 || W <= 0 || T <= 0 || n_out < 0 || (n_out > 0 && !t_out) ||
        !ORACLE_ORDER_OK(order))
        return -1;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0 || t_out[k] >= T) return -1;
    task_t tk;
    memset(&tk, 0, sizeof(tk));
    tk.stream = stream;
    tk.H = H;
    tk.W = W;
    tk.T = T;
    tk.fb = frame_bytes(H, W);
    tk.theta = theta;
    tk.t_out = t_out;
    tk.n_out = n_out;
    tk.order = order;
    tk.out = out;
    tk.win_first = win_first;
    tk.win_last = win_last;
    tk.win_n = win_n;
    run_all(&tk, nthreads);
    return 0;
}

/* Streaming (causal) reading: for each output time t, what the method gives
 * on the stream cut after frame t, at that frame.  Same layout and
 * arguments as spk_oracle_reconstruct. */
int32_t spk_oracle_reconstruct_causal(const uint8_t *stream, int32_t H, int32_t W, int32_t T,
                                      double theta, const int32_t *t_out, int32_t n_out,
                                      int32_t order, double *out, int32_t *win_first,
                                      int32_t *win_last, int32_t *win_n, int32_t nthreads)
{
    if (!stream || H <= 0 || W <= 0 || T <= 0 || n_out < 0 || (n_out > 0 && !t_out) ||
        !ORACLE_ORDER_OK(order))
        return -1;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0 || t_out[k] >= T) return -1;
    task_t tk;
    memset(&tk, 0, sizeof(tk));
    tk.stream = stream;
    tk.H = H;
    tk.W = W;
    tk.T = T;
    tk.fb = frame_bytes(H, W);
    tk.theta = theta;
    tk.t_out = t_out;
    tk.n_out = n_out;
    tk.order = order;
    tk.out = out;
    tk.win_first = win_first;
    tk.win_last = win_last;
    tk.win_n = win_n;
    tk.causal = 1;
    run_all(&tk, nthreads);
    return 0;
}

/* Every segment of every pixel: (first spike frame, last spike frame, number
 * of intervals) in [cap][H*W] arrays, total count per pixel in count[H*W]
 * (segments beyond cap are counted but not stored). */
int32_t spk_oracle_segments(const uint8_t *stream, int32_t H, int32_t W, int32_t T,
                            int32_t order, int32_t cap, int32_t *seg_first,
                            int32_t *seg_last, int32_t *seg_n, int32_t *count,
                            int32_t nthreads)
{
    if (!stream || H <= 0 || W <= 0 || T <= 0 || cap < 0 || !count ||
        (cap > 0 && (!seg_first || !seg_last || !seg_n)) ||
        !ORACLE_ORDER_OK(order))
        return -1;
    task_t tk;
    memset(&tk, 0, sizeof(tk));
    tk.stream = stream;
    tk.H = H;
    tk.W = W;
    tk.T = T;
    tk.fb = frame_bytes(H, W);
    tk.order = order;
    tk.cap = cap;
    tk.seg_first = seg_first;
    tk.seg_last = seg_last;
    tk.seg_n = seg_n;
    tk.count = count;
    run_all(&tk, nthreads);
    return 0;
}

/* ---- short-window estimate for the learned surrogate -------------------
 * For output time t (t >= 31) the window is the 32 frames t-31 .. t of the
 * pixel, taken as a stream of its own.  Its estimate is what O-1 .. O-7
 * give on that stream at its last frame: the FSR segment holding the last
 * interval (the interval in progress at t), intensity theta*N/D.  With
 * fewer than two spikes in the window the estimate is the fixed-window rate
 * theta*K/32 (TFP with a 32-frame window, Sec. II).  The window is "stable"
 * when FSR keeps it as one segment (at least two spikes, no cut). */
int32_t spk_oracle_window(const uint8_t *stream, int32_t H, int32_t W, int32_t T, double theta,
                          int32_t t, double *est, uint8_t *stable)
{
    if (!stream || !est || !stable || H <= 0 || W <= 0 || t < 31 || t >= T) return -1;
    size_t fb = frame_bytes(H, W);
    int64_t hw = (int64_t)H * W;
    int32_t tau[32], x[32], start[32], work[32];
    for (int64_t p = 0; p < hw; p++) {
        int32_t K = 0;
        for (int32_t j = 0; j < 32; j++) {
            int32_t f = t - 31 + j;
            if ((stream[(size_t)f * fb + (size_t)(p >> 3)] >> (p & 7)) & 1) tau[K++] = j;
        }
        if (K < 2) {
            est[p] = theta * (double)K / 32.0;
            stable[p] = 0;
            continue;
        }
        for (int32_t i = 0; i + 1 < K; i++) x[i] = tau[i + 1] - tau[i];
        int32_t nseg = segment_intervals(x, K - 1, ORACLE_FSR, start, work);
        int32_t a = start[nseg - 1];
        int32_t cnt = (K - 1) - a;
        est[p] = theta * (double)cnt / (double)(tau[K - 1] - tau[a]);
        stable[p] = nseg == 1;
    }
    return 0;
}

/* ---- TFP (Sec. II): spikes counted in a virtual exposure window of L
 * frames ending at the output frame, intensity theta * N_spk / L.  The
 * window is clipped at the stream's start (L = min(window, t + 1)).
 * out is [n_out][H*W]. */
int32_t spk_oracle_tfp(const uint8_t *stream, int32_t H, int32_t W, int32_t T, double theta,
                       int32_t window, const int32_t *t_out, int32_t n_out, double *out)
{
    if (!stream || H <= 0 || W <= 0 || T <= 0 || window < 1 || n_out < 0 ||
        (n_out > 0 && (!t_out || !out)))
        return -1;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0 || t_out[k] >= T) return -1;
    size_t fb = frame_bytes(H, W);
    int64_t hw = (int64_t)H * W;
    for (int32_t k = 0; k < n_out; k++) {
        int32_t t = t_out[k];
        int32_t f0 = t - window + 1 < 0 ? 0 : t - window + 1;
        for (int64_t p = 0; p < hw; p++) {
            int32_t cnt = 0;
            for (int32_t f = f0; f <= t; f++)
                cnt += (stream[(size_t)f * fb + (size_t)(p >> 3)] >> (p & 7)) & 1;
            out[(int64_t)k * hw + p] = theta * (double)cnt / (double)(t - f0 + 1);
        }
    }
    return 0;
}

/* ---- O-5: carry state -------------------------------------------------
 * The method run online, one spike at a time, with a small per-pixel state
 * carried from one batch of frames to the next (the FPGA design of Sec.
 * III-C processes the live stream in 32-frame blocks as they arrive).
 * Feeding a stream in any number of pieces and finishing gives exactly what
 * spk_oracle_reconstruct gives on the whole stream.
 *
 * State of one pixel: the last spike frame and the number of spikes; the
 * open FSR segment's S1 extremes (lo, hi); the S2 tracks of the open SSR
 * piece (at most two interval values: value, index of its latest
 * occurrence, extremes of its gaps) and, for the third order, the tracks of
 * the open third-order piece; the open segment's first spike and interval
 * count; and the first output (in time order) that waits for it.  The
 * three stages keep the order of the whole-stream functions above: an FSR
 * cut starts fresh SSR and third-order tracks, an SSR cut fresh SSR and
 * third-order tracks, a third-order cut fresh third-order tracks only (SSR
 * pieces do not see third-order cuts). */
typedef struct {
    int32_t lastspk, K;          /* last spike frame (-1: none), spikes so far */
    int32_t lo, hi;              /* open FSR segment: extremes of its intervals */
    s2_track tr[2];              /* open SSR piece: S2 tracks */
    int32_t ntr;
    v_track tt[2];               /* open third-order piece: tracks */
    int32_t ntt;
    int32_t seg_first, seg_n;    /* open segment: first spike, intervals */
    int32_t k0;                  /* first sorted output waiting for it */
} pixel_state;

struct spk_oracle_stream {
    int32_t H, W, order, n_out, fed;
    double theta;
    int32_t *t_sorted, *plane;   /* output times in time order (stable), their slots */
    double *out;
    int32_t *win_first, *win_last, *win_n;
    pixel_state *px;
};
typedef struct spk_oracle_stream spk_oracle_stream;

/* number of output times <= t */
static int32_t outputs_upto(const spk_oracle_stream *s, int32_t t)
{
    int32_t lo = 0, hi = s->n_out;
    while (lo < hi) {
        int32_t mid = (lo + hi) / 2;
        if (s->t_sorted[mid] <= t) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

static void put_window(const spk_oracle_stream *s, int64_t p, int32_t k0, int32_t k1,
                       int32_t first, int32_t last, int32_t n)
{
    int64_t hw = (int64_t)s->H * s->W;
    for (int32_t k = k0; k < k1; k++) {
        int64_t o = (int64_t)s->plane[k] * hw + p;
        /* O-7, Eq. 6; no interval (n = 0): 0 and the window (-1, -1, 0) */
        double I = n > 0 ? (s->theta * (double)n) / (double)(last - first) : 0.0;
        if (s->out) s->out[o] = I;
        if (s->win_first) s->win_first[o] = n > 0 ? first : -1;
        if (s->win_last) s->win_last[o] = n > 0 ? last : -1;
        if (s->win_n) s->win_n[o] = n;
    }
}

/* SSR stage on interval x at index m (inside the open FSR segment):
 * returns 1 when x opens a new SSR piece (ssr_refine's rule). */
static int ssr_step(pixel_state *q, int32_t x, int32_t m)
{
    for (int32_t k = 0; k < q->ntr; k++) {
        if (q->tr[k].value != x) continue;
        s2_track *t = &q->tr[k];
        int32_t d = m - t->last;
        int32_t glo = t->has_gap && t->gap_lo < d ? t->gap_lo : d;
        int32_t ghi = t->has_gap && t->gap_hi > d ? t->gap_hi : d;
        if (!zero_order_stable(glo, ghi)) return 1;
        t->gap_lo = glo;
        t->gap_hi = ghi;
        t->has_gap = 1;
        t->last = m;
        return 0;
    }
    if (q->ntr >= 2) abort(); /* an FSR segment holds at most two values */
    q->tr[q->ntr++] = (s2_track){x, m, 0, 0, 0};
    return 0;
}

/* third-order stage on interval x at index m (inside the open SSR piece):
 * returns 1 when x opens a new third-order piece (tsr_refine's rule). */
static int tsr_step(pixel_state *q, int32_t x, int32_t m)
{
    for (int32_t k = 0; k < q->ntt; k++) {
        if (q->tt[k].value != x) continue;
        v_track *t = &q->tt[k];
        int32_t d = m - t->last;
        int32_t j = -1;
        for (int32_t i = 0; i < t->nt3; i++)
            if (t->t3[i].value == d) j = i;
        if (j >= 0) {
            s3_track *u = &t->t3[j];
            int32_t g = t->n2 - u->last;
            int32_t glo = u->has_gap && u->gap_lo < g ? u->gap_lo : g;
            int32_t ghi = u->has_gap && u->gap_hi > g ? u->gap_hi : g;
            if (!zero_order_stable(glo, ghi)) return 1;
            u->gap_lo = glo;
            u->gap_hi = ghi;
            u->has_gap = 1;
            u->last = t->n2;
        } else {
            if (t->nt3 >= 2) abort(); /* S2 of a value inside an SSR piece */
            t->t3[t->nt3++] = (s3_track){d, t->n2, 0, 0, 0};
        }
        t->n2++;
        t->last = m;
        return 0;
    }
    if (q->ntt >= 2) abort();
    v_track *t = &q->tt[q->ntt++];
    t->value = x;
    t->last = m;
    t->n2 = 0;
    t->nt3 = 0;
    return 0;
}

static void tracks_fresh(pixel_state *q, int32_t x, int32_t m, int ssr_too)
{
    if (ssr_too) {
        q->ntr = 1;
        q->tr[0] = (s2_track){x, m, 0, 0, 0};
    }
    q->ntt = 1;
    q->tt[0].value = x;
    q->tt[0].last = m;
    q->tt[0].n2 = 0;
    q->tt[0].nt3 = 0;
}

/* One spike at frame f of pixel p. */
static void online_spike(spk_oracle_stream *s, int64_t p, int32_t f)
{
    pixel_state *q = &s->px[p];
    if (q->K == 0) {
        q->lastspk = f;
        q->K = 1;
        return;
    }
    int32_t x = f - q->lastspk;  /* O-2: interval T0 ending at this spike */
    int32_t m = q->K - 1;        /* its 0-based index in S1 */
    int cut = 0;
    if (m == 0) {
        /* the first interval opens the first segment */
        q->lo = q->hi = x;
        q->ntr = 0;
        tracks_fresh(q, x, m, 1);
        q->seg_first = q->lastspk;
        q->seg_n = 0;
        q->k0 = 0;
    } else if (s->order == ORACLE_TFI) {
        cut = 1;
    } else {
        int32_t nlo = x < q->lo ? x : q->lo, nhi = x > q->hi ? x : q->hi;
        if (!zero_order_stable(nlo, nhi)) {          /* O-3 */
            cut = 1;
            q->lo = q->hi = x;
            tracks_fresh(q, x, m, 1);
        } else {
            q->lo = nlo;
            q->hi = nhi;
            if (s->order != ORACLE_FSR) {
                if (ssr_step(q, x, m)) {             /* O-4 */
                    cut = 1;
                    tracks_fresh(q, x, m, 1);
                } else if (s->order == ORACLE_TSR && tsr_step(q, x, m)) {
                    cut = 1;
                    tracks_fresh(q, x, m, 0);
                }
            }
        }
    }
    if (cut) {
        /* the open segment ends at the previous spike: its outputs are the
         * waiting ones up to that spike (O-6) */
        int32_t kc = outputs_upto(s, q->lastspk);
        put_window(s, p, q->k0, kc, q->seg_first, q->lastspk, q->seg_n);
        q->seg_first = q->lastspk;
        q->seg_n = 0;
        q->k0 = kc;
    }
    q->seg_n++;
    q->lastspk = f;
    q->K++;
}

/* Outputs go to out / win_* ([n_out][H*W], any may be NULL) as segments
 * close; t_out in any order, times >= 0.  Returns NULL on a bad argument. */
spk_oracle_stream *spk_oracle_stream_create(int32_t H, int32_t W, double theta, int32_t order,
                                            const int32_t *t_out, int32_t n_out, double *out,
                                            int32_t *win_first, int32_t *win_last,
                                            int32_t *win_n)
{
    if (H <= 0 || W <= 0 || n_out < 0 || (n_out > 0 && !t_out) || !ORACLE_ORDER_OK(order))
        return NULL;
    for (int32_t k = 0; k < n_out; k++)
        if (t_out[k] < 0) return NULL;
    spk_oracle_stream *s = (spk_oracle_stream *)calloc(1, sizeof(*s));
    if (!s) return NULL;
    s->H = H;
    s->W = W;
    s->order = order;
    s->theta = theta;
    s->n_out = n_out;
    s->out = out;
    s->win_first = win_first;
    s->win_last = win_last;
    s->win_n = win_n;
    size_t n1 = (size_t)(n_out > 0 ? n_out : 1);
    s->t_sorted = (int32_t *)malloc(sizeof(int32_t) * n1);
    s->plane = (int32_t *)malloc(sizeof(int32_t) * n1);
    s->px = (pixel_state *)calloc((size_t)H * (size_t)W, sizeof(pixel_state));
    if (!s->t_sorted || !s->plane || !s->px) abort();
    /* time order, equal times in slot order (insertion sort: plain) */
    for (int32_t k = 0; k < n_out; k++) {
        int32_t j = k;
        while (j > 0 && s->t_sorted[j - 1] > t_out[k]) {
            s->t_sorted[j] = s->t_sorted[j - 1];
            s->plane[j] = s->plane[j - 1];
            j--;
        }
        s->t_sorted[j] = t_out[k];
        s->plane[j] = k;
    }
    for (int64_t p = 0; p < (int64_t)H * W; p++) s->px[p].lastspk = -1;
    return s;
}

/* The next nframes packed frames (frame-major, as spk_oracle_reconstruct
 * reads them). */
int32_t spk_oracle_stream_feed(spk_oracle_stream *s, const uint8_t *frames, int32_t nframes)
{
    if (!s || nframes < 0 || (nframes > 0 && !frames)) return -1;
    size_t fb = frame_bytes(s->H, s->W);
    for (int32_t j = 0; j < nframes; j++)
        for (int64_t p = 0; p < (int64_t)s->H * s->W; p++)
            if ((frames[(size_t)j * fb + (size_t)(p >> 3)] >> (p & 7)) & 1)
                online_spike(s, p, s->fed + j);
    s->fed += nframes;
    return 0;
}

/* Every output not yet written takes the open segment (times past the last
 * spike use the last interval, O-6), or 0 and (-1, -1, 0) for a pixel with
 * fewer than two spikes. */
int32_t spk_oracle_stream_finish(spk_oracle_stream *s)
{
    if (!s) return -1;
    for (int64_t p = 0; p < (int64_t)s->H * s->W; p++) {
        pixel_state *q = &s->px[p];
        if (q->K >= 2)
            put_window(s, p, q->k0, s->n_out, q->seg_first, q->lastspk, q->seg_n);
        else
            put_window(s, p, 0, s->n_out, -1, -1, 0);
    }
    return 0;
}

void spk_oracle_stream_destroy(spk_oracle_stream *s)
{
    if (!s) return;
    free(s->t_sorted);
    free(s->plane);
    free(s->px);
    free(s);
}
