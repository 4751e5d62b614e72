/*
 * Seeded synthetic spike-camera streams.
 *
 * This module is input generation only: it models the sensor (the discrete
 * integrate-and-fire of Eq. 2 with a subtract-threshold reset, Sec. II) and
 * writes bit-packed binary frames. It holds none of the reconstruction
 * arithmetic; both the reference oracle and the GPU library consume what it
 * writes.
 *
 * Frame layout (shared with the library's ABI): frame t starts at byte
 * t * fb with fb = ceil(H*W / 128) * 16; pixel p = y*W + x is bit (p & 7) of
 * byte (p >> 3), least significant bit first; padding bits are zero.
 *
 * Randomness: a counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA 2014,
 * with Stafford's "mix13" finaliser).  Value i of stream (seed, tag) is
 * mix(key + gamma * (i + 1)) with key = mix(seed + gamma * (tag + 1)), so
 * every pixel-frame draw is independent of thread count and visiting order.
 *
 * All accumulators are integers, so a stream is reproducible bit for bit on
 * any host.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

enum {
    TAG_V0 = 1,       /* initial accumulator per pixel            */
    TAG_BLOCK = 2,    /* block intensity                          */
    TAG_SCENE = 3,    /* grating / disk parameters                */
    TAG_POISSON = 4,  /* photon count per pixel-frame             */
    TAG_SECTOR = 5,   /* disk sector intensities                  */
};

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t rng_key(uint64_t seed, uint64_t tag)
{
    return mix64(seed + GAMMA * (tag + 1));
}

static inline uint64_t rng_at(uint64_t key, uint64_t i)
{
    return mix64(key + GAMMA * (i + 1));
}

/* uniform double in [0, 1) from the top 53 bits */
static inline double u01(uint64_t v)
{
    return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

uint64_t spkgen_rng_u64(uint64_t seed, uint64_t tag, uint64_t i)
{
    return rng_at(rng_key(seed, tag), i);
}

size_t spkgen_frame_bytes(int32_t H, int32_t W)
{
    if (H <= 0 || W <= 0) return 0;
    size_t hw = (size_t)H * (size_t)W;
    return ((hw + 127) / 128) * 16;
}

/* ------------------------------------------------------------------------ */
/* threading: pixel ranges aligned to 64 pixels so no two threads share a    */
/* byte of the output                                                        */

typedef struct job job_t;
typedef void (*range_fn)(const job_t *j, int64_t p0, int64_t p1);

struct job {
    range_fn fn;
    uint8_t *out;
    int32_t H, W, T;
    size_t fb;
    const void *ctx;
    int64_t p0, p1;
};

static void *run_job(void *arg)
{
    job_t *j = (job_t *)arg;
    j->fn(j, j->p0, j->p1);
    return NULL;
}

static void run_pixels(range_fn fn, uint8_t *out, int32_t H, int32_t W, int32_t T,
                       const void *ctx, int nthreads)
{
    int64_t hw = (int64_t)H * W;
    size_t fb = spkgen_frame_bytes(H, W);
    memset(out, 0, fb * (size_t)T);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    int64_t groups = (hw + 63) / 64;
    if (nthreads > groups) nthreads = (int)groups;
    job_t jobs[256];
    pthread_t th[256];
    for (int i = 0; i < nthreads; i++) {
        int64_t g0 = groups * i / nthreads, g1 = groups * (i + 1) / nthreads;
        jobs[i] = (job_t){fn, out, H, W, T, fb, ctx, g0 * 64, g1 * 64 < hw ? g1 * 64 : hw};
    }
    for (int i = 1; i < nthreads; i++) pthread_create(&th[i], NULL, run_job, &jobs[i]);
    run_job(&jobs[0]);
    for (int i = 1; i < nthreads; i++) pthread_join(th[i], NULL);
}

static inline void put_spike(const job_t *j, int64_t t, int64_t p)
{
    j->out[(size_t)t * j->fb + (size_t)(p >> 3)] |= (uint8_t)(1u << (p & 7));
}

/* ------------------------------------------------------------------------ */
/* 1. per-pixel increments given directly (tests, closed forms)              */

typedef struct {
    const int64_t *inc; /* [T][H*W] or [H*W] when per_frame == 0 */
    const int64_t *v0;  /* [H*W] */
    int64_t theta;
    int per_frame;
} inc_ctx;

static void inc_range(const job_t *j, int64_t p0, int64_t p1)
{
    const inc_ctx *c = (const inc_ctx *)j->ctx;
    int64_t hw = (int64_t)j->H * j->W;
    for (int64_t p = p0; p < p1; p++) {
        int64_t v = c->v0[p];
        for (int64_t t = 0; t < j->T; t++) {
            v += c->per_frame ? c->inc[t * hw + p] : c->inc[p];
            if (v >= c->theta) {
                put_spike(j, t, p);
                v -= c->theta;
            }
        }
    }
}

/* Integrate-and-fire with subtract reset (Eq. 2): V(n) = V-(n-1) + inc(n);
 * a spike when V(n) >= theta, then V-(n) = V(n) - theta.  At most one spike
 * per frame; a residual at or above theta carries to the next frame. */
int spkgen_from_increments(uint8_t *out, int32_t H, int32_t W, int32_t T,
                           const int64_t *inc, int32_t per_frame, const int64_t *v0,
                           int64_t theta, int32_t nthreads)
{
    if (!out || !inc || !v0 || H <= 0 || W <= 0 || T <= 0 || theta <= 0) return -1;
    inc_ctx c = {inc, v0, theta, per_frame};
    run_pixels(inc_range, out, H, W, T, &c, nthreads);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 2. piecewise-constant blocks, optionally translating                      */

typedef struct {
    uint64_t seed;
    int32_t block, nbx, nby;
    int64_t theta;
    int64_t vx_fp, vy_fp; /* velocity in 1/65536 px per frame */
    int64_t *q;           /* [nby*nbx] increments per frame   */
} blk_ctx;

static inline int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
    return q;
}

static inline int64_t pos_mod(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

/* block index under pixel (x, y) at frame n: the scene point seen by the
 * pixel centre at the frame's midpoint, (x + 1/2 - vx (n + 1/2), ...),
 * in units of 1/131072 px so the arithmetic is exact */
static inline int64_t blk_at(const blk_ctx *c, int64_t x, int64_t y, int64_t n)
{
    const int64_t F2 = 131072;
    int64_t X = x * F2 + F2 / 2 - c->vx_fp * (2 * n + 1);
    int64_t Y = y * F2 + F2 / 2 - c->vy_fp * (2 * n + 1);
    int64_t bx = pos_mod(floor_div(X, F2 * c->block), c->nbx);
    int64_t by = pos_mod(floor_div(Y, F2 * c->block), c->nby);
    return by * c->nbx + bx;
}

static void blk_range(const job_t *j, int64_t p0, int64_t p1)
{
    const blk_ctx *c = (const blk_ctx *)j->ctx;
    uint64_t kv = rng_key(c->seed, TAG_V0);
    int moving = (c->vx_fp != 0 || c->vy_fp != 0);
    for (int64_t p = p0; p < p1; p++) {
        int64_t x = p % j->W, y = p / j->W;
        int64_t v = (int64_t)(rng_at(kv, (uint64_t)p) % (uint64_t)c->theta);
        int64_t q = c->q[blk_at(c, x, y, 0)];
        for (int64_t t = 0; t < j->T; t++) {
            if (moving) q = c->q[blk_at(c, x, y, t)];
            v += q;
            if (v >= c->theta) {
                put_spike(j, t, p);
                v -= c->theta;
            }
        }
    }
}

static int blk_setup(blk_ctx *c, int32_t H, int32_t W, uint64_t seed, int32_t block,
                     double qmin, double qmax, double vx, double vy)
{
    if (block <= 0 || !(qmin >= 0.0) || !(qmax <= 1.0) || !(qmin <= qmax)) return -1;
    c->seed = seed;
    c->block = block;
    c->nbx = (W + block - 1) / block;
    c->nby = (H + block - 1) / block;
    c->theta = 65536;
    c->vx_fp = llround(vx * 65536.0);
    c->vy_fp = llround(vy * 65536.0);
    c->q = (int64_t *)malloc(sizeof(int64_t) * (size_t)c->nbx * (size_t)c->nby);
    if (!c->q) return -2;
    uint64_t kb = rng_key(seed, TAG_BLOCK);
    for (int64_t b = 0; b < (int64_t)c->nbx * c->nby; b++) {
        double q = qmin + (qmax - qmin) * u01(rng_at(kb, (uint64_t)b));
        c->q[b] = llround(q * (double)c->theta);
    }
    return 0;
}

/* Blocks of block x block pixels, each with a constant intensity
 * q ~ U[qmin, qmax] (increment round(q * 65536) against a threshold of
 * 65536), the whole pattern translating by (vx, vy) px per frame on a torus.
 * Each pixel's initial accumulator is uniform in [0, threshold). */
int spkgen_blocks(uint8_t *out, int32_t H, int32_t W, int32_t T, uint64_t seed,
                  int32_t block, double qmin, double qmax, double vx, double vy,
                  int32_t nthreads)
{
    if (!out || H <= 0 || W <= 0 || T <= 0) return -1;
    blk_ctx c;
    int rc = blk_setup(&c, H, W, seed, block, qmin, qmax, vx, vy);
    if (rc) return rc;
    run_pixels(blk_range, out, H, W, T, &c, nthreads);
    free(c.q);
    return 0;
}

/* Ground truth of the blocks scene: intensity q = increment / threshold of
 * the block under each pixel at frame t, for each requested frame. */
int spkgen_blocks_truth(float *out, int32_t H, int32_t W, const int32_t *frames,
                        int32_t n_frames, uint64_t seed, int32_t block, double qmin,
                        double qmax, double vx, double vy)
{
    if (!out || H <= 0 || W <= 0 || n_frames < 0 || (n_frames > 0 && !frames)) return -1;
    blk_ctx c;
    int rc = blk_setup(&c, H, W, seed, block, qmin, qmax, vx, vy);
    if (rc) return rc;
    int64_t hw = (int64_t)H * W;
    for (int32_t k = 0; k < n_frames; k++)
        for (int64_t p = 0; p < hw; p++)
            out[k * hw + p] =
                (float)((double)c.q[blk_at(&c, p % W, p / W, frames[k])] / (double)c.theta);
    free(c.q);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3. moving gratings + rotating sectored disk, Poisson photon noise         */

#define SIN_N 4096
#define LEVELS 1024

typedef struct {
    uint64_t seed;
    int32_t ng;
    double kx[3], ky[3], w[3], ph[3]; /* phase = kx x + ky y - w n + ph (cycles) */
    double cx, cy, r, omega;          /* disk, omega in cycles per frame   */
    int32_t ns;
    double sector[16];
    double phi;                       /* photons per threshold             */
    int64_t theta;
    double sin_tab[SIN_N + 1];
    double *cdf[LEVELS + 1];          /* Poisson CDF per intensity level   */
    int32_t cdf_len[LEVELS + 1];
    int32_t *guide[LEVELS + 1];       /* guide table (Chen and Asau 1974)  */
    double *ang;                      /* per-pixel polar angle (cycles)    */
} grt_ctx;

static double sin_cycles(const grt_ctx *c, double cyc)
{
    cyc -= floor(cyc);
    double f = cyc * SIN_N;
    int i = (int)f;
    if (i >= SIN_N) i = SIN_N - 1;
    double a = f - i;
    return c->sin_tab[i] + a * (c->sin_tab[i + 1] - c->sin_tab[i]);
}

/* intensity level in [10, 1024] (units of 1/1024) from a value in [0, 1] */
static inline int level_of(double v)
{
    double inten = 0.01 + 0.99 * v;
    int L = (int)(inten * LEVELS + 0.5);
    if (L < 10) L = 10;
    if (L > LEVELS) L = LEVELS;
    return L;
}

/* scene value in [0, 1] at pixel (x, y), frame n: the disk's sector value
 * inside the disk, else the mean of the gratings; both sampled at the pixel
 * centre and the frame midpoint */
static double grt_value(const grt_ctx *c, int64_t p, int64_t x, int64_t y, int64_t n)
{
    double px = x + 0.5, py = y + 0.5, tn = n + 0.5;
    double dx = px - c->cx, dy = py - c->cy;
    if (dx * dx + dy * dy <= c->r * c->r) {
        double a = c->ang[p] - c->omega * tn;
        a -= floor(a);
        int s = (int)(a * c->ns);
        if (s >= c->ns) s = c->ns - 1;
        return c->sector[s];
    }
    double v = 0.0;
    for (int g = 0; g < c->ng; g++)
        v += 0.5 + 0.5 * sin_cycles(c, c->kx[g] * px + c->ky[g] * py - c->w[g] * tn + c->ph[g]);
    return v / c->ng;
}

/* inversion: the smallest k with cdf[k] > u, started from the guide entry
 * of u's bucket (the guide holds the answer for the bucket's lower edge) */
static int64_t poisson_from_cdf(const grt_ctx *c, int level, double u)
{
    const double *cdf = c->cdf[level];
    int32_t n = c->cdf_len[level];
    int32_t k = c->guide[level][(int32_t)(u * n)];
    while (cdf[k] <= u) k++;
    return k;
}

static void grt_range(const job_t *j, int64_t p0, int64_t p1)
{
    const grt_ctx *c = (const grt_ctx *)j->ctx;
    uint64_t kv = rng_key(c->seed, TAG_V0);
    uint64_t kp = rng_key(c->seed, TAG_POISSON);
    for (int64_t p = p0; p < p1; p++) {
        int64_t x = p % j->W, y = p / j->W;
        int64_t v = (int64_t)(rng_at(kv, (uint64_t)p) % (uint64_t)c->theta);
        for (int64_t t = 0; t < j->T; t++) {
            int L = level_of(grt_value(c, p, x, y, t));
            double u = u01(rng_at(kp, (uint64_t)p * (uint64_t)j->T + (uint64_t)t));
            v += poisson_from_cdf(c, L, u);
            if (v >= c->theta) {
                put_spike(j, t, p);
                v -= c->theta;
            }
        }
    }
}

static void grt_free(grt_ctx *c)
{
    for (int L = 0; L <= LEVELS; L++) {
        free(c->cdf[L]);
        free(c->guide[L]);
    }
    free(c->ang);
}

static int grt_setup(grt_ctx *c, int32_t H, int32_t W, uint64_t seed, double phi)
{
    memset(c, 0, sizeof(*c));
    if (!(phi >= 1.0) || !(phi <= 1e6)) return -1;
    c->seed = seed;
    c->phi = phi;
    c->theta = llround(phi);
    for (int i = 0; i <= SIN_N; i++) c->sin_tab[i] = sin(2.0 * M_PI * (double)i / SIN_N);
    uint64_t ks = rng_key(seed, TAG_SCENE);
    uint64_t i = 0;
#define U() u01(rng_at(ks, i++))
    c->ng = 1 + (int)(U() * 3.0);
    if (c->ng > 3) c->ng = 3;
    for (int g = 0; g < c->ng; g++) {
        double period = 4.0 + 60.0 * U();
        double orient = M_PI * U();
        double speed = 0.01 + 0.49 * U();
        c->kx[g] = cos(orient) / period;
        c->ky[g] = sin(orient) / period;
        c->w[g] = speed / period;
        c->ph[g] = U();
    }
    c->cx = W * U();
    c->cy = H * U();
    c->r = 30.0 + 70.0 * U();
    c->ns = 8 + (int)(U() * 9.0);
    if (c->ns > 16) c->ns = 16;
    double rim = 0.05 + 0.45 * U();
    double sgn = U() < 0.5 ? -1.0 : 1.0;
    c->omega = sgn * rim / (2.0 * M_PI * c->r);
#undef U
    uint64_t kq = rng_key(seed, TAG_SECTOR);
    for (int s = 0; s < c->ns; s++) c->sector[s] = u01(rng_at(kq, (uint64_t)s));
    int64_t hw = (int64_t)H * W;
    c->ang = (double *)malloc(sizeof(double) * (size_t)hw);
    if (!c->ang) return -2;
    for (int64_t p = 0; p < hw; p++) {
        double a = atan2(p / W + 0.5 - c->cy, p % W + 0.5 - c->cx) / (2.0 * M_PI);
        c->ang[p] = a - floor(a);
    }
    /* Poisson(lambda) CDF per level, lambda = phi * L / 1024, until it
     * reaches 1 in double precision */
    for (int L = 0; L <= LEVELS; L++) {
        double lam = phi * (double)L / LEVELS;
        int32_t cap = (int32_t)(lam + 20.0 * sqrt(lam + 1.0) + 40.0);
        c->cdf[L] = (double *)malloc(sizeof(double) * (size_t)cap);
        if (!c->cdf[L]) return -2;
        double pk = exp(-lam), acc = 0.0;
        int32_t k = 0;
        /* start from the mode in log space to avoid underflow of exp(-lam) */
        if (pk == 0.0) {
            acc = 0.0;
            for (k = 0; k < cap; k++) {
                double lp = -lam + k * log(lam) - lgamma(k + 1.0);
                acc += exp(lp);
                c->cdf[L][k] = acc;
                if (acc >= 1.0) break;
            }
        } else {
            for (k = 0; k < cap; k++) {
                acc += pk;
                c->cdf[L][k] = acc;
                if (acc >= 1.0) break;
                pk *= lam / (double)(k + 1);
            }
        }
        if (k >= cap) k = cap - 1;
        c->cdf[L][k] = 2.0; /* every u in [0,1) resolves */
        c->cdf_len[L] = k + 1;
        int32_t n = k + 1;
        c->guide[L] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
        if (!c->guide[L]) return -2;
        int32_t g = 0;
        for (int32_t b = 0; b <= n; b++) {
            double edge = (double)b / n;
            while (g < n - 1 && c->cdf[L][g] <= edge) g++;
            c->guide[L][b] = g;
        }
    }
    return 0;
}

/* One to three sinusoidal gratings (period U[4,64] px, orientation U[0,pi),
 * speed U[0.01,0.5] px/frame along the normal) averaged, plus a rotating
 * disk (radius U[30,100] px, 8-16 sectors of random intensity, rim speed
 * U[0.05,0.5] px/frame).  Intensity in [0.01, 1] quantised to 1/1024; the
 * photons of a frame are Poisson(phi * intensity) against a threshold of
 * phi photons. */
int spkgen_gratings(uint8_t *out, int32_t H, int32_t W, int32_t T, uint64_t seed,
                    double phi, int32_t nthreads)
{
    if (!out || H <= 0 || W <= 0 || T <= 0) return -1;
    grt_ctx *c = (grt_ctx *)malloc(sizeof(grt_ctx));
    if (!c) return -2;
    int rc = grt_setup(c, H, W, seed, phi);
    if (rc == 0) run_pixels(grt_range, out, H, W, T, c, nthreads);
    grt_free(c);
    free(c);
    return rc;
}

/* Ground truth of the gratings scene: intensity (level / 1024) per pixel at
 * each requested frame. */
int spkgen_gratings_truth(float *out, int32_t H, int32_t W, const int32_t *frames,
                          int32_t n_frames, uint64_t seed, double phi)
{
    if (!out || H <= 0 || W <= 0 || n_frames < 0 || (n_frames > 0 && !frames)) return -1;
    grt_ctx *c = (grt_ctx *)malloc(sizeof(grt_ctx));
    if (!c) return -2;
    int rc = grt_setup(c, H, W, seed, phi);
    int64_t hw = (int64_t)H * W;
    if (rc == 0)
        for (int32_t k = 0; k < n_frames; k++)
            for (int64_t p = 0; p < hw; p++)
                out[k * hw + p] =
                    (float)level_of(grt_value(c, p, p % W, p / W, frames[k])) / LEVELS;
    grt_free(c);
    free(c);
    return rc;
}
