/*
 * CPU replay of the library's Eq. 6 quotient (test infrastructure).
 *
 * The reconstruction kernels evaluate a segment's intensity
 * theta * N / D (Eq. 6, with the 8-bit scale replaced by theta) as a double
 * quotient x / d, x = theta * N (rounded to double), d = D, and round it once
 * to float.  On the GPU the quotient is formed from the hardware reciprocal
 * y0 ~ 1/d by two Newton-Raphson refinements y <- y + y * (1 - d * y), the
 * product q = x * y, its residual r = x - d * q (one fma, exact) and one
 * correction q + r * y (Markstein's method), without the exponent scaling
 * and special-case steps of a general IEEE division.
 *
 * The reciprocal instruction's exact output is not modelled here.  Instead
 * each check starts from y0 = RN(1/d) * (1 + delta) for a set of relative
 * errors delta far larger than any hardware reciprocal's, in both
 * directions, and requires the replayed quotient to equal the correctly
 * rounded double x / d exactly.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static double replay(double x, double d, double y0, int32_t nr)
{
    double y = y0;
    for (int32_t i = 0; i < nr; i++) {
        const double e = fma(-d, y, 1.0);
        y = fma(y, e, y);
    }
    const double q = x * y;
    const double r = fma(-d, q, x);
    return fma(r, y, q);
}

/* Check every d in [d0, d1) against every x in xs[0..nx) and every
 * perturbation in deltas[0..nd), with nr refinements (the library uses 2).
 * Returns the number of mismatches; the first one is stored in bad[0..2]
 * (x, d, delta). */
int64_t check_range(int64_t d0, int64_t d1, const double *xs, int32_t nx, const double *deltas,
                    int32_t nd, int32_t nr, double *bad)
{
    int64_t fails = 0;
    for (int64_t di = d0; di < d1; di++) {
        const double d = (double)di;
        const double r0 = 1.0 / d;
        for (int32_t k = 0; k < nd; k++) {
            const double y0 = r0 * (1.0 + deltas[k]);
            for (int32_t i = 0; i < nx; i++) {
                const double got = replay(xs[i], d, y0, nr);
                const double want = xs[i] / d;
                if (memcmp(&got, &want, sizeof got) != 0) {
                    if (fails == 0) {
                        bad[0] = xs[i];
                        bad[1] = d;
                        bad[2] = deltas[k];
                    }
                    fails++;
                }
            }
        }
    }
    return fails;
}

/* The same on explicit (x, d) pairs (random samples of the whole domain). */
int64_t check_pairs(const double *xs, const double *ds, int64_t n, const double *deltas,
                    int32_t nd, int32_t nr, double *bad)
{
    int64_t fails = 0;
    for (int64_t j = 0; j < n; j++) {
        const double r0 = 1.0 / ds[j];
        for (int32_t k = 0; k < nd; k++) {
            const double got = replay(xs[j], ds[j], r0 * (1.0 + deltas[k]), nr);
            const double want = xs[j] / ds[j];
            if (memcmp(&got, &want, sizeof got) != 0) {
                if (fails == 0) {
                    bad[0] = xs[j];
                    bad[1] = ds[j];
                    bad[2] = deltas[k];
                }
                fails++;
            }
        }
    }
    return fails;
}
