/*
 * indicators.c -- FP64 CPU oracle of the quality indicators the paper
 * reports beside IGD: the hypervolume of Appendix C.2 and the expected
 * utility of the neuroevolution appendix.
 *
 * TEST INFRASTRUCTURE ONLY, like rvea_oracle.c: nothing on the product path
 * links, loads or calls it, and it shares no code with the HIP library.
 *
 * Readings (the paper gives the definitions, not these details):
 *   - "normalised objective values": f' = (f - lo) / (hi - lo) per
 *     objective, with lo and hi supplied by the caller (the known front's
 *     range for the test problems, whose fronts span [0, 1] in every
 *     objective, so f' = f there).
 *   - The reference point is the vector of ones (App. C.2); a row adds
 *     volume only inside the box [f', 1].  Rows that are not valid or have a
 *     non-finite objective are ignored.
 *   - Expected utility: the utility of a solution under weight w is -w . f'
 *     (the objectives here are minimised; the paper's rewards are
 *     maximised), and W is a finite set of weight vectors with equal
 *     probability, so EU = mean over w of max over rows of -w . f'.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "rvea_oracle.h"

/* normalised points of the valid, finite rows (n_out of them) */
static double *normalise(int m, int64_t n, const double *F, const uint8_t *valid,
                         const double *lo, const double *hi, int64_t *n_out)
{
    double *P = (double *)malloc((size_t)(n > 0 ? n : 1) * m * sizeof(double));
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (valid && !valid[i]) continue;
        int ok = 1;
        for (int j = 0; j < m; ++j) ok = ok && isfinite(F[i * m + j]);
        if (!ok) continue;
        for (int j = 0; j < m; ++j) P[k * m + j] = (F[i * m + j] - lo[j]) / (hi[j] - lo[j]);
        ++k;
    }
    *n_out = k;
    return P;
}

static int cmp_x(const void *a, const void *b)
{
    const double *p = (const double *)a, *q = (const double *)b;
    if (p[0] < q[0]) return -1;
    if (p[0] > q[0]) return 1;
    return 0;
}

/* Area dominated by 2-D points (x, y) inside the box up to (1, 1): sweep in
 * ascending x keeping the lowest y so far; the strip between consecutive
 * x values (the last one up to 1) is dominated down from height 1 to that
 * lowest y.  pts is n x 2 and is sorted here. */
static double area2(double *pts, int64_t n)
{
    qsort(pts, (size_t)n, 2 * sizeof(double), cmp_x);
    double a = 0.0, ymin = 1.0;
    for (int64_t i = 0; i < n; ++i) {
        const double x = pts[2 * i], y = pts[2 * i + 1];
        if (y < ymin) ymin = y;
        const double xn = i + 1 < n ? pts[2 * i + 2] : 1.0;
        if (ymin < 1.0) a += (xn - x) * (1.0 - ymin);
    }
    return a;
}

typedef struct {
    double z;
    int64_t i;
} zkey;

static int cmp_z(const void *a, const void *b)
{
    const zkey *p = (const zkey *)a, *q = (const zkey *)b;
    if (p->z < q->z) return -1;
    if (p->z > q->z) return 1;
    return p->i < q->i ? -1 : (p->i > q->i);
}

/* App. C.2 hypervolume with reference point (1, ..., 1), m = 2 or 3.
 * m = 2: the area of the union of the boxes [f', 1] (sweep above).
 * m = 3: slices along the third objective: between consecutive third
 * components (the last slice up to 1) the dominated cross-section is the
 * 2-D area of the points whose third component lies at or below the slice. */
double ora_hypervolume(int m, int64_t n, const double *F, const uint8_t *valid, const double *lo,
                       const double *hi)
{
    if (m < 2 || m > 3) return NAN;
    int64_t k = 0;
    double *P = normalise(m, n, F, valid, lo, hi, &k);
    /* keep the points strictly inside the reference box */
    int64_t q = 0;
    for (int64_t i = 0; i < k; ++i) {
        int in = 1;
        for (int j = 0; j < m; ++j) in = in && P[i * m + j] < 1.0;
        if (in) {
            for (int j = 0; j < m; ++j) P[q * m + j] = P[i * m + j];
            ++q;
        }
    }
    double hv = 0.0;
    if (q > 0 && m == 2) {
        hv = area2(P, q);
    } else if (q > 0) {
        zkey *Z = (zkey *)malloc((size_t)q * sizeof(zkey));
        for (int64_t i = 0; i < q; ++i) {
            Z[i].z = P[i * 3 + 2];
            Z[i].i = i;
        }
        qsort(Z, (size_t)q, sizeof(zkey), cmp_z);
        double *pts = (double *)malloc((size_t)q * 2 * sizeof(double));
        for (int64_t s = 0; s < q; ++s) {
            const double z = Z[s].z, zn = s + 1 < q ? Z[s + 1].z : 1.0;
            if (zn <= z) continue; /* empty slice (equal third components) */
            for (int64_t t = 0; t <= s; ++t) {
                pts[2 * t] = P[Z[t].i * 3];
                pts[2 * t + 1] = P[Z[t].i * 3 + 1];
            }
            hv += (zn - z) * area2(pts, s + 1);
        }
        free(pts);
        free(Z);
    }
    free(P);
    return hv;
}

/* Expected utility over the weight set W (nw x m, equal probabilities):
 * mean over w of the best utility -w . f' over the valid rows. */
double ora_expected_utility(int m, int64_t n, const double *F, const uint8_t *valid,
                            const double *lo, const double *hi, int64_t nw, const double *W)
{
    int64_t k = 0;
    double *P = normalise(m, n, F, valid, lo, hi, &k);
    if (nw < 1) {
        free(P);
        return NAN;
    }
    if (k == 0) { /* no solution: the best utility of every weight is -inf */
        free(P);
        return -INFINITY;
    }
    double sum = 0.0;
    for (int64_t w = 0; w < nw; ++w) {
        double best = -INFINITY;
        for (int64_t i = 0; i < k; ++i) {
            double u = 0.0;
            for (int j = 0; j < m; ++j) u = fma(W[w * m + j], P[i * m + j], u);
            if (-u > best) best = -u;
        }
        sum += best;
    }
    free(P);
    return sum / (double)nw;
}
