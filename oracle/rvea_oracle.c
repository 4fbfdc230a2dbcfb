/*
 * rvea_oracle.c -- plain, slow, FP64 CPU oracle of one TensorRVEA generation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the HIP
 * library; the two meet only through seeded inputs and the written contract
 * below.
 *
 * What it follows (Liang, Jiang, Sun, Cheng, "GPU-accelerated Evolutionary
 * Multiobjective Optimization Using Tensorized RVEA", GECCO'24):
 *   - Alg. 2 (main framework of RVEA, Appendix A): init, offspring, merge,
 *     RVEA selection, reference-vector update, for t = 1..t_max.
 *   - Appendix B, SBX equations (B, B', X_cross) and polynomial mutation
 *     (C, Delta, X_mut).
 *   - Alg. 1 (tensorized selection) with Eq. 2 (association), Eq. 4 (APD)
 *     and Eq. 5 (gamma).
 *   - Appendix C.2, the IGD definition.
 * Readings where the paper is silent or garbled are listed in the header of
 * each function and collected in the design notes of the repository.
 *
 * Floating point: every quantity is computed in binary64.  Genes are stored
 * as binary32 (the population tensor's storage type); a child gene is the
 * binary64 result rounded once to binary32.  Dot products and squared norms
 * are written as explicit fma() chains in ascending objective order so that
 * the operation sequence is part of the contract.  Build with
 * -ffp-contract=off.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), written here from that
 * paper's definition.  Key = (seed low 32 bits, seed high 32 bits); counter
 * = (sub-index, individual or pair, generation, stream tag).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "rvea_oracle.h"

/* ------------------------------------------------------------------------ */
/* Philox4x32-10                                                            */
/* ------------------------------------------------------------------------ */

/* One Philox S-box round: two 32x32->64 multiplies; the high halves are
 * xored with the other two counter words and the round key, the words are
 * permuted as the SC'11 paper specifies for N=4. */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        philox_round(c, k);
        /* Weyl key schedule: golden ratio and sqrt(3)-1 in 32-bit fixed point */
        k[0] += 0x9E3779B9u;
        k[1] += 0xBB67AE85u;
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

static void draw(uint64_t seed, uint32_t sub, uint32_t idx, uint32_t gen, uint32_t tag,
                 uint32_t w[4])
{
    const uint32_t ctr[4] = {sub, idx, gen, tag};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    ora_philox4x32_10(ctr, key, w);
}

/* uniform on [0,1) with 24 random bits: the top 24 bits of one word */
static double u24(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

/* uniform on [0,1) with 53 random bits from two words */
static double u53(uint32_t a, uint32_t b)
{
    const uint64_t v = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return (double)v * 0x1p-53;
}

/* uniform integer in [0, n): multiply-shift of one 32-bit word */
static uint32_t uint_below(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

static double clipd(double x, double lb, double ub)
{
    if (x < lb) x = lb;
    if (x > ub) x = ub;
    return x;
}

/* ------------------------------------------------------------------------ */
/* Reference vectors: Das-Dennis lattice (Alg. 2 input V_0, unit vectors)   */
/* ------------------------------------------------------------------------ */

int64_t ora_binomial(int64_t n, int64_t k)
{
    if (k < 0 || n < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    int64_t r = 1;
    for (int64_t i = 1; i <= k; ++i) {
        /* exact: r * (n-k+i) is divisible by i at every step */
        r = r * (n - k + i) / i;
        if (r < 0 || r > (int64_t)1 << 52) return -1;
    }
    return r;
}

int64_t ora_lattice_count(int H, int m)
{
    if (H < 1 || m < 1) return 0;
    return ora_binomial((int64_t)H + m - 1, (int64_t)m - 1);
}

/* All weight vectors w in {0,1/H,...,1}^m with sum 1.  Row order: the
 * (m-1)-subsets c_1<...<c_{m-1} of {1..H+m-1} in lexicographic order, with
 * a_i = c_i - c_{i-1} - 1 (c_0 = 0, c_m = H+m) and w_i = a_i / H.
 * Writes K = C(H+m-1, m-1) rows; returns K. */
int64_t ora_lattice(int H, int m, double *W, int64_t cap)
{
    const int64_t K = ora_lattice_count(H, m);
    if (K <= 0 || K > cap) return -1;
    const int k = m - 1;
    const int n = H + m - 1;
    int c[64];
    if (k > 63) return -1;
    for (int i = 0; i < k; ++i) c[i] = i + 1;
    for (int64_t row = 0; row < K; ++row) {
        int prev = 0;
        for (int i = 0; i < k; ++i) {
            W[row * m + i] = (double)(c[i] - prev - 1) / (double)H;
            prev = c[i];
        }
        W[row * m + (m - 1)] = (double)(H + m - prev - 1) / (double)H;
        /* next subset in lexicographic order */
        int i = k - 1;
        while (i >= 0 && c[i] == n - k + i + 1) --i;
        if (i < 0) break;
        c[i] += 1;
        for (int j = i + 1; j < k; ++j) c[j] = c[j - 1] + 1;
    }
    return K;
}

static double sqnorm(const double *a, int m)
{
    double s = a[0] * a[0];
    for (int k = 1; k < m; ++k) s = fma(a[k], a[k], s);
    return s;
}

static double dotm(const double *a, const double *b, int m)
{
    double s = a[0] * b[0];
    for (int k = 1; k < m; ++k) s = fma(a[k], b[k], s);
    return s;
}

/* v = w / ||w||_2 row by row */
void ora_normalize_rows(const double *W, int64_t K, int m, double *V)
{
    for (int64_t j = 0; j < K; ++j) {
        const double nrm = sqrt(sqnorm(W + j * m, m));
        for (int k = 0; k < m; ++k) V[j * m + k] = W[j * m + k] / nrm;
    }
}

/* ------------------------------------------------------------------------ */
/* gamma: Eq. 5 -- smallest angle from v_j to any other reference vector.   */
/* Reading: the RowMin of Alg. 1 runs over i != j (Eq. 5); the bracket of   */
/* Eq. 5 denotes the angle.  Exactly parallel vectors (cosine >= 1) are     */
/* skipped; with no other vector gamma = pi/2.                              */
/* ------------------------------------------------------------------------ */
static double gamma_one(int64_t K, int m, const double *V, const double *vn, int64_t j)
{
    double best = -2.0;
    int found = 0;
    for (int64_t i = 0; i < K; ++i) {
        if (i == j) continue;
        const double c = dotm(V + i * m, V + j * m, m) / (vn[i] * vn[j]);
        if (c >= 1.0) continue;
        if (!found || c > best) {
            best = c;
            found = 1;
        }
    }
    return found ? acos(best < -1.0 ? -1.0 : best) : 1.5707963267948966;
}

void ora_gamma_rows(int64_t K, int m, const double *V, const int64_t *rows, int64_t n,
                    double *out)
{
    double *vn = (double *)malloc(sizeof(double) * (size_t)K);
    for (int64_t j = 0; j < K; ++j) vn[j] = sqrt(sqnorm(V + j * m, m));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n; ++q) out[q] = gamma_one(K, m, V, vn, rows ? rows[q] : q);
    free(vn);
}

void ora_gamma(int64_t K, int m, const double *V, double *gamma)
{
    ora_gamma_rows(K, m, V, NULL, K, gamma);
}

/* ------------------------------------------------------------------------ */
/* Stand-in test problems.  The paper's DTLZ definitions are not part of    */
/* it; these are this repository's own synthetic problems with the same     */
/* shape: m objectives, d >= m variables in [0,1], the first m-1 variables  */
/* place a point on the front, the other k = d-m+1 set a distance term      */
/* g >= 0 that is 0 exactly when every one of them equals 1/2.              */
/*   position map: sorted position variables y_(1)<=..<=y_(m-1) give the    */
/*     uniform-spacings simplex point w = (y_(1), y_(2)-y_(1), ...,         */
/*     1-y_(m-1)), so sum(w) = 1, w >= 0.                                  */
/*   unimodal  g = (4/k) sum (z-1/2)^2                                      */
/*   multimodal g = (1/k) sum [10 (z-1/2)^2 + 2 sin^2(4 pi (z-1/2))]         */
/*   linear front: f = (1+g) w          (front: sum f = 1)                  */
/*   sphere front: f = (1+g) w/||w||    (front: sum f^2 = 1)                */
/* problem 1 = linear+multimodal, 2 = sphere+unimodal, 3 = sphere+multimodal */
/* ------------------------------------------------------------------------ */
int ora_evaluate_one(int problem, int m, int d, const float *x, double *f)
{
    if (problem < 1 || problem > 3 || m < 2 || d < m || m > 64) return ORA_EINVAL;
    double y[64], w[64];
    for (int i = 0; i < m - 1; ++i) y[i] = (double)x[i];
    /* insertion sort of the position variables */
    for (int i = 1; i < m - 1; ++i) {
        const double v = y[i];
        int j = i - 1;
        while (j >= 0 && y[j] > v) {
            y[j + 1] = y[j];
            --j;
        }
        y[j + 1] = v;
    }
    w[0] = y[0];
    for (int i = 1; i < m - 1; ++i) w[i] = y[i] - y[i - 1];
    w[m - 1] = 1.0 - y[m - 2];

    const int k = d - m + 1;
    double g = 0.0;
    for (int i = m - 1; i < d; ++i) {
        const double t = (double)x[i] - 0.5;
        if (problem == 2) {
            g += t * t;
        } else {
            const double s = sin(4.0 * M_PI * t);
            g += 10.0 * t * t + 2.0 * s * s;
        }
    }
    g = (problem == 2) ? 4.0 * g / (double)k : g / (double)k;

    if (problem == 1) {
        for (int i = 0; i < m; ++i) f[i] = (1.0 + g) * w[i];
    } else {
        const double nrm = sqrt(sqnorm(w, m));
        for (int i = 0; i < m; ++i) f[i] = (1.0 + g) * w[i] / nrm;
    }
    return ORA_OK;
}

int ora_evaluate(int problem, int m, int d, int64_t n, const float *X, int64_t ldx, double *F)
{
    if (problem < 1 || problem > 3 || m < 2 || d < m) return ORA_EINVAL;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i)
        bad |= ora_evaluate_one(problem, m, d, X + i * ldx, F + i * m) != ORA_OK;
    return bad ? ORA_EINVAL : ORA_OK;
}

/* Points of the true front, used as F* in IGD: the Das-Dennis lattice W(Hs,m)
 * (linear front) or its rows normalised (sphere front). */
int64_t ora_front(int problem, int m, int Hs, double *Fs, int64_t cap)
{
    const int64_t n = ora_lattice(Hs, m, Fs, cap);
    if (n <= 0) return n;
    if (problem != 1) ora_normalize_rows(Fs, n, m, Fs);
    return n;
}

/* IGD (Appendix C.2): mean over f* in F* of min over f in F of ||f - f*||. */
double ora_igd(const double *F, int64_t n, const double *Fs, int64_t ns, int m)
{
    double total = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t a = 0; a < ns; ++a) {
        double best = INFINITY;
        for (int64_t b = 0; b < n; ++b) {
            double s = 0.0;
            for (int k = 0; k < m; ++k) {
                const double dd = F[b * m + k] - Fs[a * m + k];
                s += dd * dd;
            }
            if (s < best) best = s;
        }
        total += sqrt(best);
    }
    return total / (double)ns;
}

/* ------------------------------------------------------------------------ */
/* Policy-rollout problem (the neuroevolution-shaped workload, m = 2).      */
/* An individual is the flattened weights of a 32 -> 64 -> 64 -> 8 tanh     */
/* policy: W1 (64x32, row-major [out][in]), b1 (64), W2 (64x64, no bias),   */
/* W3 (8x64), b3 (8): d = 6,728.  For each of E rollouts from x0[e], T      */
/* steps of  h1 = tanh(W1 x + b1), h2 = tanh(W2 h1), u = tanh(W3 h2 + b3),  */
/* x <- A x + B u;  f1 = sum_t |x_t|^2 (t = 1..T), f2 = sum_t |u_t|^2        */
/* (t = 0..T-1), each averaged over the rollouts.  Weight matrices and      */
/* every layer input are rounded to bfloat16 (round to nearest even); the   */
/* biases, A and B stay as given; sums are binary64.                        */
/* ------------------------------------------------------------------------ */
double ora_bf16(double x)
{
    /* round to nearest even at 8 significant bits (bfloat16), from binary64 */
    if (!isfinite(x) || x == 0.0) return x;
    int e;
    const double fr = frexp(x, &e);  /* |fr| in [0.5, 1) */
    const double scaled = ldexp(fr, 8);
    const double r = nearbyint(scaled); /* default rounding mode: to nearest even */
    return ldexp(r, e - 8);
}

/* out = tanh(W in + b): W already rounded, in rounded here */
static void layer(int nout, int nin, const double *W, const float *b, const double *in,
                  double *out)
{
    double inr[64];
    for (int k = 0; k < nin; ++k) inr[k] = ora_bf16(in[k]);
    for (int j = 0; j < nout; ++j) {
        double s = b ? (double)b[j] : 0.0;
        for (int k = 0; k < nin; ++k) s += W[j * nin + k] * inr[k];
        out[j] = tanh(s);
    }
}

int ora_policy_evaluate(int64_t n, const float *X, int64_t ldx, int E, int T, const float *A,
                        const float *B, const float *x0, double *F)
{
    if (E < 1 || T < 1) return ORA_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        const float *w = X + i * ldx;
        /* weight matrices in bfloat16; biases b1 (at 2048) and b3 (at 6720) as given */
        double W1[64 * 32], W2[64 * 64], W3[8 * 64];
        for (int k = 0; k < 64 * 32; ++k) W1[k] = ora_bf16((double)w[k]);
        for (int k = 0; k < 64 * 64; ++k) W2[k] = ora_bf16((double)w[2112 + k]);
        for (int k = 0; k < 8 * 64; ++k) W3[k] = ora_bf16((double)w[6208 + k]);
        const float *b1 = w + 2048, *b3 = w + 6720;
        double f1 = 0.0, f2 = 0.0;
        for (int e = 0; e < E; ++e) {
            double x[32], h1[64], h2[64], u[8], xn[32];
            for (int k = 0; k < 32; ++k) x[k] = (double)x0[e * 32 + k];
            for (int t = 0; t < T; ++t) {
                layer(64, 32, W1, b1, x, h1);
                layer(64, 64, W2, NULL, h1, h2);
                layer(8, 64, W3, b3, h2, u);
                for (int q = 0; q < 8; ++q) f2 += u[q] * u[q];
                for (int r = 0; r < 32; ++r) {
                    double s = 0.0;
                    for (int k = 0; k < 32; ++k) s += (double)A[r * 32 + k] * x[k];
                    for (int q = 0; q < 8; ++q) s += (double)B[r * 8 + q] * u[q];
                    xn[r] = s;
                }
                for (int r = 0; r < 32; ++r) {
                    x[r] = xn[r];
                    f1 += x[r] * x[r];
                }
            }
        }
        F[i * 2 + 0] = f1 / (double)E;
        F[i * 2 + 1] = f2 / (double)E;
    }
    return ORA_OK;
}

/* Gaussian initialization N(0, sigma) clipped to [lb, ub]: the four words of
 * counter (q, i, 0, TAG_INIT) give two Box-Muller pairs for genes 4q..4q+3:
 * u1 = (top 24 bits + 1)/2^24 in (0,1], u2 = top 24 bits / 2^24,
 * (r cos 2 pi u2, r sin 2 pi u2) with r = sqrt(-2 log u1). */
static void init_row_gauss(uint64_t seed, int64_t i, int d, double sigma, double lb, double ub,
                           float *x, double *pre)
{
    for (int q = 0; 4 * q < d; ++q) {
        uint32_t w[4];
        draw(seed, (uint32_t)q, (uint32_t)i, 0u, ORA_TAG_INIT, w);
        double z[4];
        for (int h = 0; h < 2; ++h) {
            const double u1 = (double)((w[2 * h] >> 8) + 1u) * 0x1p-24;
            const double u2 = (double)(w[2 * h + 1] >> 8) * 0x1p-24;
            const double r = sqrt(-2.0 * log(u1));
            const double a = 2.0 * M_PI * u2;
            z[2 * h] = r * cos(a);
            z[2 * h + 1] = r * sin(a);
        }
        for (int k = 0; k < 4 && 4 * q + k < d; ++k) {
            const double v = clipd(sigma * z[k], lb, ub);
            x[4 * q + k] = (float)v;
            if (pre) pre[4 * q + k] = v;
        }
    }
}

/* rows: individual index of each output row (NULL = 0..n-1); pre (nullable)
 * receives the binary64 values before rounding */
void ora_init_gauss_rows(uint64_t seed, const int64_t *rows, int64_t n, int d, double sigma,
                         double lb, double ub, float *X, double *pre)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q)
        init_row_gauss(seed, rows ? rows[q] : q, d, sigma, lb, ub, X + q * (int64_t)d,
                       pre ? pre + q * (int64_t)d : NULL);
}

/* objectives of n rows of any supported problem */
static int evaluate_any(const ora_params *P, int problem, int m, int d, int64_t n,
                        const float *X, int64_t ldx, double *F)
{
    if (problem != ORA_POLICY_LQ) return ora_evaluate(problem, m, d, n, X, ldx, F);
    const ora_lq *q = P->lq;
    if (!q || m != 2 || d != ORA_POLICY_D) return ORA_EINVAL;
    return ora_policy_evaluate(n, X, ldx, q->E, q->T, q->A, q->B, q->x0, F);
}

/* ------------------------------------------------------------------------ */
/* Initialization (Alg. 2): n randomized individuals.                       */
/* Reading: uniform in [lb, ub]; slots 0..N-1 valid, N..K-1 empty.          */
/* gene g of slot i: Philox counter (g/4, i, 0, TAG_INIT), word g%4.        */
/* ------------------------------------------------------------------------ */
static void init_row(uint64_t seed, int64_t i, int d, double lb, double ub, float *x)
{
    for (int g = 0; g < d; ++g) {
        uint32_t w[4];
        draw(seed, (uint32_t)(g / 4), (uint32_t)i, 0u, ORA_TAG_INIT, w);
        const double u = u24(w[g % 4]);
        const double span = ub - lb;
        const double scaled = span * u;
        x[g] = (float)(lb + scaled);
    }
}

void ora_init(uint64_t seed, int64_t N, int d, double lb, double ub, float *X, int64_t ldx)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) init_row(seed, i, d, lb, ub, X + i * ldx);
}

/* initial genes of the listed slots only (n x d) */
void ora_init_rows(uint64_t seed, const int64_t *rows, int64_t n, int d, double lb, double ub,
                   float *X)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) init_row(seed, rows[q], d, lb, ub, X + q * (int64_t)d);
}

/* ------------------------------------------------------------------------ */
/* Mating (Alg. 2 "generate offspring from P_t"; Appendix B partitions the  */
/* mating pool into two halves X_1, X_2).                                   */
/* Reading: the pool holds N' = 2*ceil(N/2) parents drawn uniformly with    */
/* replacement from the valid slots (listed in ascending slot order); pair  */
/* p is (pool[p], pool[p + N'/2]); draw with counter (0, p, t, TAG_MATE),   */
/* words 0 and 1.  Returns the number of valid slots (0 = nothing drawn).   */
/* ------------------------------------------------------------------------ */
int64_t ora_mate(uint64_t seed, int64_t t, int64_t K, int64_t N, const uint8_t *valid,
                 int32_t *parents)
{
    int32_t *vs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
    int64_t nv = 0;
    for (int64_t j = 0; j < K; ++j)
        if (valid[j]) vs[nv++] = (int32_t)j;
    if (nv > 0) {
        const int64_t P = (N + 1) / 2;
        for (int64_t p = 0; p < P; ++p) {
            uint32_t w[4];
            draw(seed, 0u, (uint32_t)p, (uint32_t)t, ORA_TAG_MATE, w);
            parents[2 * p + 0] = vs[uint_below(w[0], (uint32_t)nv)];
            parents[2 * p + 1] = vs[uint_below(w[1], (uint32_t)nv)];
        }
    }
    free(vs);
    return nv;
}

/* ------------------------------------------------------------------------ */
/* SBX + polynomial mutation (Appendix B).                                  */
/*                                                                          */
/* SBX, per pair p and gene g, from the word (g%4) of counter               */
/* (g/4, p, t, TAG_SBX):  M_c = top 24 bits / 2^24;  bit 7 set  <=> R_1 >= */
/* 1/2 (so sgn(R_1-1/2) = +1);  bit 6 set <=> R_2 > 1/2.  R_3 is word 0 of  */
/* counter (0, p, t, TAG_SBXPAIR) / 2^32, drawn only when p_c < 1.          */
/*   beta = (2 M_c)^(1/(eta+1))          if M_c < 1/2                       */
/*        = (2 - 2 M_c)^(-1/(eta+1))     otherwise                          */
/*   B = sgn(R_1 - 1/2) beta; B = 1 where R_2 > 1/2 or R_3 > p_c            */
/*   child1 = ((1+B) x1 + (1-B) x2) / 2, child2 = ((1-B) x1 + (1+B) x2) / 2 */
/* H(x) = [x > 0], so H(0) = 0.  Reading: children are clipped to [lb,ub]   */
/* before mutation (the mutation formula needs x in the box).               */
/* Offspring o < N'/2 is child1 of pair o, o >= N'/2 is child2 of pair      */
/* o - N'/2; only o < N is kept.                                            */
/*                                                                          */
/* Polynomial mutation: site (o, g) mutates with probability p_m/d          */
/* (C = H(p_m/d - R_4)).  Sites are drawn as geometric gaps, which gives    */
/* the same i.i.d. Bernoulli sites: event e of child o uses counter         */
/* (e, o, t, TAG_MUT); words 0,1 give U in (0,1], gap = floor(log U /       */
/* log(1-p)); words 2,3 give M_mut in [0,1) for that site.  Delta follows   */
/* Appendix B with xi = eta_m; the result is clipped to [lb,ub] and rounded */
/* to binary32.                                                             */
/* ------------------------------------------------------------------------ */
double ora_sbx_beta(double mc, double eta)
{
    const double e = 1.0 / (eta + 1.0);
    if (mc < 0.5) return pow(2.0 * mc, e);
    return pow(2.0 - 2.0 * mc, -e);
}


double ora_pm_delta(double x, double lb, double ub, double mm, double xi)
{
    const double span = ub - lb;
    const double e = 1.0 / (xi + 1.0);
    if (mm < 0.5) {
        const double d1 = (x - lb) / span;
        const double base = 2.0 * mm + (1.0 - 2.0 * mm) * pow(1.0 - d1, xi + 1.0);
        return span * (pow(base, e) - 1.0);
    }
    if (mm > 0.5) {
        const double d2 = (ub - x) / span;
        const double base = 2.0 * (1.0 - mm) + 2.0 * (mm - 0.5) * pow(1.0 - d2, xi + 1.0);
        return span * (1.0 - pow(base, e));
    }
    return 0.0;
}

/* geometric-gap sites of one child: writes up to cap ascending positions */
int ora_mutation_sites(uint64_t seed, int64_t t, int64_t o, int d, double p_m, int32_t *sites,
                       double *mags, int cap)
{
    double p = p_m / (double)d;
    if (!(p > 0.0)) return 0;
    if (p > 1.0) p = 1.0;
    const double lq = log1p(-p); /* -inf when p == 1: every gap is 0 */
    int64_t pos = -1;
    int n = 0;
    for (uint32_t e = 0;; ++e) {
        uint32_t w[4];
        draw(seed, e, (uint32_t)o, (uint32_t)t, ORA_TAG_MUT, w);
        const double U = 1.0 - u53(w[0], w[1]);
        double q = log(U) / lq;
        if (!(q >= 0.0)) q = 0.0; /* -0 or NaN guard (U == 1 or p == 1) */
        const double gap = floor(q);
        if (gap >= (double)d) break;
        pos += 1 + (int64_t)gap;
        if (pos >= d) break;
        if (n < cap) {
            sites[n] = (int32_t)pos;
            mags[n] = u53(w[2], w[3]);
        }
        ++n;
    }
    return n;
}

/* apply polynomial mutation to one child in place, site by site */
void ora_mutate_child(uint64_t seed, int64_t t, int64_t o, int d, double p_m, double lb,
                      double ub, double eta_m, double *c)
{
    double p = p_m / (double)d;
    if (!(p > 0.0)) return;
    if (p > 1.0) p = 1.0;
    const double lq = log1p(-p);
    int64_t pos = -1;
    for (uint32_t e = 0;; ++e) {
        uint32_t w[4];
        draw(seed, e, (uint32_t)o, (uint32_t)t, ORA_TAG_MUT, w);
        const double U = 1.0 - u53(w[0], w[1]);
        double q = log(U) / lq;
        if (!(q >= 0.0)) q = 0.0;
        const double gap = floor(q);
        if (gap >= (double)d) break;
        pos += 1 + (int64_t)gap;
        if (pos >= d) break;
        const double x = c[pos];
        c[pos] = clipd(x + ora_pm_delta(x, lb, ub, u53(w[2], w[3]), eta_m), lb, ub);
    }
}

/* children of pair p (Appendix B), clipped, mutated, before rounding */
static void pair_children(const ora_params *P, uint64_t seed, int64_t t, int64_t N, int d,
                          const float *x1, const float *x2, int64_t p, double *c1, double *c2)
{
    const int64_t Pp = (N + 1) / 2;
    const double lb = P->lb, ub = P->ub;
    int nocross = 0;
    if (P->p_c < 1.0) {
        uint32_t w[4];
        draw(seed, 0u, (uint32_t)p, (uint32_t)t, ORA_TAG_SBXPAIR, w);
        nocross = ((double)w[0] * 0x1p-32) > P->p_c;
    }
    for (int g = 0; g < d; ++g) {
        uint32_t w[4];
        draw(seed, (uint32_t)(g / 4), (uint32_t)p, (uint32_t)t, ORA_TAG_SBX, w);
        const uint32_t word = w[g % 4];
        const double mc = u24(word);
        const double sgn = ((word >> 7) & 1u) ? 1.0 : -1.0;
        const int r2_high = (int)((word >> 6) & 1u);
        double B = sgn * ora_sbx_beta(mc, P->eta_c);
        if (r2_high || nocross) B = 1.0;
        const double a = (double)x1[g], b = (double)x2[g];
        const double up = 1.0 + B, dn = 1.0 - B;
        const double v1 = (up * a + dn * b) / 2.0;
        const double v2 = (dn * a + up * b) / 2.0;
        c1[g] = clipd(v1, lb, ub);
        c2[g] = clipd(v2, lb, ub);
    }
    if (p < N) ora_mutate_child(seed, t, p, d, P->p_m, lb, ub, P->eta_m, c1);
    if (p + Pp < N) ora_mutate_child(seed, t, p + Pp, d, P->p_m, lb, ub, P->eta_m, c2);
}

int ora_reproduce(const ora_params *P, uint64_t seed, int64_t t, int64_t K, int64_t N, int d,
                  const float *X, int64_t ldx, const int32_t *parents, float *Xoff,
                  int64_t ldo, double *pre)
{
    (void)K;
    const int64_t Pp = (N + 1) / 2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < Pp; ++p) {
        double *c1 = (double *)malloc(sizeof(double) * (size_t)d);
        double *c2 = (double *)malloc(sizeof(double) * (size_t)d);
        pair_children(P, seed, t, N, d, X + (int64_t)parents[2 * p] * ldx,
                      X + (int64_t)parents[2 * p + 1] * ldx, p, c1, c2);
        for (int which = 0; which < 2; ++which) {
            const int64_t o = which ? p + Pp : p;
            if (o >= N) continue;
            const double *c = which ? c2 : c1;
            for (int g = 0; g < d; ++g) {
                Xoff[o * ldo + g] = (float)c[g];
                if (pre) pre[o * (int64_t)d + g] = c[g];
            }
        }
        free(c1);
        free(c2);
    }
    return ORA_OK;
}

/* Children of the listed pairs only (pairs[q] indexes the full pair list);
 * out1/out2 receive the two children of each listed pair (n x d); a child
 * index >= N is left untouched. */
int ora_reproduce_pairs(const ora_params *P, uint64_t seed, int64_t t, int64_t N, int d,
                        const float *X, int64_t ldx, const int32_t *parents, const int64_t *pairs,
                        int64_t n, float *out1, float *out2)
{
    const int64_t Pp = (N + 1) / 2;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < n; ++q) {
        const int64_t p = pairs[q];
        if (p < 0 || p >= Pp) continue;
        double *c1 = (double *)malloc(sizeof(double) * (size_t)d);
        double *c2 = (double *)malloc(sizeof(double) * (size_t)d);
        pair_children(P, seed, t, N, d, X + (int64_t)parents[2 * p] * ldx,
                      X + (int64_t)parents[2 * p + 1] * ldx, p, c1, c2);
        for (int g = 0; g < d; ++g) {
            out1[q * (int64_t)d + g] = (float)c1[g];
            if (p + Pp < N) out2[q * (int64_t)d + g] = (float)c2[g];
        }
        free(c1);
        free(c2);
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Selection (Alg. 1; Eq. 2, Eq. 4, Eq. 5).                                 */
/* Merged population: rows 0..K-1 are the parent slots, K..K+N-1 the        */
/* offspring; a row takes part iff mvalid[i] and all of F_i is finite.      */
/*   z*_k  = min over taking-part rows of F_ik            (Alg. 1)         */
/*   f'_i  = F_i - z*                                      (Alg. 1)         */
/*   A(i)  = argmax_j cos(f'_i, v_j), lowest j on ties     (Alg. 1, Eq. 2)  */
/*           (= argmin of the angle).  ||f'_i|| = 0 gives A(i) = 0,         */
/*           theta = pi/2 and APD 0.                                        */
/*   APD_i = (1 + m (t/t_max)^alpha theta_i / gamma_A(i)) ||f'_i||  (Eq. 4) */
/*   surv(j) = argmin over {i : A(i) = j} of APD_i, lowest i on ties;       */
/*             -1 when no row is associated with j (Alg. 1).                */
/* Readings: t is the 1-based generation of this selection; Alg. 1's -1     */
/* mask is the partition tensor's (an APD entry is never -1).              */
/* ------------------------------------------------------------------------ */
/* association, angle and APD of one objective row (Eq. 2, Eq. 4) */
static void assoc_one(int m, int64_t K, const double *Fi, const double *zstar, const double *V,
                      const double *vn, const double *gamma, double pen, int32_t *assoc,
                      double *theta, double *apd)
{
    double f[64] = {0};
    for (int k = 0; k < m; ++k) f[k] = Fi[k] - zstar[k];
    const double nrm = sqrt(sqnorm(f, m));
    int64_t best = 0;
    double bestc = -INFINITY;
    if (nrm > 0.0) {
        for (int64_t j = 0; j < K; ++j) {
            const double c = dotm(f, V + j * m, m) / (nrm * vn[j]);
            if (c > bestc) {
                bestc = c;
                best = j;
            }
        }
    }
    double th;
    if (nrm > 0.0) {
        double c = bestc;
        if (c > 1.0) c = 1.0;
        if (c < -1.0) c = -1.0;
        th = acos(c);
    } else {
        th = 1.5707963267948966;
    }
    *assoc = (int32_t)best;
    *theta = th;
    *apd = (1.0 + pen * th / gamma[best]) * nrm;
}

/* the same for selected rows, given the ideal point (for sampled checks of
 * populations too large for the full selection) */
void ora_assoc_rows(int m, int64_t K, int64_t t, int t_max, double alpha, const double *Frows,
                    int64_t n, const double *zstar, const double *V, const double *gamma,
                    int32_t *assoc, double *theta, double *apd)
{
    double *vn = (double *)malloc(sizeof(double) * (size_t)K);
    for (int64_t j = 0; j < K; ++j) vn[j] = sqrt(sqnorm(V + j * m, m));
    const double pen = (double)m * pow((double)t / (double)t_max, alpha);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n; ++q)
        assoc_one(m, K, Frows + q * m, zstar, V, vn, gamma, pen, assoc + q, theta + q, apd + q);
    free(vn);
}

int ora_select(int m, int64_t K, int64_t N, int64_t t, int t_max, double alpha, const double *Fm,
               const uint8_t *mvalid, const double *V, const double *gamma, double *zstar,
               int32_t *assoc, double *theta, double *apd, int32_t *surv)
{
    const int64_t M = K + N;
    if (m < 1 || m > 64 || K < 1 || N < 0) return ORA_EINVAL;
    uint8_t *take = (uint8_t *)malloc((size_t)M);
    for (int k = 0; k < m; ++k) zstar[k] = INFINITY;
    for (int64_t i = 0; i < M; ++i) {
        int ok = mvalid[i] != 0;
        for (int k = 0; k < m && ok; ++k) ok = isfinite(Fm[i * m + k]);
        take[i] = (uint8_t)ok;
        if (ok)
            for (int k = 0; k < m; ++k)
                if (Fm[i * m + k] < zstar[k]) zstar[k] = Fm[i * m + k];
    }
    double *vn = (double *)malloc(sizeof(double) * (size_t)K);
    for (int64_t j = 0; j < K; ++j) vn[j] = sqrt(sqnorm(V + j * m, m));
    const double pen = (double)m * pow((double)t / (double)t_max, alpha);

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < M; ++i) {
        if (!take[i]) {
            assoc[i] = -1;
            theta[i] = NAN;
            apd[i] = INFINITY;
            continue;
        }
        assoc_one(m, K, Fm + i * m, zstar, V, vn, gamma, pen, assoc + i, theta + i, apd + i);
    }

    for (int64_t j = 0; j < K; ++j) surv[j] = -1;
    for (int64_t i = 0; i < M; ++i) {
        if (!take[i]) continue;
        const int64_t j = assoc[i];
        if (surv[j] < 0 || apd[i] < apd[surv[j]]) surv[j] = (int32_t)i;
    }
    free(vn);
    free(take);
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Reference-vector adaptation (Alg. 2, "update V_{t+1} from V_t and V_0"). */
/* The paper gives no formula; reading: the cited RVEA's rule               */
/*   V_j = V0_j o (z_max - z_min) / || V0_j o (z_max - z_min) ||            */
/* with z_min, z_max the per-objective extremes over the valid survivors,   */
/* applied when t is a multiple of ceil(fr * t_max).  If some range is not  */
/* positive and finite, V is left unchanged.  Returns 1 if V changed.       */
/* ------------------------------------------------------------------------ */
int ora_adapt(int64_t K, int m, const double *V0, const double *F, const uint8_t *valid, double *V)
{
    double lo[64], hi[64], r[64];
    if (m < 1 || m > 64) return 0;
    for (int k = 0; k < m; ++k) {
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
    }
    for (int64_t j = 0; j < K; ++j) {
        if (!valid[j]) continue;
        for (int k = 0; k < m; ++k) {
            if (F[j * m + k] < lo[k]) lo[k] = F[j * m + k];
            if (F[j * m + k] > hi[k]) hi[k] = F[j * m + k];
        }
    }
    for (int k = 0; k < m; ++k) {
        r[k] = hi[k] - lo[k];
        if (!(r[k] > 0.0) || !isfinite(r[k])) return 0;
    }
    for (int64_t j = 0; j < K; ++j) {
        double w[64] = {0};
        for (int k = 0; k < m; ++k) w[k] = V0[j * m + k] * r[k];
        const double nrm = sqrt(sqnorm(w, m));
        for (int k = 0; k < m; ++k) V[j * m + k] = w[k] / nrm;
    }
    return 1;
}

int ora_adapt_period(double fr, int t_max)
{
    /* ceil(fr * t_max), robust to the binary64 representation of fr */
    const double x = fr * (double)t_max;
    double c = ceil(x - 1e-9 * (x > 1.0 ? x : 1.0));
    if (c < 1.0) c = 1.0;
    return (int)c;
}

/* ------------------------------------------------------------------------ */
/* One generation of Alg. 2 on an explicit state (slot-ordered X, F, valid). */
/* ------------------------------------------------------------------------ */
int ora_generation(const ora_params *P, int problem, int m, int d, int64_t N, int64_t K,
                   uint64_t seed, int64_t t, float *X, double *F, uint8_t *valid, double *V,
                   const double *V0, double *gamma, float *Xoff_out, double *Foff_out,
                   int32_t *parents_out, int32_t *surv_out, int *adapted)
{
    const int64_t Pp = (N + 1) / 2;
    const int64_t M = K + N;
    int rc = ORA_OK;
    int32_t *parents = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * Pp));
    float *Xoff = (float *)malloc(sizeof(float) * (size_t)(N * d));
    double *Fm = (double *)malloc(sizeof(double) * (size_t)(M * m));
    uint8_t *mvalid = (uint8_t *)malloc((size_t)M);
    int32_t *assoc = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    double *theta = (double *)malloc(sizeof(double) * (size_t)M);
    double *apd = (double *)malloc(sizeof(double) * (size_t)M);
    int32_t *surv = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    double zstar[64];
    if (adapted) *adapted = 0;

    if (ora_mate(seed, t, K, N, valid, parents) <= 0) {
        rc = ORA_ESTATE;
        goto out;
    }
    rc = ora_reproduce(P, seed, t, K, N, d, X, d, parents, Xoff, d, NULL);
    if (rc != ORA_OK) goto out;
    memcpy(Fm, F, sizeof(double) * (size_t)(K * m));
    rc = evaluate_any(P, problem, m, d, N, Xoff, d, Fm + K * m);
    if (rc != ORA_OK) goto out;
    for (int64_t i = 0; i < K; ++i) mvalid[i] = valid[i];
    for (int64_t i = K; i < M; ++i) mvalid[i] = 1;
    ora_select(m, K, N, t, P->t_max, P->alpha, Fm, mvalid, V, gamma, zstar, assoc, theta, apd,
               surv);
    if (Xoff_out) memcpy(Xoff_out, Xoff, sizeof(float) * (size_t)(N * d));
    if (Foff_out) memcpy(Foff_out, Fm + K * m, sizeof(double) * (size_t)(N * m));
    if (parents_out) memcpy(parents_out, parents, sizeof(int32_t) * (size_t)(2 * Pp));
    if (surv_out) memcpy(surv_out, surv, sizeof(int32_t) * (size_t)K);
    {
        /* new population: slot j <- merged row surv(j) (Alg. 1) */
        float *Xn = (float *)malloc(sizeof(float) * (size_t)(K * d));
        for (int64_t j = 0; j < K; ++j) {
            const int32_t s = surv[j];
            if (s < 0) {
                valid[j] = 0;
                memset(Xn + j * d, 0, sizeof(float) * (size_t)d);
                for (int k = 0; k < m; ++k) F[j * m + k] = NAN;
                continue;
            }
            valid[j] = 1;
            const float *src = (s < K) ? X + (int64_t)s * d : Xoff + (int64_t)(s - K) * d;
            memcpy(Xn + j * d, src, sizeof(float) * (size_t)d);
            for (int k = 0; k < m; ++k) F[j * m + k] = Fm[(int64_t)s * m + k];
        }
        memcpy(X, Xn, sizeof(float) * (size_t)(K * d));
        free(Xn);
    }
    if (t % ora_adapt_period(P->fr, P->t_max) == 0) {
        if (ora_adapt(K, m, V0, F, valid, V)) {
            ora_gamma(K, m, V, gamma);
            if (adapted) *adapted = 1;
        }
    }
out:
    free(parents);
    free(Xoff);
    free(Fm);
    free(mvalid);
    free(assoc);
    free(theta);
    free(apd);
    free(surv);
    return rc;
}

/* Whole run: lattice, init, then generations t0+1 .. t0+gens. */
int ora_run(const ora_params *P, int problem, int m, int d, int64_t N, int64_t K, uint64_t seed,
            int gens, float *X, double *F, uint8_t *valid, double *V, double *V0, double *gamma)
{
    int H = 0;
    for (int h = 1; h < 1000000; ++h) {
        const int64_t c = ora_lattice_count(h, m);
        if (c == K) {
            H = h;
            break;
        }
        if (c > K || c < 0) break;
    }
    if (H == 0 || N < 1 || N > K || d < m) return ORA_EINVAL;
    double *W = (double *)malloc(sizeof(double) * (size_t)(K * m));
    ora_lattice(H, m, W, K);
    ora_normalize_rows(W, K, m, V0);
    free(W);
    memcpy(V, V0, sizeof(double) * (size_t)(K * m));
    ora_gamma(K, m, V, gamma);
    memset(X, 0, sizeof(float) * (size_t)(K * d));
    if (problem == ORA_POLICY_LQ) {
        if (!P->lq) return ORA_EINVAL;
        ora_init_gauss_rows(seed, NULL, N, d, P->lq->sigma, P->lb, P->ub, X, NULL);
    } else {
        ora_init(seed, N, d, P->lb, P->ub, X, d);
    }
    for (int64_t j = 0; j < K; ++j) valid[j] = (uint8_t)(j < N);
    for (int64_t j = 0; j < K * m; ++j) F[j] = NAN;
    int rc = evaluate_any(P, problem, m, d, N, X, d, F);
    if (rc != ORA_OK) return rc;
    for (int64_t t = 1; t <= gens; ++t) {
        rc = ora_generation(P, problem, m, d, N, K, seed, t, X, F, valid, V, V0, gamma, NULL,
                            NULL, NULL, NULL, NULL);
        if (rc != ORA_OK) return rc;
    }
    return ORA_OK;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
