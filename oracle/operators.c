/*
 * operators.c -- FP64 CPU oracle of the other reproduction operators that
 * the paper's extensibility experiments (Sec. 4, Extensibility; the
 * appendix's setup table) put in place of the genetic operators (SBX +
 * polynomial mutation): PSO, DE, CSO, and random reproduction as the
 * baseline.  The paper names the operators but does not define them; each
 * is the update of its original method, written out below with the
 * readings this repository takes.  Selection (Alg. 1) and adaptation (Alg. 2) are the
 * ones of rvea_oracle.c, unchanged.
 *
 * TEST INFRASTRUCTURE ONLY, like rvea_oracle.c: nothing on the product path
 * links, loads or calls it, and it shares no code with the HIP library.
 *
 * Random numbers (Philox4x32-10 keyed by the run seed, as everywhere here):
 *   selection draws of unit u (a child for DE and PSO, a pair for CSO):
 *     the word stream W[0], W[1], ... of counters (e, u, t, TAG_OPSEL),
 *     e = 0, 1, ..., four words each; an index below n is (W n) >> 32
 *   per-gene uniforms: u24 of word g % 4 of counter (g / 4, u, t,
 *     TAG_OPGENE) for DE and PSO; words 0 and 1 of counter (g, u, t,
 *     TAG_OPGENE) for CSO (two uniforms per gene)
 * The population P is the valid slots in ascending order (as for mating).
 *
 * DE/rand/1/bin (Storn and Price, 1997), parameters F and CR: child o has
 * target t = P[W0], j_rand = W1 below d, and donors r1, r2, r3 drawn from
 * W2, W3, ... as P[W_i], each accepted when it differs from the target and
 * from the donors already accepted (when the population has at least four
 * members; otherwise, or after 64 candidates, every candidate is accepted).
 * Gene g takes the mutant x_r1 + F (x_r2 - x_r3) when U_g < CR or g = j_rand,
 * else the target's gene; the mutant is clipped to [lb, ub].
 *
 * PSO with inertia weight (Kennedy and Eberhart, 1995; Shi and Eberhart,
 * 1998), parameters w and c: each individual carries a velocity (zero when
 * created).  Child o is particle i = P[W0] moved toward the leader
 * l = P[W1]: v' = w v_i + c r (x_l - x_i), x' = clip(x_i + v'), and the
 * child carries v'.  Reading: the canonical update's personal-best term
 * vanishes, because each population member is the best individual found
 * for its reference vector (its own personal best), and the leader is
 * drawn uniformly from the population, every member of which is the elite
 * of its vector.
 *
 * Random reproduction (the study's baseline): every child is drawn anew,
 * gene g = lb + (ub - lb) u24(word g % 4 of counter (g / 4, o, t,
 * TAG_OPGENE)), the initialization's uniform draw (reading: uniform in the
 * box for every problem).
 *
 * CSO (Cheng and Jin, 2015), competitive swarm: pair p draws a = P[W0] and
 * b = P[W1]; the member with the smaller sum of objectives wins (ties: the
 * lower slot).  Child p (p < N' / 2) is the loser l moved toward the winner
 * w: v' = r1 v_l + r2 (x_w - x_l), x' = clip(x_l + v'); child p + N' / 2
 * is the winner, genes and velocity unchanged.  Reading: phi = 0 (no pull
 * toward the swarm mean), and the sum of objectives serves as the
 * competition's fitness.
 *
 * Arithmetic: binary64 from the binary32 genes and velocities, each
 * operation in the order written above (x_r2 - x_r3, times F, plus x_r1;
 * x_l - x_i, times r, times c, plus w v_i; x_w - x_l, times r2, plus r1
 * v_l), then rounded once to binary32.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "rvea_oracle.h"

static void words(uint64_t seed, uint32_t sub, uint32_t unit, uint32_t t, uint32_t tag,
                  uint32_t w[4])
{
    const uint32_t ctr[4] = {sub, unit, t, tag};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    ora_philox4x32_10(ctr, key, w);
}

/* word i of unit u's selection stream */
static uint32_t sel_word(uint64_t seed, int64_t u, int64_t t, int i)
{
    uint32_t w[4];
    words(seed, (uint32_t)(i / 4), (uint32_t)u, (uint32_t)t, ORA_TAG_OPSEL, w);
    return w[i % 4];
}

static uint32_t below(uint32_t w, uint32_t n) { return (uint32_t)(((uint64_t)w * n) >> 32); }
static double u24w(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }
static double clip(double x, double lb, double ub) { return x < lb ? lb : (x > ub ? ub : x); }

int ora_de_draws(uint64_t seed, int64_t t, int64_t o, int d, const int32_t *P, int64_t nv,
                 int32_t out[5])
{
    if (nv < 1) return ORA_ESTATE;
    const int32_t tgt = P[below(sel_word(seed, o, t, 0), (uint32_t)nv)];
    const int32_t jr = (int32_t)below(sel_word(seed, o, t, 1), (uint32_t)d);
    int32_t r[3];
    int n = 0;
    for (int i = 2; n < 3; ++i) {
        const int32_t c = P[below(sel_word(seed, o, t, i), (uint32_t)nv)];
        int ok = 1;
        if (nv >= 4 && i < 66) {
            ok = c != tgt;
            for (int k = 0; k < n; ++k) ok = ok && c != r[k];
        }
        if (ok) r[n++] = c;
    }
    out[0] = tgt;
    out[1] = r[0];
    out[2] = r[1];
    out[3] = r[2];
    out[4] = jr;
    return ORA_OK;
}

static double fitness(const double *F, int m, int32_t s)
{
    double a = 0.0;
    for (int k = 0; k < m; ++k) a += F[(int64_t)s * m + k];
    return a;
}

int ora_reproduce_op(const ora_params *Pr, const ora_op *op, uint64_t seed, int64_t t,
                     int64_t K, int64_t N, int d, int m, const float *X, const float *Vel,
                     const uint8_t *valid, const double *F, float *Xoff, float *Voff)
{
    int32_t *P = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
    int64_t nv = 0;
    for (int64_t j = 0; j < K; ++j)
        if (valid[j]) P[nv++] = (int32_t)j;
    if (nv == 0) {
        free(P);
        return ORA_ESTATE;
    }
    const double lb = Pr->lb, ub = Pr->ub;
    if (op->op == ORA_OP_DE) {
        const double Fm = op->a, CR = op->b;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t o = 0; o < N; ++o) {
            int32_t dr[5];
            ora_de_draws(seed, t, o, d, P, nv, dr);
            const float *xt = X + (int64_t)dr[0] * d, *x1 = X + (int64_t)dr[1] * d;
            const float *x2 = X + (int64_t)dr[2] * d, *x3 = X + (int64_t)dr[3] * d;
            for (int g = 0; g < d; ++g) {
                uint32_t w[4];
                words(seed, (uint32_t)(g / 4), (uint32_t)o, (uint32_t)t, ORA_TAG_OPGENE, w);
                double v = (double)xt[g];
                if (u24w(w[g % 4]) < CR || g == dr[4]) {
                    const double diff = (double)x2[g] - (double)x3[g];
                    const double step = Fm * diff;
                    v = clip((double)x1[g] + step, lb, ub);
                }
                Xoff[o * (int64_t)d + g] = (float)v;
                if (Voff) Voff[o * (int64_t)d + g] = 0.0f;
            }
        }
    } else if (op->op == ORA_OP_PSO) {
        const double wi = op->a, c = op->b;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t o = 0; o < N; ++o) {
            const int32_t i = P[below(sel_word(seed, o, t, 0), (uint32_t)nv)];
            const int32_t l = P[below(sel_word(seed, o, t, 1), (uint32_t)nv)];
            const float *xi = X + (int64_t)i * d, *xl = X + (int64_t)l * d;
            const float *vi = Vel + (int64_t)i * d;
            for (int g = 0; g < d; ++g) {
                uint32_t w[4];
                words(seed, (uint32_t)(g / 4), (uint32_t)o, (uint32_t)t, ORA_TAG_OPGENE, w);
                const double r = u24w(w[g % 4]);
                const double diff = (double)xl[g] - (double)xi[g];
                const double pull = c * (r * diff);
                const double vn = wi * (double)vi[g] + pull;
                Xoff[o * (int64_t)d + g] = (float)clip((double)xi[g] + vn, lb, ub);
                Voff[o * (int64_t)d + g] = (float)vn;
            }
        }
    } else if (op->op == ORA_OP_RAND) {
        const double span = ub - lb;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t o = 0; o < N; ++o) {
            for (int g = 0; g < d; ++g) {
                uint32_t w[4];
                words(seed, (uint32_t)(g / 4), (uint32_t)o, (uint32_t)t, ORA_TAG_OPGENE, w);
                Xoff[o * (int64_t)d + g] = (float)(lb + span * u24w(w[g % 4]));
                if (Voff) Voff[o * (int64_t)d + g] = 0.0f;
            }
        }
    } else if (op->op == ORA_OP_CSO) {
        const int64_t Pp = (N + 1) / 2;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t p = 0; p < Pp; ++p) {
            const int32_t a = P[below(sel_word(seed, p, t, 0), (uint32_t)nv)];
            const int32_t b = P[below(sel_word(seed, p, t, 1), (uint32_t)nv)];
            const double fa = fitness(F, m, a), fb = fitness(F, m, b);
            const int a_wins = fa < fb || (fa == fb && a <= b);
            const int32_t win = a_wins ? a : b, los = a_wins ? b : a;
            const float *xw = X + (int64_t)win * d, *xl = X + (int64_t)los * d;
            const float *vw = Vel + (int64_t)win * d, *vl = Vel + (int64_t)los * d;
            for (int g = 0; g < d; ++g) {
                uint32_t w[4];
                words(seed, (uint32_t)g, (uint32_t)p, (uint32_t)t, ORA_TAG_OPGENE, w);
                const double r1 = u24w(w[0]), r2 = u24w(w[1]);
                const double diff = (double)xw[g] - (double)xl[g];
                const double vn = r1 * (double)vl[g] + r2 * diff;
                Xoff[p * (int64_t)d + g] = (float)clip((double)xl[g] + vn, lb, ub);
                Voff[p * (int64_t)d + g] = (float)vn;
                if (p + Pp < N) {
                    Xoff[(p + Pp) * (int64_t)d + g] = xw[g];
                    Voff[(p + Pp) * (int64_t)d + g] = vw[g];
                }
            }
        }
    } else {
        free(P);
        return ORA_EINVAL;
    }
    free(P);
    return ORA_OK;
}

/* One generation with operator op: offspring, evaluation,
 * selection (Alg. 1), new population with each survivor's velocity,
 * adaptation (Alg. 2).  Vel: K x d slot velocities (ops 2, 3; may be NULL
 * for DE). */
int ora_generation_op(const ora_params *Pr, const ora_op *op, int problem, int m, int d,
                      int64_t N, int64_t K, uint64_t seed, int64_t t, float *X, float *Vel,
                      double *F, uint8_t *valid, double *V, const double *V0, double *gamma,
                      float *Xoff_out, float *Voff_out, double *Foff_out, int32_t *surv_out,
                      int *adapted)
{
    const int64_t M = K + N;
    int rc;
    float *Xoff = (float *)malloc(sizeof(float) * (size_t)(N * d));
    float *Voff = (float *)calloc((size_t)(N * d), sizeof(float));
    double *Fm = (double *)malloc(sizeof(double) * (size_t)(M * m));
    uint8_t *mvalid = (uint8_t *)malloc((size_t)M);
    int32_t *assoc = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    double *theta = (double *)malloc(sizeof(double) * (size_t)M);
    double *apd = (double *)malloc(sizeof(double) * (size_t)M);
    int32_t *surv = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    double zstar[64];
    if (adapted) *adapted = 0;
    rc = ora_reproduce_op(Pr, op, seed, t, K, N, d, m, X, Vel, valid, F, Xoff, Voff);
    if (rc != ORA_OK) goto out;
    memcpy(Fm, F, sizeof(double) * (size_t)(K * m));
    if (problem == ORA_POLICY_LQ) {
        const ora_lq *q = Pr->lq;
        rc = q ? ora_policy_evaluate(N, Xoff, d, q->E, q->T, q->A, q->B, q->x0, Fm + K * m)
               : ORA_EINVAL;
    } else {
        rc = ora_evaluate(problem, m, d, N, Xoff, d, Fm + K * m);
    }
    if (rc != ORA_OK) goto out;
    for (int64_t i = 0; i < K; ++i) mvalid[i] = valid[i];
    for (int64_t i = K; i < M; ++i) mvalid[i] = 1;
    ora_select(m, K, N, t, Pr->t_max, Pr->alpha, Fm, mvalid, V, gamma, zstar, assoc, theta, apd,
               surv);
    if (Xoff_out) memcpy(Xoff_out, Xoff, sizeof(float) * (size_t)(N * d));
    if (Voff_out) memcpy(Voff_out, Voff, sizeof(float) * (size_t)(N * d));
    if (Foff_out) memcpy(Foff_out, Fm + K * m, sizeof(double) * (size_t)(N * m));
    if (surv_out) memcpy(surv_out, surv, sizeof(int32_t) * (size_t)K);
    {
        float *Xn = (float *)calloc((size_t)(K * d), sizeof(float));
        float *Vn = (float *)calloc((size_t)(K * d), sizeof(float));
        for (int64_t j = 0; j < K; ++j) {
            const int32_t s = surv[j];
            if (s < 0) {
                valid[j] = 0;
                for (int k = 0; k < m; ++k) F[j * m + k] = NAN;
                continue;
            }
            valid[j] = 1;
            const float *xs = s < K ? X + (int64_t)s * d : Xoff + (int64_t)(s - K) * d;
            memcpy(Xn + j * d, xs, sizeof(float) * (size_t)d);
            if (Vel) {
                const float *vs = s < K ? Vel + (int64_t)s * d : Voff + (int64_t)(s - K) * d;
                memcpy(Vn + j * d, vs, sizeof(float) * (size_t)d);
            }
            for (int k = 0; k < m; ++k) F[j * m + k] = Fm[(int64_t)s * m + k];
        }
        memcpy(X, Xn, sizeof(float) * (size_t)(K * d));
        if (Vel) memcpy(Vel, Vn, sizeof(float) * (size_t)(K * d));
        free(Xn);
        free(Vn);
    }
    if (t % ora_adapt_period(Pr->fr, Pr->t_max) == 0) {
        if (ora_adapt(K, m, V0, F, valid, V)) {
            ora_gamma(K, m, V, gamma);
            if (adapted) *adapted = 1;
        }
    }
out:
    free(Xoff);
    free(Voff);
    free(Fm);
    free(mvalid);
    free(assoc);
    free(theta);
    free(apd);
    free(surv);
    return rc;
}
