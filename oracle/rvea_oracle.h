/*
 * rvea_oracle.h -- declarations of the FP64 CPU oracle (test infrastructure
 * only; see rvea_oracle.c).  This header belongs to the oracle alone: the
 * HIP library neither includes it nor shares any of its definitions.
 */
#ifndef RVEA_ORACLE_H
#define RVEA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ESTATE (-4)

/* Philox stream tags (fourth counter word) */
#define ORA_TAG_INIT 0u
#define ORA_TAG_MATE 1u
#define ORA_TAG_SBX 2u
#define ORA_TAG_SBXPAIR 3u
#define ORA_TAG_MUT 4u
#define ORA_TAG_OPSEL 5u  /* other operators: selection draws */
#define ORA_TAG_OPGENE 6u /* other operators: per-gene uniforms */

/* reproduction operators of the extensibility experiments (operators.c) */
#define ORA_OP_GA 0 /* SBX + polynomial mutation (Appendix B), rvea_oracle.c */
#define ORA_OP_DE 1
#define ORA_OP_PSO 2
#define ORA_OP_CSO 3
#define ORA_OP_RAND 4
typedef struct ora_op {
    int32_t op;
    int32_t pad_;
    double a, b; /* DE: F, CR; PSO: w, c; CSO, random: unused */
} ora_op;

/* Linear system of the policy-rollout problem (problem id ORA_POLICY_LQ):
 * A 32x32 and B 32x8 row-major, x0 E x 32 rollout start states, T steps,
 * initial genes N(0, sigma) clipped to the bounds. */
#define ORA_POLICY_LQ 100
#define ORA_POLICY_D 6728
typedef struct ora_lq {
    const float *A, *B, *x0;
    int32_t E, T;
    double sigma;
} ora_lq;

typedef struct ora_params {
    double alpha;  /* APD penalty rate (Eq. 4) */
    double fr;     /* reference-vector adaptation frequency */
    int32_t t_max; /* maximal number of generations */
    int32_t pad_;
    double eta_c; /* SBX distribution index */
    double eta_m; /* polynomial-mutation distribution index (xi) */
    double p_c;   /* crossover probability */
    double p_m;   /* mutation probability; per-site rate is p_m / d */
    double lb, ub;
    const ora_lq *lq; /* policy-rollout problem only, else NULL */
} ora_params;

double ora_bf16(double x);
int ora_policy_evaluate(int64_t n, const float *X, int64_t ldx, int E, int T, const float *A,
                        const float *B, const float *x0, double *F);
void ora_init_gauss_rows(uint64_t seed, const int64_t *rows, int64_t n, int d, double sigma,
                         double lb, double ub, float *X, double *pre);
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int64_t ora_binomial(int64_t n, int64_t k);
int64_t ora_lattice_count(int H, int m);
int64_t ora_lattice(int H, int m, double *W, int64_t cap);
void ora_normalize_rows(const double *W, int64_t K, int m, double *V);
void ora_gamma(int64_t K, int m, const double *V, double *gamma);
void ora_gamma_rows(int64_t K, int m, const double *V, const int64_t *rows, int64_t n,
                    double *out);
int ora_evaluate_one(int problem, int m, int d, const float *x, double *f);
int ora_evaluate(int problem, int m, int d, int64_t n, const float *X, int64_t ldx, double *F);
int64_t ora_front(int problem, int m, int Hs, double *Fs, int64_t cap);
double ora_igd(const double *F, int64_t n, const double *Fs, int64_t ns, int m);
void ora_init(uint64_t seed, int64_t N, int d, double lb, double ub, float *X, int64_t ldx);
void ora_init_rows(uint64_t seed, const int64_t *rows, int64_t n, int d, double lb, double ub,
                   float *X);
int64_t ora_mate(uint64_t seed, int64_t t, int64_t K, int64_t N, const uint8_t *valid,
                 int32_t *parents);
double ora_sbx_beta(double mc, double eta);
double ora_pm_delta(double x, double lb, double ub, double mm, double xi);
int ora_mutation_sites(uint64_t seed, int64_t t, int64_t o, int d, double p_m, int32_t *sites,
                       double *mags, int cap);
void ora_mutate_child(uint64_t seed, int64_t t, int64_t o, int d, double p_m, double lb,
                      double ub, double eta_m, double *c);
int ora_reproduce(const ora_params *P, uint64_t seed, int64_t t, int64_t K, int64_t N, int d,
                  const float *X, int64_t ldx, const int32_t *parents, float *Xoff,
                  int64_t ldo, double *pre);
int ora_reproduce_pairs(const ora_params *P, uint64_t seed, int64_t t, int64_t N, int d,
                        const float *X, int64_t ldx, const int32_t *parents, const int64_t *pairs,
                        int64_t n, float *out1, float *out2);
void ora_assoc_rows(int m, int64_t K, int64_t t, int t_max, double alpha, const double *Frows,
                    int64_t n, const double *zstar, const double *V, const double *gamma,
                    int32_t *assoc, double *theta, double *apd);
int ora_select(int m, int64_t K, int64_t N, int64_t t, int t_max, double alpha, const double *Fm,
               const uint8_t *mvalid, const double *V, const double *gamma, double *zstar,
               int32_t *assoc, double *theta, double *apd, int32_t *surv);
int ora_adapt(int64_t K, int m, const double *V0, const double *F, const uint8_t *valid,
              double *V);
int ora_adapt_period(double fr, int t_max);
int ora_generation(const ora_params *P, int problem, int m, int d, int64_t N, int64_t K,
                   uint64_t seed, int64_t t, float *X, double *F, uint8_t *valid, double *V,
                   const double *V0, double *gamma, float *Xoff_out, double *Foff_out,
                   int32_t *parents_out, int32_t *surv_out, int *adapted);
int ora_run(const ora_params *P, int problem, int m, int d, int64_t N, int64_t K, uint64_t seed,
            int gens, float *X, double *F, uint8_t *valid, double *V, double *V0, double *gamma);
/* operators.c: DE, PSO, CSO and random reproduction */
int ora_de_draws(uint64_t seed, int64_t t, int64_t o, int d, const int32_t *P, int64_t nv,
                 int32_t out[5]);
int ora_reproduce_op(const ora_params *Pr, const ora_op *op, uint64_t seed, int64_t t,
                     int64_t K, int64_t N, int d, int m, const float *X, const float *Vel,
                     const uint8_t *valid, const double *F, float *Xoff, float *Voff);
int ora_generation_op(const ora_params *Pr, const ora_op *op, int problem, int m, int d,
                      int64_t N, int64_t K, uint64_t seed, int64_t t, float *X, float *Vel,
                      double *F, uint8_t *valid, double *V, const double *V0, double *gamma,
                      float *Xoff_out, float *Voff_out, double *Foff_out, int32_t *surv_out,
                      int *adapted);
/* indicators.c: App. C.2 hypervolume (m = 2, 3; reference point ones on
 * f' = (f - lo) / (hi - lo)) and the expected utility over a weight set */
double ora_hypervolume(int m, int64_t n, const double *F, const uint8_t *valid, const double *lo,
                       const double *hi);
double ora_expected_utility(int m, int64_t n, const double *F, const uint8_t *valid,
                            const double *lo, const double *hi, int64_t nw, const double *W);
int ora_num_threads(void);
void ora_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
