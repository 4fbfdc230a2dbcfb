/*
 * rvea.h -- C ABI of the MI355X TensorRVEA generation library (librvea.so).
 *
 * The library runs one generation of the reference-vector guided
 * evolutionary algorithm as tensorized by Liang, Jiang, Sun and Cheng,
 * "GPU-accelerated Evolutionary Multiobjective Optimization Using
 * Tensorized RVEA" (GECCO'24), on one AMD Instinct MI355X (gfx950):
 *   rvea_step   -- random mating, SBX crossover and polynomial mutation
 *                  (Appendix B), evaluation of the offspring;
 *   rvea_select -- translation by the ideal point, association of the
 *                  merged population to the reference vectors, angle-
 *                  penalized distance, per-vector argmin (Alg. 1,
 *                  Eqs. 2-5), new population;
 *   rvea_adapt  -- reference-vector update of Alg. 2.
 * The problem statement it serves is Eq. 1 (minimise f(x) in R^m over
 * x in R^d).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an rvea_status; nothing throws across the ABI.
 *   - Device memory is owned by the caller.  rvea_create receives one
 *     device workspace of at least rvea_footprint() bytes and never
 *     allocates device memory itself; the workspace must stay alive and
 *     untouched by the caller until rvea_destroy.  Host pointers passed to
 *     the state accessors are read or written before the call returns.
 *   - Work is enqueued asynchronously on the HIP stream given to
 *     rvea_create (NULL = the default stream); rvea_synchronize or any
 *     accessor that returns data waits for it.
 *   - A run handle is not thread safe; distinct handles are independent.
 *   - Call order per generation: rvea_step, rvea_select, rvea_adapt.
 *     A call out of this order returns RVEA_ESTATE and enqueues nothing.
 *   - On RVEA_EDEVICE the HIP error text is available from
 *     rvea_last_error(run); for a failed rvea_create, from
 *     rvea_last_error(NULL) on the same thread.
 */
#ifndef RVEA_H
#define RVEA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rvea_status {
    RVEA_OK = 0,
    RVEA_EINVAL = -1,      /* an argument is out of range */
    RVEA_ENOMEM = -2,      /* workspace smaller than rvea_footprint() */
    RVEA_EDEVICE = -3,     /* a HIP call failed; see rvea_last_error */
    RVEA_ESTATE = -4,      /* call out of order, or no valid individual left */
    RVEA_EUNSUPPORTED = -5 /* a configuration this build does not run */
} rvea_status;

/* Test problems.  The paper benchmarks on DTLZ, which it does not define;
 * these are the library's own problems of the same shape on [0,1]^d: the
 * first m-1 variables place a point w on the simplex (uniform spacings of
 * the sorted variables), the remaining k = d-m+1 set a distance term g >= 0
 * that is 0 when all of them equal 1/2.
 *   LINEAR_MULTIMODAL : f = (1+g) w,          g = mean(10 t^2 + 2 sin^2(4 pi t))
 *   SPHERE_UNIMODAL   : f = (1+g) w / |w|,    g = 4 mean(t^2)
 *   SPHERE_MULTIMODAL : f = (1+g) w / |w|,    g as LINEAR_MULTIMODAL
 * with t = x - 1/2 over the distance variables. */
typedef enum rvea_problem {
    RVEA_LINEAR_MULTIMODAL = 1,
    RVEA_SPHERE_UNIMODAL = 2,
    RVEA_SPHERE_MULTIMODAL = 3,
    RVEA_POLICY_LQ = 100 /* policy rollouts, m = 2, d = 6728; see rvea_create_policy */
} rvea_problem;

/* Reproduction operators (Sec. 4, Extensibility: the genetic operators
 * swapped for those of other population methods, selection and adaptation
 * unchanged).  The paper names the operators without defining them; each
 * is the update of its original method:
 *   RVEA_OP_GA   SBX + polynomial mutation on random pairs (Appendix B);
 *   RVEA_OP_DE   DE/rand/1/bin (Storn and Price): per child a target and
 *                three distinct donors from the population, mutant
 *                x_r1 + F (x_r2 - x_r3) clipped to the box, binomial
 *                crossover with rate CR and one forced gene;
 *                op_a = F in [0, 2], op_b = CR in [0, 1];
 *   RVEA_OP_PSO  particle swarm with inertia weight (Kennedy and Eberhart;
 *                Shi and Eberhart): per child a particle i and a leader l
 *                drawn from the population, v' = w v_i + c r (x_l - x_i)
 *                with r uniform per gene, x' = clip(x_i + v'); every
 *                individual carries its velocity (zero when created);
 *                op_a = w in [0, 1], op_b = c in [0, 4];
 *   RVEA_OP_CSO  competitive swarm (Cheng and Jin): per pair of drawn
 *                members the one with the smaller objective sum wins; the
 *                loser moves, v' = r1 v_l + r2 (x_w - x_l), and the winner
 *                is carried over unchanged; op_a = op_b = 0;
 *   RVEA_OP_RAND every child drawn uniformly in the box (the study's
 *                baseline); op_a = op_b = 0.
 * Random draws come from the run's Philox4x32-10 streams; the exact
 * counters are stated in the library's oracle.  Runs of every operator can
 * join a batch (runs of one operator and segment width share a launch). */
typedef enum rvea_operator {
    RVEA_OP_GA = 0,
    RVEA_OP_DE = 1,
    RVEA_OP_PSO = 2,
    RVEA_OP_CSO = 3,
    RVEA_OP_RAND = 4
} rvea_operator;

/* Algorithm parameters (defaults from rvea_default_params in brackets). */
typedef struct rvea_params {
    double alpha;     /* APD penalty rate of Eq. 4 [2] */
    double fr;        /* adaptation every ceil(fr * t_max) generations [0.1] */
    int32_t t_max;    /* maximal number of generations, Eq. 4 [100] */
    int32_t op;       /* reproduction operator, rvea_operator [RVEA_OP_GA] */
    double eta_c;     /* SBX distribution index eta, Appendix B [20] */
    double eta_m;     /* polynomial-mutation distribution index xi [20] */
    double p_c;       /* crossover probability [1] */
    double p_m;       /* mutation probability; per-gene rate p_m/d, 0..4 [1] */
    double lb, ub;    /* box of every decision variable, lb < ub [0, 1] */
    double op_a, op_b; /* the operator's parameters (see rvea_operator) [0, 0] */
} rvea_params;

typedef struct rvea_run_s *rvea_run;

/* Fills *out with the defaults above. */
rvea_status rvea_default_params(rvea_params *out);

/* Selects operator op in *params and sets op_a, op_b to its defaults
 * (DE: F = 0.5, CR = 0.9; PSO: w = 0.5, c = 1.5; others 0); the other
 * fields are left as they are.  RVEA_EINVAL for an unknown operator. */
rvea_status rvea_operator_params(int op, rvea_params *params);

/* Reference-vector lattice (Alg. 2 input V_0): K = C(H+m-1, m-1) unit
 * vectors of the Das-Dennis simplex lattice with H divisions.  Writes the
 * H with that count for (m, K) to *H, or returns RVEA_EINVAL. */
rvea_status rvea_lattice_divisions(int m, int64_t K, int *H);

/* Device bytes a run of this shape needs (workspace size for rvea_create).
 * m in [2,8], d >= m, 1 <= N <= K, K a lattice count for m
 * (RVEA_POLICY_LQ: m = 2, d = 6728). */
rvea_status rvea_footprint(int problem, int m, int d, int64_t N, int64_t K,
                           const rvea_params *params, size_t *bytes);

/* Creates a run on the current HIP device and enqueues its initialization
 * (Alg. 2's initialization: N individuals uniform in [lb,ub]^d in slots 0..N-1, the
 * rest of the K slots empty; V = V_0; gamma of Eq. 5).
 *   workspace        device pointer, 256-byte aligned, >= footprint bytes
 *   hip_stream       hipStream_t (may be NULL)
 *   seed             key of the run's Philox4x32-10 streams
 *   params           NULL for the defaults; copied */
rvea_status rvea_create(int problem, int m, int d, int64_t N, int64_t K, uint64_t seed,
                        const rvea_params *params, void *workspace, size_t workspace_bytes,
                        void *hip_stream, rvea_run *out);

/* Policy-rollout problem (the neuroevolution setting of Sec. 4.3: objectives
 * of a policy network obtained by simulation; here a synthetic linear system
 * stands in for the physics engine).  An individual is the d = 6728 weights
 * of a 32 -> 64 -> 64 -> 8 tanh network, row-major [out][in]:
 *   W1 64x32 at 0, b1 64 at 2048, W2 64x64 at 2112, W3 8x64 at 6208, b3 8 at 6720
 * (the second hidden layer has no bias).  From each of E start states x0[e]
 * it runs T steps of  u = tanh(W3 tanh(W2 tanh(W1 x + b1)) + b3),
 * x <- A x + B u;  f1 = sum |x_t|^2 over t = 1..T and f2 = sum |u_t|^2 over
 * t = 0..T-1, each averaged over the E rollouts, both minimised.  Weight
 * matrices and layer inputs are rounded to bfloat16 and multiplied on the
 * matrix cores with binary32 accumulation; biases and the state are
 * binary32, and A x + B u is accumulated in binary32 from products of the
 * operands' bfloat16 high and low parts (hi*hi + lo*hi + hi*lo, about 2^-17
 * relative).  Initial genes are N(0, init_sigma^2) clipped to [lb, ub].
 * All pointers are host memory, read during rvea_create_policy. */
typedef struct rvea_lq_system {
    const float *A;    /* 32 x 32, row-major */
    const float *B;    /* 32 x 8, row-major */
    const float *x0;   /* E x 32 start states */
    int32_t E;         /* rollouts per individual; must be 16 */
    int32_t T;         /* steps per rollout, >= 1 */
    double init_sigma; /* standard deviation of the initial genes, > 0 */
} rvea_lq_system;

/* rvea_create for RVEA_POLICY_LQ (m = 2, d = 6728; the footprint is
 * rvea_footprint(RVEA_POLICY_LQ, 2, 6728, N, K, ...)).  rvea_create rejects
 * that problem id, and a policy run cannot join a batch (RVEA_EUNSUPPORTED).
 * The library keeps its own copy of the system. */
rvea_status rvea_create_policy(int64_t N, int64_t K, uint64_t seed, const rvea_params *params,
                               const rvea_lq_system *system, void *workspace,
                               size_t workspace_bytes, void *hip_stream, rvea_run *out);

/* Alg. 2's offspring step and Appendix B for generation t = completed + 1: draws the
 * N offspring by random mating, SBX and polynomial mutation from the
 * current population, and evaluates them (Eq. 1). */
rvea_status rvea_step(rvea_run run);

/* Alg. 2's selection step / Alg. 1: selects at most one survivor per reference
 * vector from the K parent slots and the N offspring, writes the new
 * population into the slots and counts the generation as completed. */
rvea_status rvea_select(rvea_run run);

/* Alg. 2's update of V: when the completed generation count is a multiple of
 * ceil(fr * t_max), updates V from V_0 and the survivors' objective ranges
 * and recomputes gamma; otherwise does nothing. */
rvea_status rvea_adapt(rvea_run run);

/* n x (rvea_step, rvea_select, rvea_adapt).  Unless disabled with
 * rvea_set_graphs or while kernel timing is on, up to 16 consecutive
 * generations (a multiple of the adaptation period when that is at most 16)
 * go out as one launch of a HIP graph, captured on first use for that length
 * and those adapting positions; a run keeps at most 8 such graphs.  Results
 * are identical either way. */
rvea_status rvea_run_generations(rvea_run run, int n);

/* Captures, without running anything, the graphs that
 * rvea_run_generations(run, n) would launch from the current generation, so
 * that the capture cost is not paid inside a latency- or time-critical call.
 * Nothing to do when graphs are disabled.  RVEA_ESTATE between rvea_step and
 * rvea_adapt or while the run belongs to a batch. */
rvea_status rvea_prepare_generations(rvea_run run, int n);

/* 1 (default) = rvea_run_generations replays captured HIP graphs, 0 = it
 * launches every kernel individually. */
rvea_status rvea_set_graphs(rvea_run run, int enable);

/* Association (Alg. 1, Eq. 2) through an index of the reference vectors
 * (1, the default for m = 2 and m = 3) or by a scan of all K vectors per row
 * (0).  Both give the same association, angle and APD for every row: the
 * index hands each row candidates that include its vector of largest cosine
 * and every vector tied with it (m = 3: a list per grid cell; m = 2: the
 * cells of a line walked outward until no further vector can tie), and the
 * cosines are computed the same way.  The index is rebuilt whenever V
 * changes.  RVEA_EUNSUPPORTED to enable it for m > 3; only between
 * generations and outside a batch (RVEA_ESTATE). */
rvea_status rvea_set_index(rvea_run run, int enable);

/* Copies the run state to host memory (waits for the stream).  Any pointer
 * may be NULL.  Layouts, row-major: X K x d float, F K x m float,
 * valid K bytes (1 = slot holds an individual), V and V0 K x m double,
 * gamma K double; *t = completed generations.  Empty slots hold NaN in F. */
rvea_status rvea_get_state(rvea_run run, float *X, float *F, uint8_t *valid, double *V,
                           double *V0, double *gamma, int64_t *t);

/* Replaces the run state from host memory (same layouts; V0 stays the
 * lattice).  X, F and valid are required; V and gamma may be NULL to keep
 * the current ones.  Only allowed between generations. */
rvea_status rvea_set_state(rvea_run run, const float *X, const float *F,
                           const uint8_t *valid, const double *V, const double *gamma,
                           int64_t t);

/* The offspring X (N x d float), their objectives F (N x m float) and the
 * mating pairs (ceil(N/2) x 2 slot indices; for RVEA_OP_CSO the pair's
 * winner and loser, for the other non-GA operators -1) of the generation in progress
 * (after rvea_step) or, between generations, of the last completed one
 * (also after rvea_run_generations or a batch step; the next rvea_step
 * reuses their rows).  RVEA_ESTATE when no generation has completed since
 * creation, rvea_set_state or rvea_autotune.  Any pointer may be NULL.
 * Waits for the stream. */
rvea_status rvea_get_offspring(rvea_run run, float *X, float *F, int32_t *parents);

/* After rvea_select: the ideal point (m float), the association of each
 * merged row (K+N int32, -1 for rows that did not take part), its APD
 * (K+N double, +inf when not taking part) and the survivor of each vector
 * (K int32 merged-row index, -1 if none).  Waits for the stream. */
rvea_status rvea_get_selection(rvea_run run, float *zstar, int32_t *assoc, double *apd,
                               int32_t *surv);

/* Velocities of the swarm operators (RVEA_OP_PSO, RVEA_OP_CSO): those of
 * the population's slots (offspring = 0; K x d float, 0 for empty slots;
 * valid between generations) or of the offspring (offspring = 1; N x d
 * float; valid whenever rvea_get_offspring is).  A velocity belongs to its
 * individual: a survivor keeps the one it was created with.  RVEA_EINVAL
 * for runs of other operators.  Waits for the stream. */
rvea_status rvea_get_velocities(rvea_run run, int offspring, float *Vel);

/* Sets the slots' velocities (K x d float, rows of empty slots ignored)
 * of a PSO or CSO run; rvea_set_state sets them to zero.  Only allowed
 * between generations. */
rvea_status rvea_set_velocities(rvea_run run, const float *Vel);

/* Selected rows only: idx[0..n) are slot indices (offspring = 0) or
 * offspring indices (offspring = 1); writes their genes (n x d float) and
 * objectives (n x m float).  Either output may be NULL.  Valid between
 * generations (slots) or whenever rvea_get_offspring is (offspring).
 * Waits for the stream. */
rvea_status rvea_get_rows(rvea_run run, int offspring, const int64_t *idx, int64_t n, float *X,
                          float *F);

/* Counters since creation: rows dropped as non-finite, individuals whose
 * association needed the full double-precision scan. */
typedef struct rvea_counters {
    int64_t nonfinite_rows;
    int64_t full_rescans;
    int64_t generations;
} rvea_counters;
rvea_status rvea_get_counters(rvea_run run, rvea_counters *out);

/* Per-kernel timing with HIP events recorded on the run's stream around the
 * selected kernels.  Kernel ids: 0 reproduce+evaluate, 1 association,
 * 2 re-rank+APD, 3 adaptation (vectors + gamma), 4 policy rollouts
 * (RVEA_POLICY_LQ; id 0 then covers reproduction only); kernel_mask bit k enables
 * id k, 0 disables timing.  rvea_kernel_time returns the summed
 * milliseconds and launch count since timing was last set (waits for the
 * stream). */
rvea_status rvea_set_timing(rvea_run run, int kernel_mask);
rvea_status rvea_kernel_time(rvea_run run, int kernel, double *ms, int64_t *launches);

/* Launch time of the three hot kernels without per-launch event overhead:
 * between rvea_step and rvea_select, each of reproduce+evaluate (id 0; the
 * policy rollouts excluded), association and re-rank is launched reps times
 * back to back on the current state between two HIP events; ms[0..2]
 * receives milliseconds per launch.  Every launch rewrites the same outputs
 * from the same inputs, so the state and the counters are as before; the
 * call waits for the stream.  RVEA_ESTATE outside that phase, in a batch or
 * with kernel timing on. */
rvea_status rvea_time_kernels(rvea_run run, int reps, double *ms);

/* Association tile autotuner.  The association pass (Alg. 1's angle
 * computation, Eq. 2) can run with 1, 2 or 4 rows per lane and with vector
 * chunks of 32..1024 vectors (at least the default length; fewer chunks mean
 * fewer per-chunk partials to write and re-read), and its binary64 re-rank
 * with 4, 8 or 16 rows per wavefront.  Association shapes are timed together
 * with the re-rank that reads their partials.  rvea_autotune draws the
 * next generation's offspring and ideal point without committing anything,
 * times every candidate on them (five launches back to back between two HIP
 * events, per-launch time, best of two such rounds) and keeps the fastest
 * for the rest of the run.  The adaptation's gamma pass
 * (its rows are the K vectors) gets its own rows per lane and chunk length,
 * timed the same way on the current vectors.  Results do not depend on the choice: the association is
 * finished in binary64 over candidate tiles.  Needs the run between
 * generations, outside a batch and with timing off (RVEA_ESTATE); waits for
 * the stream; afterwards rvea_get_selection reports RVEA_ESTATE until the
 * next rvea_select.  out may be NULL. */
typedef struct rvea_tuning {
    int32_t rows_per_lane;      /* association: chosen rows per lane */
    int32_t chunk_vectors;      /* association: chosen chunk length */
    int32_t rerank_rows;        /* binary64 re-rank: chosen rows per wavefront (4, 8, 16) */
    int32_t candidates;         /* configurations timed */
    double assoc_us;            /* association + re-rank per launch, chosen shape */
    double default_us;          /* association + re-rank, default shape */
    double rerank_us;           /* best time of the chosen re-rank configuration */
    double rerank_default_us;   /* best time of the default one */
    int32_t gamma_rows_per_lane;  /* gamma pass (rows = vectors): chosen rows per lane */
    int32_t gamma_chunk_vectors;  /* gamma pass: chosen chunk length */
    double gamma_us;              /* gamma pass (both passes), chosen shape */
    double gamma_default_us;      /* gamma pass, default shape */
} rvea_tuning;
rvea_status rvea_autotune(rvea_run run, rvea_tuning *out);

rvea_status rvea_synchronize(rvea_run run);
rvea_status rvea_destroy(rvea_run run);

/* ---------------------------------------------------------------- batches
 * A batch advances many independent runs (any problem, m, d, N, K) one
 * generation per rvea_batch_step: each phase of the generation is one launch
 * covering every admitted run (runs grouped by segment width or objective
 * count; runs with the index of rvea_set_index associate through it and keep
 * it rebuilt in phases of their own), and the launch sequence is captured into one HIP graph that is
 * replayed until the membership changes.  Each run keeps its own workspace,
 * state and Philox stream, so a run's results do not depend on what else is
 * in the batch.  Adaptation is decided on the device per run.
 *   workspace   device memory of rvea_batch_footprint(max_runs) bytes,
 *               256-byte aligned, owned by the caller (run tables and spans)
 *   hip_stream  the stream every batched generation is enqueued on
 * While admitted, a run rejects rvea_step/select/adapt/run_generations and
 * rvea_set_state (RVEA_ESTATE); its accessors wait for the batch stream.
 * Admission needs the run between generations and timing off; it fails with
 * RVEA_ENOMEM when max_runs runs are admitted. */
typedef struct rvea_batch_s *rvea_batch;
rvea_status rvea_batch_footprint(int max_runs, size_t *bytes);
rvea_status rvea_batch_create(int max_runs, void *workspace, size_t workspace_bytes,
                              void *hip_stream, rvea_batch *out);
rvea_status rvea_batch_admit(rvea_batch batch, rvea_run run);
rvea_status rvea_batch_retire(rvea_batch batch, rvea_run run);
rvea_status rvea_batch_step(rvea_batch batch);
/* 1 (default) = replay captured graphs once the membership is stable. */
rvea_status rvea_batch_set_graphs(rvea_batch batch, int enable);
rvea_status rvea_batch_size(rvea_batch batch, int *n);
rvea_status rvea_batch_synchronize(rvea_batch batch);
rvea_status rvea_batch_destroy(rvea_batch batch);
const char *rvea_batch_last_error(rvea_batch batch);

/* ------------------------------------------------------------- indicators
 * Quality indicators of a set of objective rows, computed on the device.
 *   F         device, n x m float, row-major
 *   valid     device, n bytes (1 = the row counts) or NULL (every row counts);
 *             a row with a non-finite objective never counts
 *   lo, hi    host, m doubles each, finite, hi > lo: every objective is
 *             normalised to f' = (f - lo) / (hi - lo) in binary64
 *   out       device, one double, written when the enqueued work completes
 *   workspace device, 256-byte aligned, at least rvea_indicator_footprint
 *             bytes, owned by the caller, contents arbitrary on entry and
 *             clobbered; it must not be reused until the work completes
 * The work is enqueued on hip_stream (NULL = default stream); nothing waits.
 * Argument errors return before anything is enqueued; launch errors return
 * RVEA_EDEVICE with the text in rvea_last_error(NULL) on the same thread. */

/* Workspace bytes for either indicator: n rows, nw weight rows
 * (m in [2, 8], 0 <= n <= 2^24, 0 <= nw <= 2^24). */
rvea_status rvea_indicator_footprint(int m, int64_t n, int64_t nw, size_t *bytes);

/* Hypervolume of App. C.2: the volume of the union of the boxes [f', 1]
 * (reference point: the vector of ones) over the counted rows whose f' lies
 * strictly below 1 in every objective; m = 2 or 3, 0 <= n <= 2^18 (the work
 * grows as n^2).  A sum of non-negative binary64 terms: relative error below
 * about 4 n 2^-53.  n = 0 gives 0. */
rvea_status rvea_hypervolume(int m, int64_t n, const float *F, const uint8_t *valid,
                             const double *lo, const double *hi, double *out, void *workspace,
                             size_t workspace_bytes, void *hip_stream);

/* rvea_hypervolume for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument, and no device memory is allocated or
 * freed.  Its working memory is a static 8 MiB array of the library on each
 * GPU it runs on (kept until the process ends), so n may be at most 131,072
 * (RVEA_ENOMEM beyond, with the reason in rvea_last_error(NULL)).  Every call
 * on one GPU uses that GPU's array: calls that overlap on one GPU (different
 * streams, different threads) race and must be serialised by the caller;
 * consecutive calls on one stream are safe.  Same arguments, result and
 * errors as rvea_hypervolume otherwise. */
rvea_status rvea_hypervolume_noalloc(int m, int64_t n, const float *F, const uint8_t *valid,
                                     const double *lo, const double *hi, double *out,
                                     void *hip_stream);

/* Expected utility over a weight set (the neuroevolution appendix's EU, for
 * minimised objectives): the mean over the nw weight rows w of W (device,
 * nw x m double, each equally likely) of the best utility -(w . f') over the
 * counted rows; -inf when no row counts.  m in [2, 8], nw >= 1. */
rvea_status rvea_expected_utility(int m, int64_t n, const float *F, const uint8_t *valid,
                                  const double *lo, const double *hi, int64_t nw,
                                  const double *W, double *out, void *workspace,
                                  size_t workspace_bytes, void *hip_stream);

const char *rvea_status_str(rvea_status s);
const char *rvea_last_error(rvea_run run);

#ifdef __cplusplus
}
#endif
#endif
