// rvea_dev.h -- device-side definitions shared by the library's kernels.
//
// Contents: the run view handed to every kernel, Philox4x32-10 (Salmon,
// Moraes, Dror, Shaw, SC'11) in its counter-based form, the uniform
// variates built from its words, and order-preserving float encodings used
// by the atomic min/max reductions.  gfx950 only; compiled with
// -ffp-contract=off, so every fused multiply-add below is written as fma().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rvea {

// Philox stream tags (fourth counter word).  The other three counter words
// are (sub-index, individual or pair, generation); the key is the run seed.
enum : uint32_t {
    TAG_INIT = 0, TAG_MATE = 1, TAG_SBX = 2, TAG_SBXPAIR = 3, TAG_MUT = 4,
    TAG_OPSEL = 5,  // member draws of the other reproduction operators
    TAG_OPGENE = 6  // their per-gene uniforms
};

// reproduction operators (ids as in rvea.h)
enum : int { OP_GA = 0, OP_DE = 1, OP_PSO = 2, OP_CSO = 3, OP_RAND = 4 };

constexpr int kMaxM = 8;         // objectives supported
constexpr int kTile = 32;        // reference vectors per association tile
constexpr int kMaxSites = 32;    // mutation sites held per child
constexpr int kBlock = 256;      // threads per block for the streaming kernels
constexpr int kPolicy = 100;     // problem id of the policy-rollout problem
constexpr int kPolicyD = 6728;   // its gene count (32 -> 64 -> 64 -> 8 policy)
constexpr int kPolicyE = 16;     // its rollouts per individual

// Everything a kernel needs to find the run's buffers.  Passed by value.
struct RunView {
    int m, d, ld, problem;
    int64_t N, K, M;  // parent slots K, offspring N, merged rows M = K + N
    uint32_t key0, key1;
    int t_max, period;
    double alpha, eta_c, eta_m, p_c, p_m, lb, ub;
    int KC, CS;  // association: number of vector chunks and chunk length
    int rr;      // association: rows per lane (1, 2 or 4)
    int rk;      // re-rank: rows per wave (4, 8 or 16)
    int gKC, gCS, grr;  // the same three for the gamma pass (rows = vectors)

    float *X;           // (K+N) x ld physical gene rows
    // The population after p generations lives in buffer p & 1 of each
    // pair below; generation p+1 reads it and writes population p+1 into
    // the other buffer, so the new population needs no copy-back.
    int32_t *slot_rows; // 2 x K: physical row of each slot
    int32_t *off_row;   // N: physical row of each offspring this generation
    uint8_t *valids;    // 2 x K
    float *Fms;         // 2 x M x m merged objectives (slots, then offspring)
    uint8_t *mvalid;    // M: row takes part in the selection
    int32_t *parents;   // ceil(N/2) x 2 slot indices
    int osplit;         // segments per parent pair in the offspring kernel (1: one)
    double *gpart;      // ceil(N/2) x osplit x 2 partial distance sums (osplit > 1)
    int op;             // reproduction operator (OP_*)
    double op_a, op_b;  // its parameters
    float *Vel;         // (K+N) x ld velocities by physical row (PSO, CSO), else null
    // index of the reference vectors (k_grid.hip): a grid of G x G cells
    // (three objectives) or a line of G cells (two); "cells" below is G*G or G
    int gG;             // cells per side (0: association by full scan)
    int64_t gcap;       // list records: a slot of equal size per cell (grid only)
    double *gr;         // m: the scaling r the cells' coordinates divide by
    int32_t *gcell;     // K: cell of each vector (-1: outside the line)
    int32_t *gcnt;      // cells: vectors per cell, then fill cursors (build)
    int32_t *gstart;    // cells: first position of each cell's vectors
    int32_t *gnum;      // cells: vectors of each cell
    int32_t *gvec;      // K: vector ids by cell
    double *gvh;        // K x 4: by cell, their unit directions (grid) or
                        // (v, |v|) (line)
    int32_t *lcnt;      // cells: candidate-list length (-1: full scan; grid only)
    int32_t *lstart;    // cells: first record of each list (-1: full scan; grid only)
    unsigned long long *gtot;  // 4: the allocator of the cells' vector ranges (build),
                               // 1 when the build left some vector's gamma,
                               // 1 when some vector is outside the
                               // line (every row then scans all vectors), spare
    double *lrec;       // gcap x 4: (v, |v|) of the list entries
    int32_t *lidx;      // gcap: vector id of each record
    int32_t *vs;        // K x 2: valid slots, ascending, each with its physical row
    int32_t *nvalid;    // 1
    int32_t *stamp;     // K+N: the generation that will read the row (rows of
                        // the current population carry t_done + 1)
    int32_t *bcount;    // per-256-slot-block valid counts of the current population
    int32_t *freecnt;   // 1: free rows handed out (prepare)
    double *V0, *V;     // K x m
    float *V32;         // K x 4 or K x 8 (padded with zeros)
    double *vn;         // K norms of V
    double *gamma;      // K
    uint32_t *zbits;    // 2 x m ordered-encoded ideal point, by generation parity
    uint32_t *rbits;    // 2m ordered-encoded survivor min / max
    float *pmax;        // KC x M chunk maxima
    uint32_t *pmask;    // KC x M candidate-tile masks
    int32_t *assoc;     // M
    double *apd;        // M
    unsigned long long *key;  // K: min over associated rows of (APD, row), packed
    int kb;             // row-index bits of a key: M < 2^kb
    int32_t *surv;      // K: survivor's merged row of the last selection, or -1
    int64_t *t_done;    // completed generations
    uint32_t *ndone;    // 1: k_newpop workgroups finished (the last one counts the generation)
    unsigned long long *counters;  // 0 non-finite rows, 1 full rescans, 2 site overflow
    int32_t *vchanged;  // 1: adaptation changed V
    double *pen;        // 1: m (t/t_max)^alpha of the current generation
    // policy-rollout problem only: A (32x32), B (32x8), x0 (E x 32), binary32
    const float *lq;
    int lq_E, lq_T;
    double lq_sigma;    // initial genes N(0, sigma^2)
};

// buffers of population p (the state after p generations)
__device__ __forceinline__ int32_t *slot_row_of(const RunView &R, int64_t p)
{
    return R.slot_rows + (p & 1) * R.K;
}
__device__ __forceinline__ uint8_t *valid_of(const RunView &R, int64_t p)
{
    return R.valids + (p & 1) * R.K;
}
__device__ __forceinline__ float *fm_of(const RunView &R, int64_t p)
{
    return R.Fms + (p & 1) * R.M * R.m;
}

// cells of an index of side G: a G x G grid for three objectives, a line of
// G cells for two
__host__ __device__ inline int64_t index_cells(int m, int G)
{
    return m == 3 ? (int64_t)G * G : (int64_t)G;
}

// One run's share of a batched launch: blocks [start, next start) belong to
// run `run` of the device run table; nbx is the row-block count of a 2-D
// (row block x vector chunk) phase.
struct Span {
    int64_t start;
    int32_t run;
    int32_t nbx;
};

// index of the span holding block b (spans sorted by start, first start 0)
__device__ __forceinline__ int find_span(const Span *sp, int n, int64_t b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sp[mid].start <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Batched phases that most generations skip (the index build, the gamma
// passes) give each workgroup U consecutive blocks of the span table, so a
// generation in which every run's phase is off (open(R) false) launches U
// times fewer workgroups (their launch, not their work, is what such a
// generation pays for).  The U steps are unrolled (a loop around the body
// keeps far more registers live; so can U inlined copies of a large body,
// which a caller then keeps out of line).  body(R, local block, nbx); every value
// that steers the steps is uniform over the workgroup, and a barrier
// separates one block's use of shared memory from the next.
template <int U, typename Open, typename Body>
__device__ __forceinline__ void span_blocks(const RunView *runs, const Span *sp, int n,
                                            int64_t total, Open open, Body body)
{
    const int64_t b0 = (int64_t)blockIdx.x * U;
    int s = find_span(sp, n, b0), cur = -1;
    bool on = false;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t b = b0 + u;
        if (b >= total) break;
        while (s + 1 < n && sp[s + 1].start <= b) ++s;
        if (s != cur) {
            cur = s;
            on = open(runs[sp[s].run]);
        }
        if (on) {
            if (u > 0) __syncthreads();
            body(runs[sp[s].run], b - sp[s].start, sp[s].nbx);
        }
    }
}

// the gamma pass of a run runs after its vectors changed, and, with an
// index, only when the index build left some vector's gamma
__device__ __forceinline__ bool gamma_open(const RunView &R)
{
    return *R.vchanged != 0 && (R.gG == 0 || R.gtot[1] != 0);
}

// ---------------------------------------------------------------- Philox
struct W4 {
    uint32_t w[4];
};

__device__ __forceinline__ W4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1)
{
    // the key schedule is computed round by round with scalar adds; a table
    // of the 20 round keys hoisted out of the callers' loops would not fit
    // in scalar registers and be reloaded from spill lanes every round.  The
    // key is a run's seed, uniform over the wavefront (one run per workgroup).
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t x0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t x2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = x0;
        c2 = x2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    W4 r;
    r.w[0] = c0;
    r.w[1] = c1;
    r.w[2] = c2;
    r.w[3] = c3;
    return r;
}

__device__ __forceinline__ W4 draw(const RunView &R, uint32_t sub, uint32_t idx, uint32_t gen,
                                   uint32_t tag)
{
    return philox4x32_10(sub, idx, gen, tag, R.key0, R.key1);
}

// top 24 bits as a uniform in [0,1)
__device__ __forceinline__ double unif24(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

// 53-bit uniform in [0,1) from two words
__device__ __forceinline__ double unif53(uint32_t a, uint32_t b)
{
    const uint64_t v = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return (double)v * 0x1p-53;
}

// integer uniform in [0,n) by multiply-shift
__device__ __forceinline__ uint32_t below(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

// ------------------------------------------------- ordered float encodings
__device__ __forceinline__ uint32_t ord_enc(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_dec(uint32_t e)
{
    const uint32_t u = (e & 0x80000000u) ? (e & 0x7FFFFFFFu) : ~e;
    return __uint_as_float(u);
}

// Partner of each lane at level L of a reduction over groups of 32 lanes,
// every lane active: swaps within quads, the half-row and row mirrors (DPP),
// then the other half of the 32 (a swizzle, xor 16).  Each level pairs two
// sub-groups whose lanes already agree, so after the five levels every lane
// holds its group's result.
template <int L>
__device__ __forceinline__ int partner32(int v)
{
    if constexpr (L == 0) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);
    else if constexpr (L == 1) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);
    else if constexpr (L == 2) return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
    else if constexpr (L == 3) return __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);
    else return __builtin_amdgcn_ds_swizzle(v, 0x401F);  // and 0x1f, xor 0x10
}
template <int L>
__device__ __forceinline__ double partner32(double x)
{
    const int lo = partner32<L>(__double2loint(x)), hi = partner32<L>(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
template <int L>
__device__ __forceinline__ int64_t partner32(int64_t x)
{
    const uint32_t lo = (uint32_t)partner32<L>((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)partner32<L>((int)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The whole-wavefront helpers below (wave_incl_scan, wave_min, wave_max,
// seg_sum<64>) read neighbouring lanes through DPP and lane
// reads, so they are correct only with all 64 lanes active; every call site
// is outside divergent code.  A build with -DRVEA_CHECK_LANES stops a
// wavefront that calls one with inactive lanes (a debugging aid, never
// enabled in the library or its tests).
#ifdef RVEA_CHECK_LANES
#define RVEA_ASSERT_FULL_WAVE()                                                              \
    do {                                                                                     \
        if (__builtin_amdgcn_read_exec() != ~0ull) __builtin_trap();                         \
    } while (0)
#else
#define RVEA_ASSERT_FULL_WAVE() \
    do {                        \
    } while (0)
#endif

// Sum over the S lanes of a segment (S a power of two, 4 <= S <= 64; a
// segment's lanes are all active or all inactive): the pairings of
// partner32, which stay within groups of S lanes, then for a whole
// wavefront the two halves' sums read out and added.  Every lane of the
// segment ends with the same value.
template <int S>
__device__ __forceinline__ double seg_sum(double v)
{
    static_assert(S >= 4 && S <= 64 && (S & (S - 1)) == 0, "segment width");
    v += partner32<0>(v);
    v += partner32<1>(v);
    if constexpr (S >= 8) v += partner32<2>(v);
    if constexpr (S >= 16) v += partner32<3>(v);
    if constexpr (S >= 32) v += partner32<4>(v);
    if constexpr (S == 64) {
        RVEA_ASSERT_FULL_WAVE();
        const double a = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                          __builtin_amdgcn_readlane(__double2loint(v), 0));
        const double b = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 32),
                                          __builtin_amdgcn_readlane(__double2loint(v), 32));
        v = a + b;
    }
    return v;
}

// Inclusive prefix sum over the 64 lanes of a converged wavefront (DPP):
// shifts by 1, 2, 4 and 8 within each row of 16 lanes (lanes without a
// source add 0), then each row adds the last lane of the rows before it
// (row broadcasts of lanes 15 and 31).
__device__ __forceinline__ int wave_incl_scan(int v)
{
    RVEA_ASSERT_FULL_WAVE();
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Wave-wide minimum / maximum of an ordered encoding, for a converged
// wavefront: four DPP steps give every row of 16 lanes its extreme (swaps
// within quads, then the half-row and row mirrors), and the four rows'
// values are read out and combined as scalars (the result is uniform).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t wave_min(uint32_t v)
{
    RVEA_ASSERT_FULL_WAVE();
    v = min(v, dpp_u32<0xB1>(v));   // quad_perm [1,0,3,2]
    v = min(v, dpp_u32<0x4E>(v));   // quad_perm [2,3,0,1]
    v = min(v, dpp_u32<0x141>(v));  // row_half_mirror
    v = min(v, dpp_u32<0x140>(v));  // row_mirror
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return min(min(a, b), min(c, d));
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
    RVEA_ASSERT_FULL_WAVE();
    v = max(v, dpp_u32<0xB1>(v));
    v = max(v, dpp_u32<0x4E>(v));
    v = max(v, dpp_u32<0x141>(v));
    v = max(v, dpp_u32<0x140>(v));
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return max(max(a, b), max(c, d));
}

// Ideal point z* of generation gen (Alg. 1): two buffers alternate by
// parity, so a generation's minima can be reset by the generation before and
// the last selection's z* stays readable.
__device__ __forceinline__ uint32_t *zbuf(const RunView &R, int64_t gen)
{
    return R.zbits + (gen & 1) * R.m;
}

// Child objectives f (m values) of merged row `row` (>= K): the row takes
// part in the selection if finite (else counted), and its values lower the
// ideal point.  Called by one lane per child; the wave's minima are merged
// with one atomic per objective, skipped when the current value is already
// lower (values only decrease, so a stale read only costs an atomic).
__device__ __forceinline__ void child_ideal(const RunView &R, int64_t gen, bool has,
                                            int64_t row, const float *f)
{
    bool ok = has;
    if (has) {
        for (int k = 0; k < R.m; ++k) ok = ok && isfinite(f[k]);
        if (!ok) atomicAdd(&R.counters[0], 1ull);
        R.mvalid[row] = ok ? 1 : 0;
    }
    uint32_t *zb = zbuf(R, gen);
    for (int k = 0; k < R.m; ++k) {
        const uint32_t e = wave_min(ok ? ord_enc(f[k]) : 0xffffffffu);
        if ((threadIdx.x & 63) == 0 &&
            e < __hip_atomic_load(&zb[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMin(&zb[k], e);
    }
}

// x clipped to [lo, hi] (lo <= hi, x not NaN): one binary64 max and min
__device__ __forceinline__ double dclip(double x, double lo, double hi)
{
    return __builtin_fmin(__builtin_fmax(x, lo), hi);
}

}  // namespace rvea
