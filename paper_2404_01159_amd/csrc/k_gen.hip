// k_gen.hip -- population-side kernels: initialization (Alg. 2),
// per-generation bookkeeping of valid slots and free gene rows, and the
// fused offspring kernel (random mating, SBX, polynomial mutation of
// Appendix B, evaluation of Eq. 1).
//
// Layout: genes live in a pool of K+N physical rows of ld floats (ld a
// multiple of 32, rows 128-byte aligned).  slot_row maps each of the K
// population slots to its row; survivors are never copied, offspring are
// written into rows no slot references.
//
// The offspring kernel streams each parent pair once: a segment of S lanes
// (S = 4..64, one wave at most) owns a pair, each lane handles one quad of
// 4 consecutive genes per step (16-byte loads and stores, one Philox call per
// quad giving the 4 genes' SBX variates), and the children's distance terms
// are summed on the fly so evaluation costs no extra pass over the genes.
#include "rvea_dev.h"
#include "rvea_problems.h"
#include "rvea_internal.h"

namespace rvea {

// ------------------------------------------------------------------ scans
// The population's rows are stamped with the generation that will read
// them, and each block of 256 slots counts its valid slots, when the
// population is written (k_newpop, or k_stamp after initialization).  Then,
// before the offspring, each block adds the counts of the blocks before it
// and writes its valid slots to their ascending positions, and reserves room
// for its unstamped (free) rows with one atomic add.  The order of the free
// rows does not matter: it only decides where each child's genes are stored.

// Prepare generation gen = t_done + 1 from population p = t_done (one
// kernel): reset the selection's per-vector minima and the survivors'
// extremes, flag the parent slots that take part (valid, finite F) with
// their share of the ideal point, list the valid slots in ascending order
// (block offsets from the per-block counts left by the previous generation's
// k_newpop, or by k_stamp), and hand out free gene rows for the offspring
// (rows whose stamp is not gen; the free-row counter was cleared by the same
// earlier kernel).
__device__ __forceinline__ void prep_body(const RunView &R, int64_t bx)
{
    const int64_t j = bx * 256 + threadIdx.x;
    // every load first: the row stamp and the earlier blocks' counts do not
    // depend on the generation counter; the slot's flag, objectives and row do
    const int32_t stampj = j < R.K + R.N ? R.stamp[j] : 0;
    int pre = 0;  // valid slots of the earlier blocks (partial sum)
    for (int b = threadIdx.x; b < (int)bx && b < (int)((R.K + 255) / 256); b += 256)
        pre += R.bcount[b];
    const int64_t p = *R.t_done;
    const int32_t gen = (int32_t)(p + 1);
    const float *Fm = fm_of(R, p);
    int v = 0;
    int32_t rowj = 0;
    float fj[kMaxM];
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) fj[k] = 0.f;
    if (j < R.K) {
        v = valid_of(R, p)[j] ? 1 : 0;
        rowj = slot_row_of(R, p)[j];
#pragma unroll
        for (int k = 0; k < kMaxM; ++k)
            if (k < R.m) fj[k] = Fm[j * R.m + k];
    }
    if (j < R.K) R.key[j] = ~0ull;
    if (j < R.m) {
        R.rbits[j] = 0xffffffffu;  // survivors' minimum
        R.rbits[R.m + j] = 0u;     // survivors' maximum
    }
    // Eq. 4 penalty factor m (t/t_max)^alpha of this generation, computed by
    // the last block (free rows only, the least work), off the others' path
    if (bx == (R.K + R.N + 255) / 256 - 1 && threadIdx.x == 0)
        *R.pen = (double)R.m * pow((double)gen / (double)R.t_max, R.alpha);
    bool take = false;
    if (j < R.K) {
        bool fin = true;
#pragma unroll
        for (int k = 0; k < kMaxM; ++k)
            if (k < R.m) fin = fin && isfinite(fj[k]);
        if (v && !fin) atomicAdd(&R.counters[0], 1ull);
        take = v && fin;
        R.mvalid[j] = take ? 1 : 0;
    }
    const int fr = (j < R.K + R.N && stampj != gen) ? 1 : 0;
    // the block's three sums in one scan: earlier blocks' valid slots, this
    // block's valid slots (positions), its free rows (positions)
    __shared__ int wsum[3][4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int x0 = wave_incl_scan(pre), x1 = wave_incl_scan(v), x2 = wave_incl_scan(fr);
    if (lane == 63) {
        wsum[0][wid] = x0;
        wsum[1][wid] = x1;
        wsum[2][wid] = x2;
    }
    // each wavefront's minima in a slot of its own (no shared initial value
    // that another wavefront could reach first), merged after the barrier
    __shared__ uint32_t zw[4][kMaxM];
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
        if (k < R.m) {
            const uint32_t e = wave_min(take ? ord_enc(fj[k]) : 0xffffffffu);
            if (lane == 0) zw[wid][k] = e;
        }
    }
    __syncthreads();
    int offset = 0, tot = 0, ftot = 0, before1 = 0, before2 = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        offset += wsum[0][w];
        tot += wsum[1][w];
        ftot += wsum[2][w];
        before1 += w < wid ? wsum[1][w] : 0;
        before2 += w < wid ? wsum[2][w] : 0;
    }
    const int pos = before1 + x1 - v, fpos = before2 + x2 - fr;
    if (v)  // the slot and its row: a parent's genes are one lookup away
        reinterpret_cast<int2 *>(R.vs)[offset + pos] = make_int2((int32_t)j, rowj);
    const int64_t nblk = (R.K + 255) / 256;
    if (bx == nblk - 1 && threadIdx.x == 0) *R.nvalid = offset + tot;
    if (threadIdx.x < R.m) {
        const int k = threadIdx.x;
        const uint32_t e = min(min(zw[0][k], zw[1][k]), min(zw[2][k], zw[3][k]));
        if (e != 0xffffffffu) atomicMin(&zbuf(R, gen)[k], e);
    }
    // free rows of this block: one atomic reserves their places
    __shared__ int fbase;
    if (threadIdx.x == 0) fbase = ftot ? atomicAdd(R.freecnt, ftot) : 0;
    __syncthreads();
    if (fr && fbase + fpos < R.N) R.off_row[fbase + fpos] = (int32_t)j;
}

__global__ __launch_bounds__(256) void k_prep(RunView R) { prep_body(R, blockIdx.x); }

// Row stamps, per-block valid counts and a cleared free-row counter for the
// current population p = t_done, as k_newpop leaves them; run after
// initialization and after the state is set from the host.
__device__ __forceinline__ void stamp_body(const RunView &R, int64_t bx)
{
    const int64_t j = bx * 256 + threadIdx.x;
    const int64_t p = *R.t_done;
    int v = 0;
    if (j < R.K && valid_of(R, p)[j]) {
        v = 1;
        R.stamp[slot_row_of(R, p)[j]] = (int32_t)(p + 1);
    }
    const unsigned long long b = __ballot(v);
    __shared__ int wc[4];
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        R.bcount[bx] = wc[0] + wc[1] + wc[2] + wc[3];
        if (bx == 0) *R.freecnt = 0;
    }
}

__global__ __launch_bounds__(256) void k_stamp(RunView R) { stamp_body(R, blockIdx.x); }

// --------------------------------------------------------------- helpers
// z^n for a positive integer n (square and multiply, n uniform); the
// default distribution index eta = 20 (n = 21) gets straight-line code
__device__ __forceinline__ double ipow(double z, int n)
{
    if (n == 21) {
        const double z2 = z * z, z4 = z2 * z2, z8 = z4 * z4, z16 = z8 * z8;
        return (z16 * z4) * z;
    }
    double r = 1.0, b = z;
    while (n) {
        if (n & 1) r *= b;
        n >>= 1;
        if (n) b *= b;
    }
    return r;
}

// 1/z for z in (0, 4): hardware estimate plus two Newton-Raphson steps,
// within one binary64 ulp
__device__ __forceinline__ double recip(double z)
{
    double r = __builtin_amdgcn_rcp(z);
    r = fma(r, fma(-z, r, 1.0), r);
    r = fma(r, fma(-z, r, 1.0), r);
    return r;
}

// a^(-1/n), a in (0, 2], n a positive integer (NR > 0: n = NR fixed at
// compile time, else n = nrt).  A single-precision estimate z (relative error
// below 1e-6) and one third-order correction: with e = 1 - a z^n the root is
// z (1 - e)^(-1/n) = z (1 + e/n + (n+1)/(2n^2) e^2 + O(e^3)), and the O(e^3)
// remainder is below 1e-18.  The rounding of a z^n (about n/2 binary64 ulps)
// enters divided by n, so the result is within a few binary64 ulps.
template <int NR>
__device__ __forceinline__ double inv_root(double a, int nrt)
{
    const int n = NR > 0 ? NR : nrt;
    // callers pass a >= 1e-30 (a normal binary32), so the hardware log2 and
    // exp2 (no denormal handling) suffice for the estimate
    const float ninv = 1.0f / (float)n;
    const double z = (double)__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf((float)a) * ninv);
    const double e = fma(-a, ipow(z, n), 1.0);
    const double dn = 1.0 / (double)n;
    const double c2 = (double)(n + 1) / (2.0 * (double)n * (double)n);
    return fma(z * e, fma(e, c2, dn), z);
}

// polynomial mutation shift Delta of Appendix B, binary64:
//   M < 1/2: (ub-lb) [(2M + (1-2M)(1-d1)^(xi+1))^(1/(xi+1)) - 1]
//   M > 1/2: (ub-lb) [1 - (2(1-M) + 2(M-1/2)(1-d2)^(xi+1))^(1/(xi+1))]
// d1 = (x-lb)/(ub-lb), d2 = (ub-x)/(ub-lb).  For integer n = xi+1 the
// power is a product and the root the one above; otherwise pow().
__device__ __attribute__((noinline)) double pm_delta_pow(double x, double lb, double ub,
                                                        double mm, double xi)
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

// NR > 0: n = xi + 1 = NR fixed at compile time; else n = nrt (0: not an
// integer in [1, 64], pow())
template <int NR>
__device__ __forceinline__ double pm_delta(double x, double lb, double ub, double mm, double xi,
                                           int nrt)
{
    const int n = NR > 0 ? NR : nrt;
    if (NR <= 0 && n <= 0) return pm_delta_pow(x, lb, ub, mm, xi);
    if (mm == 0.5) return 0.0;
    const double span = ub - lb;
    const bool lo = mm < 0.5;
    const double dd = lo ? (x - lb) / span : (ub - x) / span;
    const double base = lo ? 2.0 * mm + (1.0 - 2.0 * mm) * ipow(1.0 - dd, n)
                           : 2.0 * (1.0 - mm) + 2.0 * (mm - 0.5) * ipow(1.0 - dd, n);
    if (base > 0.0 && base < 1e-30) return pm_delta_pow(x, lb, ub, mm, xi);  // below float range
    const double r = base > 0.0 ? recip(inv_root<NR>(base, n)) : 0.0;
    return lo ? span * (r - 1.0) : span * (1.0 - r);
}

__device__ __attribute__((noinline)) double sbx_beta_pow(double mc, double eta)
{
    const double e = 1.0 / (eta + 1.0);
    if (mc < 0.5) return pow(2.0 * mc, e);
    return pow(2.0 - 2.0 * mc, -e);
}

// SBX spread factor (Appendix B): (2 M_c)^(1/(eta+1)) below 1/2,
// (2 - 2 M_c)^(-1/(eta+1)) above, in binary64.  When n = eta+1 is a small
// integer (NR > 0: n = NR fixed at compile time, else n = nrt > 0) the root
// a^(-1/n) is inv_root's, and 1/root below 1/2; other eta use pow().  Branch
// free: M_c = 0 (spread 0) computes the root of 1 and discards it.
template <int NR>
__device__ __forceinline__ double sbx_beta(double mc, double eta, int nrt)
{
    if (NR > 0 || nrt > 0) {
        const bool lo = mc < 0.5;
        const bool zero = mc == 0.0;
        double a = lo ? 2.0 * mc : 2.0 - 2.0 * mc;
        a = zero ? 1.0 : a;
        const double z = inv_root<NR>(a, nrt);
        const double b = lo ? recip(z) : z;
        return zero ? 0.0 : b;
    }
    return sbx_beta_pow(mc, eta);
}

// ------------------------------------------------------------------- init
// Slot i < N: genes from counter (q, i, 0, TAG_INIT), gene 4q+k from word k,
// x = lb + (ub-lb) u24 rounded to float; evaluated in the same pass.
template <int S>
__global__ __launch_bounds__(kBlock) void k_init(RunView R)
{
    const int seg = threadIdx.x / S, lane = threadIdx.x % S;
    const int64_t i = (int64_t)blockIdx.x * (kBlock / S) + seg;
    if (i >= R.N) return;  // uniform per segment
    const int Q = (R.d + 3) / 4;
    float *row = R.X + i * (int64_t)R.ld;
    const double span = R.ub - R.lb;
    double gsum = 0.0;
    float pv[4] = {0.f, 0.f, 0.f, 0.f};
    for (int q = lane; q < Q; q += S) {
        const W4 w = draw(R, (uint32_t)q, (uint32_t)i, 0u, TAG_INIT);
        float x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double scaled = span * unif24(w.w[k]);
            x[k] = (float)(R.lb + scaled);
            const int g = 4 * q + k;
            if (g < R.d && g >= R.m - 1) gsum += (double)dist_term(R.problem, x[k]);
        }
        if (q < 2) {
#pragma unroll
            for (int k = 0; k < 4; ++k) pv[k] = x[k];
        }
        *reinterpret_cast<float4 *>(row + 4 * q) = make_float4(x[0], x[1], x[2], x[3]);
    }
    gsum = seg_sum<S>(gsum);
    float pos[kMaxM];
#pragma unroll
    for (int k = 0; k < kMaxM - 1; ++k) pos[k] = __shfl(pv[k & 3], k >> 2, S);
    if (lane == 0) {
        float f[kMaxM];
        finish_objectives(R.problem, R.m, R.d, pos, gsum, f);
        for (int k = 0; k < R.m; ++k) R.Fms[i * R.m + k] = f[k];  // population 0
        R.valids[i] = 1;
        R.slot_rows[i] = (int32_t)i;
    }
}

// empty slots N..K-1 and the generation counter
__global__ void k_init_empty(RunView R)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + R.N;
    if (j < R.K) {
        R.valids[j] = 0;  // population 0
        R.slot_rows[j] = (int32_t)j;
        for (int k = 0; k < R.m; ++k) R.Fms[j * R.m + k] = __int_as_float(0x7fc00000);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *R.t_done = 0;
}

// --------------------------------------------------------------- offspring
// Mutation sites of child o: events e = 0,1,... with counter (e, o, t,
// TAG_MUT); U = 1 - u53(w0,w1) in (0,1], gap = floor(log U / log(1-p)),
// site_e = site_{e-1} + 1 + gap while it stays below d; M_mut = u53(w2,w3).
// Both children of a pair are drawn at once, S/2 lanes each per round.
template <int S>
__device__ void draw_sites(const RunView &R, uint32_t t, int64_t o1, int64_t o2, bool has2,
                           double lq, int lane, int32_t *s1, double *m1, int32_t *s2, double *m2,
                           int *n1, int *n2)
{
    constexpr int H2 = S / 2;
    const int c = lane / H2, hl = lane % H2;
    const int64_t o = c ? o2 : o1;
    int32_t *sites = c ? s2 : s1;
    double *mags = c ? m2 : m1;
    int cur = -1;           // position before this round
    bool done = c ? !has2 : false;
    int count = 0;
    for (int round = 0;; ++round) {
        const bool any_left = __any(!done);  // wave-uniform continuation
        if (!any_left) break;
        const uint32_t e = (uint32_t)(round * H2 + hl);
        int step = 0;
        double mag = 0.0;
        if (!done) {
            const W4 w = draw(R, e, (uint32_t)o, t, TAG_MUT);
            const double U = 1.0 - unif53(w.w[0], w.w[1]);
            double q = log(U) / lq;
            if (!(q >= 0.0)) q = 0.0;
            const double gap = floor(q);
            step = gap >= (double)R.d ? R.d + 1 : 1 + (int)gap;
            mag = unif53(w.w[2], w.w[3]);
        }
        int incl = step;
#pragma unroll
        for (int off = 1; off < H2; off <<= 1) {
            const int y = __shfl_up(incl, off, H2);
            if (hl >= off) incl += y;
        }
        const int pos = cur + incl;
        if (!done && pos < R.d) {
            const int idx = round * H2 + hl;
            if (idx < kMaxSites) {
                sites[idx] = pos;
                mags[idx] = mag;
            } else {
                atomicAdd(&R.counters[2], 1ull);
            }
        }
        const int last = __shfl(pos, H2 - 1, H2);
        int mine = (!done && pos < R.d) ? 1 : 0;
#pragma unroll
        for (int off = H2 / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off, H2);
        if (!done) {
            count += mine;
            cur = last;
            if (last >= R.d) done = true;
        }
    }
    const int cnt1 = __shfl(count, 0, S);
    const int cnt2 = __shfl(count, H2, S);
    *n1 = cnt1 < kMaxSites ? cnt1 : kMaxSites;
    *n2 = cnt2 < kMaxSites ? cnt2 : kMaxSites;
}

// Distance term of one gene: DK = 1 multimodal, 2 quadratic, -1 chosen by
// the problem id at run time.
template <int DK>
__device__ __forceinline__ float dterm(int problem, float z)
{
    return dist_term(DK > 0 ? DK : problem, z);
}

// One segment of S lanes per parent pair.  NR > 0 compiles in the root index
// n = eta + 1 = NR of both SBX and mutation; DK = 0 skips evaluation (the
// policy problem has its own rollout kernel), DK > 0 fixes the distance term
// and DK = -1 reads problem and indices from the run (the batched kernel).
// Every variant takes the same arithmetic steps, so results do not depend on
// which one ran.
template <int S, int NR, int DK, int BS>
__device__ __forceinline__ void offspring_body(const RunView &R, int64_t bx)
{
    constexpr int SEGS = BS / S;
    __shared__ int32_t sh_sites[SEGS][2][kMaxSites];
    __shared__ double sh_mags[SEGS][2][kMaxSites];
    __shared__ float sh_vals[SEGS][2][kMaxSites];  // mutated gene at each site
    __shared__ uint32_t szmin[kMaxM];
    if (threadIdx.x < kMaxM) szmin[threadIdx.x] = 0xffffffffu;

    const int seg = threadIdx.x / S, lane = threadIdx.x % S;
    const int64_t P = (R.N + 1) / 2;
    // segment u of the grid: pair p, part sp of its genes (osplit parts)
    const int ns = R.osplit;
    const int64_t u = bx * SEGS + seg;
    const int64_t p = ns == 1 ? u : u / ns;
    const int sp = ns == 1 ? 0 : (int)(u - p * ns);
    const bool active = p < P;
    const int64_t pop = *R.t_done;  // the parents' population
    const uint32_t t = (uint32_t)(pop + 1);
    float *Fm = fm_of(R, pop);
    const int64_t o1 = p, o2 = p + P;
    const bool has2 = o2 < R.N;
    const uint32_t nv = (uint32_t)*R.nvalid;
    if (nv == 0) {  // no parent left (every row was non-finite): offspring are empty
        if (active && lane == 0 && sp == 0) {
            for (int k = 0; k < R.m; ++k) {
                Fm[(R.K + o1) * R.m + k] = __int_as_float(0x7fc00000);
                if (has2) Fm[(R.K + o2) * R.m + k] = __int_as_float(0x7fc00000);
            }
            R.mvalid[R.K + o1] = 0;
            if (has2) R.mvalid[R.K + o2] = 0;
            atomicAdd(&R.counters[0], has2 ? 2ull : 1ull);
        }
        return;  // uniform over the grid
    }

    // random mating: two uniform draws over the valid slots
    // (inactive segments draw too and leave the values unused: without a
    // conditional join the loads are waited for only where they are used)
    const W4 wm = draw(R, 0u, (uint32_t)p, t, TAG_MATE);
    const int2 ea = reinterpret_cast<const int2 *>(R.vs)[below(wm.w[0], nv)];
    const int2 eb = reinterpret_cast<const int2 *>(R.vs)[below(wm.w[1], nv)];
    const int32_t a = ea.x, rowa = ea.y, b = eb.x, rowb = eb.y;

    // the children's rows: they do not depend on the mating, so their loads
    // are issued before the sites are drawn (clamped indices for inactive
    // segments and a missing second child, values unused)
    const int32_t orow1 = R.off_row[active ? o1 : 0];
    const int32_t orow2 = R.off_row[active && has2 ? o2 : 0];

    // mutation sites of both children
    int n1 = 0, n2 = 0;
    const double pr = R.p_m / (double)R.d;
    if (pr > 0.0) {
        const double lq = log1p(-(pr > 1.0 ? 1.0 : pr));
        if (active)
            draw_sites<S>(R, t, o1, o2, has2, lq, lane, sh_sites[seg][0], sh_mags[seg][0],
                          sh_sites[seg][1], sh_mags[seg][1], &n1, &n2);
    }
    __syncthreads();
    const bool evaluate = DK > 0 || (DK < 0 && R.problem != kPolicy);
    if (active) {
        bool nocross = false;
        if (R.p_c < 1.0) {
            const W4 w = draw(R, 0u, (uint32_t)p, t, TAG_SBXPAIR);
            nocross = ((double)w.w[0] * 0x1p-32) > R.p_c;
        }

        const float *x1row = R.X + (int64_t)rowa * R.ld;
        const float *x2row = R.X + (int64_t)rowb * R.ld;
        float *c1row = R.X + (int64_t)orow1 * R.ld;
        float *c2row = has2 ? R.X + (int64_t)orow2 * R.ld : nullptr;
        const int Q = (R.d + 3) / 4;
        // this segment's quads: part sp of ns contiguous parts
        const int qn = ns == 1 ? Q : (Q + ns - 1) / ns;
        const int qa = sp * qn, qb = qa + qn < Q ? qa + qn : Q;
        const double lb = R.lb, ub = R.ub;
        const float flb = (float)lb, fub = (float)ub;
        const double np1 = R.eta_c + 1.0;
        const int nroot =
            NR > 0 ? NR : (np1 >= 1.0 && np1 <= 64.0 && np1 == (double)(int)np1) ? (int)np1 : 0;
        const double nm1 = R.eta_m + 1.0;
        const int nroot_m =
            NR > 0 ? NR : (nm1 >= 1.0 && nm1 <= 64.0 && nm1 == (double)(int)nm1) ? (int)nm1 : 0;
        const int mlo = R.m - 1;  // first distance variable
        double g1 = 0.0, g2 = 0.0;
        float pv1[4] = {0.f, 0.f, 0.f, 0.f}, pv2[4] = {0.f, 0.f, 0.f, 0.f};

        // the pair's mutation sites in this segment's genes, one lane per
        // site and both children at once: the site's SBX child (the binary64
        // steps of the streaming loop below, from the same Philox word) and
        // its polynomial mutation, kept as the final binary32 gene, so the
        // loop only substitutes them
        const int nsites = n1 + n2;
        for (int b0 = 0; b0 < nsites; b0 += S) {  // uniform per segment
            const int idx = b0 + lane;
            const int c = idx < n1 ? 0 : 1;
            const int k = c ? idx - n1 : idx;
            const int g = idx < nsites ? sh_sites[seg][c][k] : -1;
            if (g >= 4 * qa && g < 4 * qb) {
                const W4 w = draw(R, (uint32_t)(g >> 2), (uint32_t)p, t, TAG_SBX);
                const int kk = g & 3;
                const uint32_t word = kk == 0 ? w.w[0] : kk == 1 ? w.w[1] : kk == 2 ? w.w[2] : w.w[3];
                const double xa_ = (double)x1row[g], xb_ = (double)x2row[g];
                const double hs = ((word >> 7) & 1u) ? 0.5 : -0.5;
                double hB = hs * sbx_beta<NR>(unif24(word), R.eta_c, nroot);
                if (((word >> 6) & 1u) || nocross) hB = 0.5;
                const double hm = 0.5 * (xa_ + xb_), dd = xa_ - xb_;
                const double x = dclip(fma(c == 0 ? hB : -hB, dd, hm), lb, ub);
                const double mg = sh_mags[seg][c][k];
                sh_vals[seg][c][k] =
                    (float)dclip(x + pm_delta<NR>(x, lb, ub, mg, R.eta_m, nroot_m), lb, ub);
            }
        }

        // mutation sites (ascending) seen through a cursor per child: this
        // lane's quads ascend, so the next site at or after the quad is
        // found by advancing past the other lanes' sites
        const int32_t *st1 = sh_sites[seg][0], *st2 = sh_sites[seg][1];
        const float *mv1 = sh_vals[seg][0], *mv2 = sh_vals[seg][1];
        int p1 = 0, p2 = 0;
        int nx1 = n1 > 0 ? st1[0] : INT_MAX, nx2 = n2 > 0 ? st2[0] : INT_MAX;

        for (int q = qa + lane; q < qb; q += S) {
            const float4 xa = *reinterpret_cast<const float4 *>(x1row + 4 * q);
            const float4 xb = *reinterpret_cast<const float4 *>(x2row + 4 * q);
            const float pa[4] = {xa.x, xa.y, xa.z, xa.w};
            const float pb[4] = {xb.x, xb.y, xb.z, xb.w};
            const W4 w = draw(R, (uint32_t)q, (uint32_t)p, t, TAG_SBX);
            const int g0 = 4 * q;
            // children ((1 +- B) x1 + (1 -+ B) x2) / 2 in binary64 as
            // (x1 + x2)/2 +- (B/2)(x1 - x2): one rounding from the sum and
            // difference, within a few ulps of the product form (B = 1, a
            // copy, is exact), then rounded to binary32 and clipped there
            // (the same result as clipping in binary64 first, since rounding
            // to binary32 is monotone)
            float y1[4], y2[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t word = w.w[k];
                const double hs = ((word >> 7) & 1u) ? 0.5 : -0.5;
                double hB = hs * sbx_beta<NR>(unif24(word), R.eta_c, nroot);
                if (((word >> 6) & 1u) || nocross) hB = 0.5;
                const double xa_ = (double)pa[k], xb_ = (double)pb[k];
                const double hm = 0.5 * (xa_ + xb_), dd = xa_ - xb_;
                y1[k] = fminf(fmaxf((float)fma(hB, dd, hm), flb), fub);
                y2[k] = fminf(fmaxf((float)fma(-hB, dd, hm), flb), fub);
            }
            // genes of this quad that are mutation sites take their mutated
            // values (the sites ascend, so each cursor moves forward only)
            while (nx1 < g0) nx1 = ++p1 < n1 ? st1[p1] : INT_MAX;
            while (nx2 < g0) nx2 = ++p2 < n2 ? st2[p2] : INT_MAX;
            while (nx1 < g0 + 4) {
                const float v = mv1[p1];
                const int k = nx1 - g0;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) y1[kk] = kk == k ? v : y1[kk];
                nx1 = ++p1 < n1 ? st1[p1] : INT_MAX;
            }
            while (nx2 < g0 + 4) {
                const float v = mv2[p2];
                const int k = nx2 - g0;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) y2[kk] = kk == k ? v : y2[kk];
                nx2 = ++p2 < n2 ? st2[p2] : INT_MAX;
            }
            if (evaluate) {
                // the quad's distance terms, summed in single precision and
                // added to the double sums; positions and padding count 0
                float t1[4], t2[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    t1[k] = dterm<DK>(R.problem, y1[k]);
                    t2[k] = dterm<DK>(R.problem, y2[k]);
                }
                if (g0 < mlo || g0 + 4 > R.d) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (g0 + k < mlo || g0 + k >= R.d) {
                            t1[k] = 0.0f;
                            t2[k] = 0.0f;
                        }
                    }
                }
                g1 += (double)((t1[0] + t1[1]) + (t1[2] + t1[3]));
                g2 += (double)((t2[0] + t2[1]) + (t2[2] + t2[3]));
            }
            if (q < 2) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    pv1[k] = y1[k];
                    pv2[k] = y2[k];
                }
            }
            *reinterpret_cast<float4 *>(c1row + g0) = make_float4(y1[0], y1[1], y1[2], y1[3]);
            if (has2) *reinterpret_cast<float4 *>(c2row + g0) = make_float4(y2[0], y2[1], y2[2], y2[3]);
        }
        g1 = seg_sum<S>(g1);
        g2 = seg_sum<S>(g2);
        // a pair split over segments: each stores its partial sums, which
        // the finishing kernel adds in part order (kernel order makes them
        // visible) to form the pair's objectives
        bool fin = true;
        if (evaluate && ns > 1) {
            if (lane == 0) {
                double *gp = R.gpart + (p * ns + sp) * 2;
                gp[0] = g1;
                gp[1] = g2;
            }
            fin = false;
        }
        float pos1[kMaxM], pos2[kMaxM];
#pragma unroll
        for (int k = 0; k < kMaxM - 1; ++k) {
            pos1[k] = __shfl(pv1[k & 3], k >> 2, S);
            pos2[k] = __shfl(pv2[k & 3], k >> 2, S);
        }
        if (evaluate && fin && (lane == 0 || (lane == 1 && has2))) {
            // objectives, child 1 on lane 0 and child 2 on lane 1 (two lanes
            // finish them side by side); rows that take part (finite F) and
            // their LDS minima
            auto emit = [&](const float(&pos)[kMaxM], double gs, int64_t row) {
                float f[kMaxM];
                finish_objectives(R.problem, R.m, R.d, pos, gs, f);
                float *Fr = Fm + row * R.m;
                bool ok = true;
#pragma unroll
                for (int k = 0; k < kMaxM; ++k) {
                    if (k < R.m) {
                        Fr[k] = f[k];
                        ok = ok && isfinite(f[k]);
                    }
                }
                R.mvalid[row] = ok ? 1 : 0;
                if (!ok) {
                    atomicAdd(&R.counters[0], 1ull);
                    return;
                }
#pragma unroll
                for (int k = 0; k < kMaxM; ++k)
                    if (k < R.m) atomicMin(&szmin[k], ord_enc(f[k]));
            };
            float pos[kMaxM];
#pragma unroll
            for (int k = 0; k < kMaxM - 1; ++k) pos[k] = lane == 0 ? pos1[k] : pos2[k];
            pos[kMaxM - 1] = 0.f;
            emit(pos, lane == 0 ? g1 : g2, R.K + (lane == 0 ? o1 : o2));
        }
    }
    // the workgroup's share of the ideal point: one guarded atomic per
    // objective (values only decrease, so a stale read costs an atomic at most)
    __syncthreads();
    if (evaluate && threadIdx.x < R.m) {
        const uint32_t e = szmin[threadIdx.x];
        uint32_t *zb = zbuf(R, t);
        // a relaxed atomic read: unlike a volatile one it does not wait for
        // the wavefront's outstanding stores
        if (e < __hip_atomic_load(&zb[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMin(&zb[threadIdx.x], e);
    }
    // the parents' slots (kept for the host): stored last, so that no wait
    // for an earlier load also waits for this store
    if (active && lane == 0 && sp == 0) {
        R.parents[2 * p] = a;
        R.parents[2 * p + 1] = b;
    }
}

// Workgroups of one wavefront (kOffBlock): the pairs spread over the CUs in
// the finest steps (the kernel's few wavefronts per SIMD make
// whole-workgroup granularity visible as idle SIMDs).

template <int S, int NR, int DK>
__global__ __launch_bounds__(kOffBlock) void k_offspring(RunView R)
{
    offspring_body<S, NR, DK, kOffBlock>(R, blockIdx.x);
}

// Objectives of the children of pairs split over segments (osplit > 1),
// one lane per child: the parts' distance sums added in part order, the
// position genes read back from the child's row; then, as in the offspring
// kernel, the row's take-part flag, the non-finite count and the children's
// share of the ideal point.
__device__ __forceinline__ void offspring_finish_body(const RunView &R, int64_t bx)
{
    const int64_t o = bx * 256 + threadIdx.x;
    const int64_t P = (R.N + 1) / 2;
    const int64_t pop = *R.t_done;
    if (*R.nvalid == 0) return;  // no parent: the offspring kernel left empty children
    float *Fm = fm_of(R, pop);
    const bool has = o < R.N;
    float f[kMaxM] = {};
    if (has) {
        const int64_t p = o < P ? o : o - P;
        const int c = o < P ? 0 : 1;
        const int ns = R.osplit;
        double g = 0.0;
        for (int k = 0; k < ns; ++k) g += R.gpart[(p * ns + k) * 2 + c];
        const float *row = R.X + (int64_t)R.off_row[o] * R.ld;
        float pos[kMaxM];
#pragma unroll
        for (int k = 0; k < kMaxM - 1; ++k) pos[k] = k < R.m - 1 ? row[k] : 0.f;
        pos[kMaxM - 1] = 0.f;
        finish_objectives(R.problem, R.m, R.d, pos, g, f);
#pragma unroll
        for (int k = 0; k < kMaxM; ++k)
            if (k < R.m) Fm[(R.K + o) * R.m + k] = f[k];
    }
    child_ideal(R, pop + 1, has, R.K + o, f);
}

__global__ __launch_bounds__(256) void k_offspring_finish(RunView R)
{
    offspring_finish_body(R, blockIdx.x);
}

// ----------------------------------------------------- batched (many runs)
__global__ __launch_bounds__(256) void kb_prep(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    prep_body(runs[sp[s].run], blockIdx.x - sp[s].start);
}
// batched: one-wavefront workgroups as above; NR = 21 when every run of the
// launch has the default distribution indices (the same arithmetic as the
// general variant, so results do not depend on the batch's make-up)
template <int S, int NR>
__global__ __launch_bounds__(kOffBlock) void kb_offspring(const RunView *runs, const Span *sp,
                                                          int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    offspring_body<S, NR, -1, kOffBlock>(runs[sp[s].run], blockIdx.x - sp[s].start);
}
__global__ __launch_bounds__(256) void kb_offspring_finish(const RunView *runs, const Span *sp,
                                                           int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    offspring_finish_body(runs[sp[s].run], blockIdx.x - sp[s].start);
}

// ------------------------------------------------------------- launchers
int pick_segment(int d)
{
    const int Q = (d + 3) / 4;
    int S = 4;
    while (S < 64 && S < Q) S <<= 1;
    return S;
}

// The offspring kernel runs 4 wavefronts per SIMD (its register use), so
// 256 CUs hold 4,096 at once.  Rows of 256 genes or more take 32-lane
// segments (two pairs per wavefront, twice the quads per lane) instead of
// 64-lane ones when there are more pairs than resident wavefronts, and,
// for rows under 2,048 genes, already above a quarter of that: a pair's own
// work (mating, mutation sites, objectives) is then shared by the two
// pairs of a wavefront, which outweighs having fewer wavefronts; long rows
// with few pairs keep one pair per wavefront for the wavefront count.  A
// fixed constant, not the device's count, so that results (the order of the
// distance sums) do not depend on the device or on whether the run is
// batched.
constexpr int64_t kResidentOffspringWaves = 4096;

int offspring_segment(int d, int64_t N)
{
    const int S = pick_segment(d);
    const int64_t P = (N + 1) / 2;
    if (S == 64 && (P > kResidentOffspringWaves || (P > kResidentOffspringWaves / 4 && d < 2048)))
        return 32;
    return S;
}

// Few pairs of long rows (fewer pairs than the resident wavefronts, rows of
// at least two 64-lane passes): each pair's genes are split into contiguous
// parts, one 64-lane segment each, enough to fill the resident wavefronts,
// each part at least two quads per lane.  A function of d and N only, so
// that results (the order of the distance sums) do not depend on the device
// or on whether the run is batched.
int offspring_splits(int d, int64_t N)
{
    const int S = offspring_segment(d, N);
    const int64_t P = (N + 1) / 2;
    const int64_t Q = (d + 3) / 4;
    if (S < 64 || P >= kResidentOffspringWaves) return 1;
    int64_t ns = (kResidentOffspringWaves + P - 1) / P;
    const int64_t most = Q / (2 * S);
    if (ns > most) ns = most;
    if (ns > 256) ns = 256;
    return ns < 1 ? 1 : (int)ns;
}

#define RVEA_SEG_DISPATCH(S, KERNEL, GRID_UNITS, STREAM, VIEW)                                 \
    do {                                                                                     \
        const int64_t units_ = (GRID_UNITS);                                                 \
        switch (S) {                                                                         \
        case 4: KERNEL<4><<<dim3((unsigned)((units_ + 63) / 64)), kBlock, 0, STREAM>>>(VIEW);  \
            break;                                                                           \
        case 8: KERNEL<8><<<dim3((unsigned)((units_ + 31) / 32)), kBlock, 0, STREAM>>>(VIEW);  \
            break;                                                                           \
        case 16: KERNEL<16><<<dim3((unsigned)((units_ + 15) / 16)), kBlock, 0, STREAM>>>(VIEW); \
            break;                                                                           \
        case 32: KERNEL<32><<<dim3((unsigned)((units_ + 7) / 8)), kBlock, 0, STREAM>>>(VIEW);   \
            break;                                                                           \
        default: KERNEL<64><<<dim3((unsigned)((units_ + 3) / 4)), kBlock, 0, STREAM>>>(VIEW);   \
            break;                                                                           \
        }                                                                                    \
    } while (0)

hipError_t launch_batch_gen(int phase, int cls, const RunView *runs, const Span *sp, int n,
                            int64_t blocks, hipStream_t s)
{
    const dim3 g((unsigned)blocks);
    switch (phase) {
    case BP_PREP: kb_prep<<<g, 256, 0, s>>>(runs, sp, n); break;
    case BP_OFFSPRING:
#define RVEA_KBOFF(NRV)                                                                      \
    switch (cls & kSegMask) {                                                                \
    case 4: kb_offspring<4, NRV><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;                \
    case 8: kb_offspring<8, NRV><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;                \
    case 16: kb_offspring<16, NRV><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;              \
    case 32: kb_offspring<32, NRV><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;              \
    default: kb_offspring<64, NRV><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;              \
    }
        if (cls & kDefaultIndices)
            RVEA_KBOFF(21)
        else
            RVEA_KBOFF(0)
#undef RVEA_KBOFF
        break;
    case BP_OFFSPRING_FIN: kb_offspring_finish<<<g, 256, 0, s>>>(runs, sp, n); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init(const RunView &R, hipStream_t s)
{
    const int S = pick_segment(R.d);
    if (R.problem == kPolicy) {
        const hipError_t e = launch_init_gauss(R, s);
        if (e != hipSuccess) return e;
    } else if (R.N > 0) {
        RVEA_SEG_DISPATCH(S, k_init, R.N, s, R);
    }
    const int64_t empty = R.K - R.N;
    const unsigned g = (unsigned)((empty > 0 ? empty : 1) + 255) / 256;
    k_init_empty<<<g, 256, 0, s>>>(R);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && R.problem == kPolicy)  // objectives of the initial slots by rollouts
        e = launch_rollout(R, s, false);
    if (e == hipSuccess) e = launch_stamp(R, s);
    return e;
}

hipError_t launch_stamp(const RunView &R, hipStream_t s)
{
    k_stamp<<<(unsigned)((R.K + 255) / 256), 256, 0, s>>>(R);
    return hipGetLastError();
}

hipError_t launch_prepare(const RunView &R, hipStream_t s)
{
    k_prep<<<(unsigned)((R.K + R.N + 255) / 256), 256, 0, s>>>(R);
    return hipGetLastError();
}

static dim3 blocks_of(int64_t units, int per) { return dim3((unsigned)((units + per - 1) / per)); }

template <int NR, int DK>
void launch_offspring_as(const RunView &R, hipStream_t s)
{
    const int S = offspring_segment(R.d, R.N);
    const int64_t P = (R.N + 1) / 2 * R.osplit;  // segments
    switch (S) {
    case 4: k_offspring<4, NR, DK><<<blocks_of(P, kOffBlock / 4), kOffBlock, 0, s>>>(R); break;
    case 8: k_offspring<8, NR, DK><<<blocks_of(P, kOffBlock / 8), kOffBlock, 0, s>>>(R); break;
    case 16: k_offspring<16, NR, DK><<<blocks_of(P, kOffBlock / 16), kOffBlock, 0, s>>>(R); break;
    case 32: k_offspring<32, NR, DK><<<blocks_of(P, kOffBlock / 32), kOffBlock, 0, s>>>(R); break;
    default: k_offspring<64, NR, DK><<<blocks_of(P, kOffBlock / 64), kOffBlock, 0, s>>>(R); break;
    }
}

hipError_t launch_offspring(const RunView &R, hipStream_t s)
{
    if (R.op != OP_GA) return launch_operator(R, s);
    // the default distribution indices (eta_c = eta_m = 20) get the root
    // index compiled in; any other run takes the general kernel
    if (R.eta_c == 20.0 && R.eta_m == 20.0) {
        if (R.problem == kPolicy)
            launch_offspring_as<21, 0>(R, s);
        else if (R.problem == 2)
            launch_offspring_as<21, 2>(R, s);
        else
            launch_offspring_as<21, 1>(R, s);
    } else {
        launch_offspring_as<0, -1>(R, s);
    }
    if (R.osplit > 1 && R.problem != kPolicy)
        k_offspring_finish<<<(unsigned)((R.N + 255) / 256), 256, 0, s>>>(R);
    return hipGetLastError();
}

}  // namespace rvea
