// k_ops.hip -- the other reproduction operators of the extensibility study
// (Sec. 4, Extensibility): DE/rand/1/bin, PSO with inertia weight, CSO and
// random reproduction, each in place of SBX + polynomial mutation, with the
// offspring's evaluation (Eq. 1) fused as in the genetic offspring kernel.
// Selection (Alg. 1) and adaptation (Alg. 2) are unchanged.
//
// Updates (binary64 from the binary32 genes and velocities, each operation
// in the order written, rounded once to binary32):
//   DE   child o: target x_t, donors x_r1, x_r2, x_r3 (distinct from the
//        target and from each other when the population has four members
//        or more), forced gene j_rand; gene g takes clip(x_r1 + F (x_r2 -
//        x_r3)) when U_g < CR or g = j_rand, else the target's gene
//   PSO  child o: particle i and leader l; v' = w v_i + c (r (x_l - x_i)),
//        x' = clip(x_i + v'); the child carries v'
//   CSO  pair p: members a, b; the smaller objective sum wins (ties: the
//        lower slot); child p is the loser moved, v' = r1 v_l + r2 (x_w -
//        x_l), x' = clip(x_l + v'); child p + ceil(N/2) is the winner,
//        genes and velocity unchanged
//   RAND gene g = lb + (ub - lb) U_g
// Draws (Philox4x32-10 under the run seed, t the generation): member draws
// of unit u (a child, or a CSO pair) are the words W_0, W_1, ... of counters
// (i/4, u, t, TAG_OPSEL), an index below n being (W n) >> 32 into the valid
// slots in ascending order; DE's j_rand is W_1 below d and its donors come
// from W_2 on (a candidate equal to an accepted index is redrawn, up to
// W_65; from W_66 on every candidate is accepted).  Per-gene uniforms U are
// the top 24 bits of word g % 4 of counter (g/4, u, t, TAG_OPGENE); CSO
// takes r1, r2 from words 0 and 1 of counter (g, p, t, TAG_OPGENE).
//
// Velocities live in a pool of K+N rows indexed like the gene rows, so a
// survivor keeps its velocity with its row and no copy is needed.
#include "rvea_dev.h"
#include "rvea_problems.h"
#include "rvea_internal.h"

namespace rvea {

__device__ __forceinline__ uint32_t word_of(const W4 &w, int k)
{
    return k == 0 ? w.w[0] : k == 1 ? w.w[1] : k == 2 ? w.w[2] : w.w[3];
}

// DE's member draws of child o: indices (into the valid-slot list) of the
// target and the three donors, and the forced gene
struct DeDraws {
    uint32_t tgt, r1, r2, r3;
    int jr;
};

__device__ __forceinline__ DeDraws de_draws(const RunView &R, uint32_t o, uint32_t t, uint32_t nv)
{
    W4 w = draw(R, 0u, o, t, TAG_OPSEL);
    DeDraws D;
    D.tgt = below(w.w[0], nv);
    D.jr = (int)below(w.w[1], (uint32_t)R.d);
    const bool distinct = nv >= 4;
    int n = 0;
    D.r1 = D.r2 = D.r3 = 0;
    for (int i = 2; n < 3; ++i) {  // ends by i = 68 (from 66 on every candidate is taken)
        if ((i & 3) == 0) w = draw(R, (uint32_t)(i >> 2), o, t, TAG_OPSEL);
        const uint32_t c = below(word_of(w, i & 3), nv);
        bool ok = true;
        if (distinct && i < 66)
            ok = c != D.tgt && (n < 1 || c != D.r1) && (n < 2 || c != D.r2);
        if (ok) {
            if (n == 0) D.r1 = c;
            else if (n == 1) D.r2 = c;
            else D.r3 = c;
            ++n;
        }
    }
    return D;
}

// distance terms of a quad's genes (positions and padding count 0), summed
// in single precision as in the genetic offspring kernel
__device__ __forceinline__ double quad_terms(const RunView &R, int g0, const float (&y)[4])
{
    float tt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int g = g0 + k;
        tt[k] = (g >= R.m - 1 && g < R.d) ? dist_term(R.problem, y[k]) : 0.0f;
    }
    return (double)((tt[0] + tt[1]) + (tt[2] + tt[3]));
}

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void st4(float *p, const float (&y)[4])
{
    *reinterpret_cast<float4 *>(p) = make_float4(y[0], y[1], y[2], y[3]);
}

// One segment of S lanes per unit (a child; a pair for CSO), one quad of
// genes per lane and step; workgroups of one wavefront.
template <int S, int OP>
__device__ __forceinline__ void operator_body(const RunView &R, int64_t bx)
{
    constexpr int SEGS = kOffBlock / S;
    const int seg = threadIdx.x / S, lane = threadIdx.x % S;
    const int64_t P = (R.N + 1) / 2;
    const int64_t units = OP == OP_CSO ? P : R.N;
    const int64_t u = bx * SEGS + seg;
    const bool active = u < units;
    const int64_t pop = *R.t_done;  // the parents' population
    const uint32_t t = (uint32_t)(pop + 1);
    float *Fm = fm_of(R, pop);
    const int64_t o1 = u, o2 = u + P;  // CSO: the loser's child and the winner's copy
    const bool has2 = OP == OP_CSO && o2 < R.N;
    const uint32_t nv = (uint32_t)*R.nvalid;
    if (nv == 0) {  // no member left: the offspring are empty, as for the genetic operators
        if (active && lane == 0) {
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
    const int2 *vs = reinterpret_cast<const int2 *>(R.vs);
    const bool evaluate = R.problem != kPolicy;  // the rollouts evaluate policy genes
    const int Q = (R.d + 3) / 4;
    const double lb = R.lb, ub = R.ub;
    double g1 = 0.0, g2 = 0.0;
    float pv1[4] = {0.f, 0.f, 0.f, 0.f}, pv2[4] = {0.f, 0.f, 0.f, 0.f};
    int32_t pa = -1, pb = -1;  // reported pair (CSO: winner, loser)

    if (active) {
        float *c1 = R.X + (int64_t)R.off_row[o1] * R.ld;
        if constexpr (OP == OP_DE) {
            const DeDraws D = de_draws(R, (uint32_t)o1, t, nv);
            const float *xt = R.X + (int64_t)vs[D.tgt].y * R.ld;
            const float *x1 = R.X + (int64_t)vs[D.r1].y * R.ld;
            const float *x2 = R.X + (int64_t)vs[D.r2].y * R.ld;
            const float *x3 = R.X + (int64_t)vs[D.r3].y * R.ld;
            const double F = R.op_a, CR = R.op_b;
            for (int q = lane; q < Q; q += S) {
                const W4 w = draw(R, (uint32_t)q, (uint32_t)o1, t, TAG_OPGENE);
                const float4 a = ld4(xt + 4 * q), b = ld4(x1 + 4 * q), c = ld4(x2 + 4 * q),
                             e = ld4(x3 + 4 * q);
                const float va[4] = {a.x, a.y, a.z, a.w}, vb[4] = {b.x, b.y, b.z, b.w};
                const float vc[4] = {c.x, c.y, c.z, c.w}, ve[4] = {e.x, e.y, e.z, e.w};
                float y[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bool take = unif24(w.w[k]) < CR || 4 * q + k == D.jr;
                    const double diff = (double)vc[k] - (double)ve[k];
                    const double step = F * diff;
                    y[k] = take ? (float)dclip((double)vb[k] + step, lb, ub) : va[k];
                }
                if (evaluate) g1 += quad_terms(R, 4 * q, y);
                if (q < 2) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) pv1[k] = y[k];
                }
                st4(c1 + 4 * q, y);
            }
        } else if constexpr (OP == OP_PSO) {
            const W4 ws = draw(R, 0u, (uint32_t)o1, t, TAG_OPSEL);
            const int32_t ri = vs[below(ws.w[0], nv)].y, rl = vs[below(ws.w[1], nv)].y;
            const float *xi = R.X + (int64_t)ri * R.ld, *xl = R.X + (int64_t)rl * R.ld;
            const float *vi = R.Vel + (int64_t)ri * R.ld;
            float *v1 = R.Vel + (int64_t)R.off_row[o1] * R.ld;
            const double wi = R.op_a, cc = R.op_b;
            for (int q = lane; q < Q; q += S) {
                const W4 w = draw(R, (uint32_t)q, (uint32_t)o1, t, TAG_OPGENE);
                const float4 a = ld4(xi + 4 * q), b = ld4(xl + 4 * q), c = ld4(vi + 4 * q);
                const float xa[4] = {a.x, a.y, a.z, a.w}, xb[4] = {b.x, b.y, b.z, b.w};
                const float vv[4] = {c.x, c.y, c.z, c.w};
                float y[4], nvel[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double r = unif24(w.w[k]);
                    const double diff = (double)xb[k] - (double)xa[k];
                    const double pull = cc * (r * diff);
                    const double vn = wi * (double)vv[k] + pull;
                    y[k] = (float)dclip((double)xa[k] + vn, lb, ub);
                    nvel[k] = (float)vn;
                }
                if (evaluate) g1 += quad_terms(R, 4 * q, y);
                if (q < 2) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) pv1[k] = y[k];
                }
                st4(c1 + 4 * q, y);
                st4(v1 + 4 * q, nvel);
            }
        } else if constexpr (OP == OP_CSO) {
            const W4 ws = draw(R, 0u, (uint32_t)o1, t, TAG_OPSEL);
            const int2 ea = vs[below(ws.w[0], nv)], eb = vs[below(ws.w[1], nv)];
            double fa = 0.0, fb = 0.0;
            for (int k = 0; k < R.m; ++k) {
                fa += (double)Fm[(int64_t)ea.x * R.m + k];
                fb += (double)Fm[(int64_t)eb.x * R.m + k];
            }
            const bool a_wins = fa < fb || (fa == fb && ea.x <= eb.x);
            const int2 win = a_wins ? ea : eb, los = a_wins ? eb : ea;
            pa = win.x;
            pb = los.x;
            const float *xw = R.X + (int64_t)win.y * R.ld, *xl = R.X + (int64_t)los.y * R.ld;
            const float *vw = R.Vel + (int64_t)win.y * R.ld, *vl = R.Vel + (int64_t)los.y * R.ld;
            float *v1 = R.Vel + (int64_t)R.off_row[o1] * R.ld;
            float *c2 = has2 ? R.X + (int64_t)R.off_row[o2] * R.ld : nullptr;
            float *v2 = has2 ? R.Vel + (int64_t)R.off_row[o2] * R.ld : nullptr;
            for (int q = lane; q < Q; q += S) {
                const float4 a = ld4(xw + 4 * q), b = ld4(xl + 4 * q), c = ld4(vl + 4 * q);
                const float xwq[4] = {a.x, a.y, a.z, a.w}, xlq[4] = {b.x, b.y, b.z, b.w};
                const float vlq[4] = {c.x, c.y, c.z, c.w};
                float y[4], nvel[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const W4 w = draw(R, (uint32_t)(4 * q + k), (uint32_t)o1, t, TAG_OPGENE);
                    const double r1 = unif24(w.w[0]), r2 = unif24(w.w[1]);
                    const double diff = (double)xwq[k] - (double)xlq[k];
                    const double vn = r1 * (double)vlq[k] + r2 * diff;
                    y[k] = (float)dclip((double)xlq[k] + vn, lb, ub);
                    nvel[k] = (float)vn;
                }
                if (evaluate) {
                    g1 += quad_terms(R, 4 * q, y);
                    if (has2) g2 += quad_terms(R, 4 * q, xwq);
                }
                if (q < 2) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        pv1[k] = y[k];
                        pv2[k] = xwq[k];
                    }
                }
                st4(c1 + 4 * q, y);
                st4(v1 + 4 * q, nvel);
                if (has2) {
                    *reinterpret_cast<float4 *>(c2 + 4 * q) = a;
                    *reinterpret_cast<float4 *>(v2 + 4 * q) = ld4(vw + 4 * q);
                }
            }
        } else {  // OP_RAND
            const double span = ub - lb;
            for (int q = lane; q < Q; q += S) {
                const W4 w = draw(R, (uint32_t)q, (uint32_t)o1, t, TAG_OPGENE);
                float y[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double scaled = span * unif24(w.w[k]);
                    y[k] = (float)(lb + scaled);
                }
                if (evaluate) g1 += quad_terms(R, 4 * q, y);
                if (q < 2) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) pv1[k] = y[k];
                }
                st4(c1 + 4 * q, y);
            }
        }
    }
    // every lane from here on (segment sums, lane reads, the wave minima)
    if (evaluate) {
        g1 = seg_sum<S>(g1);
        if (OP == OP_CSO) g2 = seg_sum<S>(g2);
        float pos1[kMaxM], pos2[kMaxM];
#pragma unroll
        for (int k = 0; k < kMaxM - 1; ++k) {
            pos1[k] = __shfl(pv1[k & 3], k >> 2, S);
            pos2[k] = __shfl(pv2[k & 3], k >> 2, S);
        }
        pos1[kMaxM - 1] = pos2[kMaxM - 1] = 0.f;
        // child 1 on the segment's lane 0, CSO's copy on lane 1
        const bool mine = active && (lane == 0 || (lane == 1 && has2));
        const int64_t row = R.K + (lane == 0 ? o1 : o2);
        float f[kMaxM] = {};
        if (mine) {
            finish_objectives(R.problem, R.m, R.d, lane == 0 ? pos1 : pos2, lane == 0 ? g1 : g2,
                              f);
            for (int k = 0; k < R.m; ++k) Fm[row * R.m + k] = f[k];
        }
        child_ideal(R, t, mine, row, f);
    }
    // the pair report (one entry per pair; DE, PSO and random draw none)
    if (active && lane == 0 && o1 < P) {
        R.parents[2 * o1] = pa;
        R.parents[2 * o1 + 1] = pb;
    }
}

template <int S, int OP>
__global__ __launch_bounds__(kOffBlock) void k_operator(RunView R)
{
    operator_body<S, OP>(R, blockIdx.x);
}

// batched: blockIdx.x decoded into (run, local block) through the span
// table; the runs of one launch share the operator and the segment width
template <int S, int OP>
__global__ __launch_bounds__(kOffBlock) void kb_operator(const RunView *runs, const Span *sp,
                                                         int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    operator_body<S, OP>(runs[sp[s].run], blockIdx.x - sp[s].start);
}

template <int OP>
static void launch_operator_as(const RunView &R, hipStream_t s)
{
    const int S = pick_segment(R.d);
    const int64_t units = OP == OP_CSO ? (R.N + 1) / 2 : R.N;
    const dim3 g((unsigned)((units + kOffBlock / S - 1) / (kOffBlock / S)));
    switch (S) {
    case 4: k_operator<4, OP><<<g, kOffBlock, 0, s>>>(R); break;
    case 8: k_operator<8, OP><<<g, kOffBlock, 0, s>>>(R); break;
    case 16: k_operator<16, OP><<<g, kOffBlock, 0, s>>>(R); break;
    case 32: k_operator<32, OP><<<g, kOffBlock, 0, s>>>(R); break;
    default: k_operator<64, OP><<<g, kOffBlock, 0, s>>>(R); break;
    }
}

template <int OP>
static void launch_batch_operator_as(int S, const RunView *runs, const Span *sp, int n,
                                     const dim3 g, hipStream_t s)
{
    switch (S) {
    case 4: kb_operator<4, OP><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;
    case 8: kb_operator<8, OP><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;
    case 16: kb_operator<16, OP><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;
    case 32: kb_operator<32, OP><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;
    default: kb_operator<64, OP><<<g, kOffBlock, 0, s>>>(runs, sp, n); break;
    }
}

int operator_class(const RunView &R)
{
    return kOperatorClass | (R.op << 8) | pick_segment(R.d);
}

int64_t operator_blocks(const RunView &R)
{
    const int S = pick_segment(R.d);
    const int64_t units = R.op == OP_CSO ? (R.N + 1) / 2 : R.N;
    return (units + kOffBlock / S - 1) / (kOffBlock / S);
}

hipError_t launch_batch_operator(int cls, const RunView *runs, const Span *sp, int n,
                                 int64_t blocks, hipStream_t s)
{
    const dim3 g((unsigned)blocks);
    const int S = cls & kSegMask;
    switch ((cls >> 8) & 0xff) {
    case OP_DE: launch_batch_operator_as<OP_DE>(S, runs, sp, n, g, s); break;
    case OP_PSO: launch_batch_operator_as<OP_PSO>(S, runs, sp, n, g, s); break;
    case OP_CSO: launch_batch_operator_as<OP_CSO>(S, runs, sp, n, g, s); break;
    case OP_RAND: launch_batch_operator_as<OP_RAND>(S, runs, sp, n, g, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_operator(const RunView &R, hipStream_t s)
{
    switch (R.op) {
    case OP_DE: launch_operator_as<OP_DE>(R, s); break;
    case OP_PSO: launch_operator_as<OP_PSO>(R, s); break;
    case OP_CSO: launch_operator_as<OP_CSO>(R, s); break;
    case OP_RAND: launch_operator_as<OP_RAND>(R, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace rvea
