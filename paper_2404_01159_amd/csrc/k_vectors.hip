// k_vectors.hip -- reference-vector kernels.
//   k_lattice   V_0 (Alg. 2 input): row j of the Das-Dennis simplex lattice
//               with H divisions, found by unranking the j-th (m-1)-subset
//               of {1..H+m-1} in lexicographic order (parts a_i = c_i -
//               c_{i-1} - 1, w = a/H), normalised to unit length
//   (gamma of Eq. 5 runs through the association kernels, k_select.hip)
//   k_adapt_v   Alg. 2's update of V (rule of the cited RVEA): V_j = V0_j o r /
//               |V0_j o r| with r the survivors' per-objective range; left
//               unchanged if some range is not positive and finite
//   k_vec_aux   float copy of V (padded rows) and row norms
#include "rvea_dev.h"
#include "rvea_index.h"
#include "rvea_internal.h"

namespace rvea {

__device__ __forceinline__ uint64_t binom(int64_t n, int k)
{
    if (k < 0 || n < k) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
    return r;
}

__device__ __forceinline__ void write_aux(const RunView &R, int64_t j, const double *v)
{
    const int stride = R.m <= 4 ? 4 : 8;
    double n2 = v[0] * v[0];
    for (int k = 1; k < R.m; ++k) n2 = fma(v[k], v[k], n2);
    R.vn[j] = sqrt(n2);
    for (int k = 0; k < stride; ++k) R.V32[j * stride + k] = k < R.m ? (float)v[k] : 0.0f;
}

__global__ void k_lattice(RunView R, int H)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= R.K) return;
    const int m = R.m, kk = m - 1;
    const int64_t n = (int64_t)H + m - 1;
    int64_t x = j;
    int64_t prev = 0;
    double w[kMaxM];
    for (int i = 0; i < kk; ++i) {
        // subsets whose next element lies in [prev+1, v]: by the hockey-stick
        // identity C(n-prev, r+1) - C(n-v, r+1); the next element is the
        // smallest v whose count exceeds x (binary search, O(log H) counts)
        const int r = kk - 1 - i;
        const uint64_t all = binom(n - prev, r + 1);
        const uint64_t T = all - (uint64_t)x;
        int64_t lo = prev + 1, hi = n - r;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (binom(n - mid, r + 1) < T)
                hi = mid;
            else
                lo = mid + 1;
        }
        const int64_t v = lo;
        x -= (int64_t)(all - binom(n - v + 1, r + 1));
        w[i] = (double)(v - prev - 1) / (double)H;
        prev = v;
    }
    w[m - 1] = (double)((int64_t)H + m - prev - 1) / (double)H;
    double n2 = w[0] * w[0];
    for (int k = 1; k < m; ++k) n2 = fma(w[k], w[k], n2);
    const double nrm = sqrt(n2);
    double v[kMaxM];
    for (int k = 0; k < m; ++k) {
        v[k] = w[k] / nrm;
        R.V0[j * m + k] = v[k];
        R.V[j * m + k] = v[k];
    }
    write_aux(R, j, v);
}

__global__ void k_vec_aux(RunView R)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= R.K) return;
    double v[kMaxM];
    for (int k = 0; k < R.m; ++k) v[k] = R.V[j * R.m + k];
    write_aux(R, j, v);
}

// check_due: decide on the device whether this generation adapts (batched
// runs advance in lockstep but joined at different generations)
__device__ __forceinline__ void adapt_v_body(const RunView &R, int64_t bx, bool check_due)
{
    const int64_t j = bx * 256 + threadIdx.x;
    double r[kMaxM];
    bool ok = !check_due || (*R.t_done % R.period) == 0;
    for (int k = 0; k < R.m && ok; ++k) {
        const uint32_t lo = R.rbits[k], hi = R.rbits[R.m + k];
        if (lo == 0xffffffffu) {
            ok = false;
            break;
        }
        r[k] = (double)ord_dec(hi) - (double)ord_dec(lo);
        ok = ok && r[k] > 0.0 && isfinite(r[k]);
    }
    if (j == 0) *R.vchanged = ok ? 1 : 0;
    if (j == 0 && ok && R.gr) {  // the index's scaling: r over its maximum, at least 1e-6
        double mx = r[0];
        for (int k = 1; k < R.m; ++k) mx = fmax(mx, r[k]);
        for (int k = 0; k < R.m; ++k) R.gr[k] = fmax(r[k] / mx, 1e-6);
    }
    if (!ok || j >= R.K) return;
    double w[kMaxM];
    for (int k = 0; k < R.m; ++k) w[k] = R.V0[j * R.m + k] * r[k];
    double n2 = w[0] * w[0];
    for (int k = 1; k < R.m; ++k) n2 = fma(w[k], w[k], n2);
    const double nrm = sqrt(n2);
    double v[kMaxM];
    for (int k = 0; k < R.m; ++k) {
        v[k] = w[k] / nrm;
        R.V[j * R.m + k] = v[k];
    }
    write_aux(R, j, v);
    if (R.gG > 0) {
        // the index rebuild's first step for this vector: its cell under the
        // new scaling (each thread forms the scaling as thread 0 stores it),
        // counted (the counts start at zero: the last build cleared them)
        double gr[kMaxM];
        double mx = r[0];
        for (int k = 1; k < R.m; ++k) mx = fmax(mx, r[k]);
        for (int k = 0; k < R.m; ++k) gr[k] = fmax(r[k] / mx, 1e-6);
        int c;
        if (R.m == 3) {
            c = cell_of(v[0], v[1], v[2], gr, R.gG);
            if (c < 0) c = 0;  // cannot happen for a nonzero vector >= 0
        } else {
            double u;
            c = line_cell_of(v[0], v[1], gr, R.gG, u);
        }
        R.gcell[j] = c;
        if (c >= 0) atomicAdd(&R.gcnt[c], 1);
        if (j == 0) {
            R.gtot[1] = 0;  // as the bucket pass sets them
            R.gtot[2] = 0;
        }
    }
}

__global__ void k_adapt_v(RunView R) { adapt_v_body(R, blockIdx.x, false); }

__global__ __launch_bounds__(256) void kb_adapt_v(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    adapt_v_body(runs[sp[s].run], blockIdx.x - sp[s].start, true);
}

// ------------------------------------------------------------- launchers
static unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_lattice(const RunView &R, hipStream_t s, int H)
{
    k_lattice<<<blocks(R.K, 256), 256, 0, s>>>(R, H);
    return hipGetLastError();
}

hipError_t launch_vec_aux(const RunView &R, hipStream_t s)
{
    k_vec_aux<<<blocks(R.K, 256), 256, 0, s>>>(R);
    return hipGetLastError();
}

hipError_t launch_batch_vectors(int phase, int cls, const RunView *runs, const Span *sp, int n,
                                int64_t blocks, hipStream_t s)
{
    (void)cls;
    if (phase != BP_ADAPT) return hipErrorInvalidValue;
    kb_adapt_v<<<dim3((unsigned)blocks), 256, 0, s>>>(runs, sp, n);
    return hipGetLastError();
}

// block counts and template classes of the batched phases
int batch_phase_class(int phase, const RunView &R)
{
    if (phase == BP_OFFSPRING && R.op != OP_GA) return operator_class(R);
    if (phase == BP_OFFSPRING)
        return offspring_segment(R.d, R.N) |
               (R.eta_c == 20.0 && R.eta_m == 20.0 ? kDefaultIndices : 0);
    if (phase == BP_ASSOC && R.gG > 0) return kIndexedClass | R.m;
    if (phase == BP_GRID_CELLS) return R.m;  // the grid's cells, or the line's gamma
    if (phase == BP_ASSOC || phase == BP_RERANK || phase == BP_GAMMA_ASSOC ||
        phase == BP_GAMMA_RERANK)
        return R.m;
    return 0;
}

int64_t batch_phase_nbx(int phase, const RunView &R)
{
    const int64_t rows = phase == BP_GAMMA_ASSOC ? R.K : R.M;
    return (rows + assoc_rows_per_block() - 1) / assoc_rows_per_block();
}

int64_t batch_phase_blocks(int phase, const RunView &R)
{
    if (phase >= BP_GRID_RANGES && phase <= BP_GRID_CELLS) return grid_phase_blocks(phase, R);
    if (phase == BP_ASSOC && R.gG > 0) return grid_phase_blocks(phase, R);
    if (phase == BP_RERANK && R.gG > 0) return 0;  // the indexed association ranks in full
    switch (phase) {
    case BP_PREP: return (R.K + R.N + 255) / 256;
    case BP_OFFSPRING: {
        if (R.op != OP_GA) return operator_blocks(R);
        const int S = offspring_segment(R.d, R.N);
        return ((R.N + 1) / 2 * R.osplit + (kOffBlock / S) - 1) / (kOffBlock / S);
    }
    case BP_OFFSPRING_FIN:  // only runs whose pairs are split over segments
        return R.osplit > 1 ? (R.N + 255) / 256 : 0;
    case BP_ASSOC:
    case BP_GAMMA_ASSOC: return batch_phase_nbx(phase, R) * R.KC;
    case BP_RERANK: return (R.M + rerank_rows_per_wave() - 1) / rerank_rows_per_wave();
    case BP_GAMMA_RERANK: return (R.K + rerank_rows_per_wave() - 1) / rerank_rows_per_wave();
    case BP_NEWPOP:
    case BP_ADAPT: return (R.K + 255) / 256;
    }
    return 0;
}

hipError_t launch_batch(int phase, int cls, const RunView *runs, const Span *sp, int n,
                        int64_t blocks, hipStream_t s)
{
    if (phase == BP_OFFSPRING && (cls & kOperatorClass))
        return launch_batch_operator(cls, runs, sp, n, blocks, s);
    if (phase <= BP_OFFSPRING_FIN) return launch_batch_gen(phase, cls, runs, sp, n, blocks, s);
    if (phase == BP_ADAPT) return launch_batch_vectors(phase, cls, runs, sp, n, blocks, s);
    if ((phase == BP_ASSOC && (cls & kIndexedClass)) ||
        (phase >= BP_GRID_RANGES && phase <= BP_GRID_CELLS))
        return launch_batch_grid(phase, cls, runs, sp, n, blocks, s);
    return launch_batch_select(phase, cls, runs, sp, n, blocks, s);
}

hipError_t launch_adapt(const RunView &R, hipStream_t s)
{
    k_adapt_v<<<blocks(R.K, 256), 256, 0, s>>>(R);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // with the index, its build computes gamma where it can prove the nearest
    // vector is among a vector's neighbours, and the full pass runs only when
    // some vector is left
    if (R.gG > 0) {
        e = launch_grid_rebuild(R, s);  // the adaptation counted the vectors
        if (e != hipSuccess) return e;
        return launch_gamma(R, s, 2);
    }
    return launch_gamma(R, s, 0);
}

}  // namespace rvea
