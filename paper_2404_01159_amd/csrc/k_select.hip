// k_select.hip -- reference-vector guided selection (Alg. 1; Eqs. 2, 4, 5).
//
// The paper forms the n x r angle tensor, masks it per column and takes
// column-wise APD argmins.  Here the 2N x K cosine matrix is never stored:
//   k_ideal   z* = column minima over the rows that take part (Alg. 1 l.3)
//   k_assoc   single-precision pass over (row, vector) pairs: V tiles of 32
//             vectors sit in LDS and are broadcast to every lane; each lane
//             holds RR rows of f' = F - z* and keeps, per vector chunk, the
//             running maximum of f'.v and a bit mask of the tiles whose
//             maximum came within 2*eps of it (eps bounds the float error of
//             one dot product); nothing per pair is written
//   k_rerank  double precision over the candidate tiles only: cosine
//             f'.v / (|f'| |v|) written as an fma chain, argmax with lowest
//             index on ties (Eq. 2), theta = acos, APD of Eq. 4 with the
//             vector's gamma (Eq. 5); per-vector minimum APD by 64-bit atomic
//             min on the (non-negative) double's bit pattern
//   k_surv    the lowest row index attaining that minimum (Alg. 1 l.15)
//   k_newpop / k_commit  slot j <- its survivor's gene row and objectives
// Every cross-workgroup combination is an order-free min, so the result
// does not depend on scheduling.
#include "rvea_dev.h"
#include "rvea_internal.h"

namespace rvea {

__global__ void k_sel_reset(RunView R)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < R.K) {
        R.key[j] = ~0ull;
        R.surv[j] = 0x7fffffff;
    }
    if (j < R.m) {
        R.zbits[j] = 0xffffffffu;     // encodes the largest value
        R.rbits[j] = 0xffffffffu;     // survivor minimum
        R.rbits[R.m + j] = 0u;        // survivor maximum
    }
}

// rows that take part: valid parent slots and all offspring with finite F
__global__ void k_ideal(RunView R)
{
    __shared__ uint32_t smin[kMaxM];
    if (threadIdx.x < kMaxM) smin[threadIdx.x] = 0xffffffffu;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < R.M) {
        bool ok = i >= R.K || R.valid[i];
        bool fin = true;
        for (int k = 0; k < R.m; ++k) fin = fin && isfinite(R.Fm[i * R.m + k]);
        if (ok && !fin) atomicAdd(&R.counters[0], 1ull);
        ok = ok && fin;
        R.mvalid[i] = ok ? 1 : 0;
        if (ok)
            for (int k = 0; k < R.m; ++k) atomicMin(&smin[k], ord_enc(R.Fm[i * R.m + k]));
    }
    __syncthreads();
    if (threadIdx.x < R.m && smin[threadIdx.x] != 0xffffffffu)
        atomicMin(&R.zbits[threadIdx.x], smin[threadIdx.x]);
}

// 2*eps for a row of norm nrm: |f'.v (float) - f'.v (exact)| <= 6u |f'| for
// unit v with u = 2^-24 (rounding of f', of v and three operations); the
// margin used is 16u per side.
__device__ __forceinline__ float two_eps(float nrm) { return 0x1p-19f * nrm; }

template <int MD>
__device__ __forceinline__ float dotf(const float *f, const float4 *v)
{
    float s = f[0] * v[0].x;
    if (MD > 1) s = fmaf(f[1], v[0].y, s);
    if (MD > 2) s = fmaf(f[2], v[0].z, s);
    if (MD > 3) s = fmaf(f[3], v[0].w, s);
    if (MD > 4) s = fmaf(f[4], v[1].x, s);
    if (MD > 5) s = fmaf(f[5], v[1].y, s);
    if (MD > 6) s = fmaf(f[6], v[1].z, s);
    if (MD > 7) s = fmaf(f[7], v[1].w, s);
    return s;
}

template <int MD, int RR>
__global__ __launch_bounds__(256) void k_assoc(RunView R)
{
    constexpr int NV4 = MD <= 4 ? 1 : 2;  // float4 per vector
    __shared__ float4 sv[1024 * NV4];
    const int c = blockIdx.y;
    const int64_t j0 = (int64_t)c * R.CS;
    const int64_t left = R.K - j0;
    const int nvec = (int)(left < R.CS ? left : R.CS);
    const int ntile = (nvec + kTile - 1) / kTile;
    const float4 pad = make_float4(-1e30f, -1e30f, -1e30f, -1e30f);
    const float4 *Vg = reinterpret_cast<const float4 *>(R.V32);
    for (int idx = threadIdx.x; idx < ntile * kTile * NV4; idx += 256) {
        const int v = idx / NV4;
        sv[idx] = v < nvec ? Vg[(j0 + v) * NV4 + (idx % NV4)] : pad;
    }

    float z[MD];
#pragma unroll
    for (int k = 0; k < MD; ++k) z[k] = ord_dec(R.zbits[k]);
    float f[RR][MD], e2[RR], cm[RR];
    uint32_t mk[RR];
    int64_t rows[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int64_t i = (int64_t)blockIdx.x * (256 * RR) + r * 256 + threadIdx.x;
        rows[r] = i;
        const bool ok = i < R.M && R.mvalid[i];
        float n2 = 0.f;
#pragma unroll
        for (int k = 0; k < MD; ++k) {
            f[r][k] = ok ? R.Fm[i * MD + k] - z[k] : 0.f;
            n2 = fmaf(f[r][k], f[r][k], n2);
        }
        e2[r] = two_eps(sqrtf(n2));
        cm[r] = -INFINITY;
        mk[r] = 0u;
    }
    __syncthreads();

    for (int tl = 0; tl < ntile; ++tl) {
        float tm[RR];
#pragma unroll
        for (int r = 0; r < RR; ++r) tm[r] = -INFINITY;
        const float4 *tv = sv + tl * kTile * NV4;
#pragma unroll 4
        for (int jj = 0; jj < kTile; jj += 2) {
            float4 va[NV4], vb[NV4];
#pragma unroll
            for (int q = 0; q < NV4; ++q) {
                va[q] = tv[jj * NV4 + q];
                vb[q] = tv[(jj + 1) * NV4 + q];
            }
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                const float sa = dotf<MD>(f[r], va);
                const float sb = dotf<MD>(f[r], vb);
                tm[r] = fmaxf(tm[r], fmaxf(sa, sb));
            }
        }
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const uint32_t bit = 1u << tl;
            if (tm[r] > cm[r] + e2[r]) {
                cm[r] = tm[r];
                mk[r] = bit;
            } else if (tm[r] >= cm[r] - e2[r]) {
                mk[r] |= bit;
                cm[r] = fmaxf(cm[r], tm[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int64_t i = rows[r];
        if (i < R.M) {
            R.pmax[(int64_t)c * R.M + i] = cm[r];
            R.pmask[(int64_t)c * R.M + i] = mk[r];
        }
    }
}

template <int MD>
__device__ __forceinline__ double dotd(const double *a, const double *b)
{
    double s = a[0] * b[0];
#pragma unroll
    for (int k = 1; k < MD; ++k) s = fma(a[k], b[k], s);
    return s;
}

template <int MD>
__global__ __launch_bounds__(256) void k_rerank(RunView R)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R.M) return;
    if (!R.mvalid[i]) {
        R.assoc[i] = -1;
        R.apd[i] = INFINITY;
        return;
    }
    const double tcur = (double)(*R.t_done + 1);
    const double pen = (double)MD * pow(tcur / (double)R.t_max, R.alpha);
    double f[MD];
    float f32[MD];
    float n2f = 0.f;
#pragma unroll
    for (int k = 0; k < MD; ++k) {
        const float zk = ord_dec(R.zbits[k]);
        const float Fk = R.Fm[i * MD + k];
        f[k] = (double)Fk - (double)zk;
        f32[k] = Fk - zk;
        n2f = fmaf(f32[k], f32[k], n2f);
    }
    double n2 = f[0] * f[0];
#pragma unroll
    for (int k = 1; k < MD; ++k) n2 = fma(f[k], f[k], n2);
    const double nrm = sqrt(n2);
    if (nrm == 0.0) {
        R.assoc[i] = 0;
        R.apd[i] = 0.0;
        atomicMin(&R.key[0], 0ull);
        return;
    }
    const float e2 = two_eps(sqrtf(n2f));
    float gmax = -INFINITY;
    for (int c = 0; c < R.KC; ++c) gmax = fmaxf(gmax, R.pmax[(int64_t)c * R.M + i]);
    const float thr = gmax - e2;
    double best = -INFINITY;
    int64_t bj = -1;
    for (int c = 0; c < R.KC; ++c) {
        if (!(R.pmax[(int64_t)c * R.M + i] >= thr)) continue;
        uint32_t mk = R.pmask[(int64_t)c * R.M + i];
        while (mk) {
            const int tl = __ffs(mk) - 1;
            mk &= mk - 1;
            const int64_t jlo = (int64_t)c * R.CS + (int64_t)tl * kTile;
            const int64_t jhi = jlo + kTile < R.K ? jlo + kTile : R.K;
            for (int64_t j = jlo; j < jhi; ++j) {
                const double cv = dotd<MD>(f, R.V + j * MD) / (nrm * R.vn[j]);
                if (cv > best) {
                    best = cv;
                    bj = j;
                }
            }
        }
    }
    if (bj < 0) {  // no candidate survived (non-finite float pass): scan everything
        atomicAdd(&R.counters[1], 1ull);
        for (int64_t j = 0; j < R.K; ++j) {
            const double cv = dotd<MD>(f, R.V + j * MD) / (nrm * R.vn[j]);
            if (cv > best) {
                best = cv;
                bj = j;
            }
        }
        if (bj < 0) bj = 0;
    }
    const double cc = best > 1.0 ? 1.0 : (best < -1.0 ? -1.0 : best);
    const double th = acos(cc);
    const double a = (1.0 + pen * th / R.gamma[bj]) * nrm;
    R.assoc[i] = (int32_t)bj;
    R.apd[i] = a;
    atomicMin(&R.key[bj], (unsigned long long)__double_as_longlong(a));
}

__global__ void k_surv(RunView R)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R.M) return;
    const int32_t j = R.assoc[i];
    if (j < 0) return;
    if ((unsigned long long)__double_as_longlong(R.apd[i]) == R.key[j])
        atomicMin(&R.surv[j], (int32_t)i);
}

__global__ void k_newpop(RunView R)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= R.K) return;
    const int32_t s = R.surv[j];
    if (s == 0x7fffffff) {
        R.surv[j] = -1;
        R.valid_n[j] = 0;
        R.row_n[j] = R.slot_row[j];
        for (int k = 0; k < R.m; ++k) R.Fn[j * R.m + k] = __int_as_float(0x7fc00000);
        return;
    }
    R.valid_n[j] = 1;
    R.row_n[j] = s < R.K ? R.slot_row[s] : R.off_row[s - R.K];
    for (int k = 0; k < R.m; ++k) R.Fn[j * R.m + k] = R.Fm[(int64_t)s * R.m + k];
}

// commit the new population and count the generation; also reduce the
// survivors' per-objective extremes for a possible adaptation
__global__ void k_commit(RunView R)
{
    __shared__ uint32_t smin[kMaxM], smax[kMaxM];
    if (threadIdx.x < kMaxM) {
        smin[threadIdx.x] = 0xffffffffu;
        smax[threadIdx.x] = 0u;
    }
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < R.K) {
        const uint8_t v = R.valid_n[j];
        R.valid[j] = v;
        R.slot_row[j] = R.row_n[j];
        for (int k = 0; k < R.m; ++k) {
            const float x = R.Fn[j * R.m + k];
            R.Fm[j * R.m + k] = x;
            if (v) {
                atomicMin(&smin[k], ord_enc(x));
                atomicMax(&smax[k], ord_enc(x));
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < R.m) {
        if (smin[threadIdx.x] != 0xffffffffu) atomicMin(&R.rbits[threadIdx.x], smin[threadIdx.x]);
        atomicMax(&R.rbits[R.m + threadIdx.x], smax[threadIdx.x]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *R.t_done += 1;
}

// ------------------------------------------------------------- launchers
static unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_select_front(const RunView &R, hipStream_t s)
{
    const int64_t n = R.K > R.m ? R.K : R.m;
    k_sel_reset<<<blocks(n, 256), 256, 0, s>>>(R);
    k_ideal<<<blocks(R.M, 256), 256, 0, s>>>(R);
    return hipGetLastError();
}

#define RVEA_M_DISPATCH(MVAL, CALL)                                                          \
    switch (MVAL) {                                                                          \
    case 2: CALL(2); break;                                                                  \
    case 3: CALL(3); break;                                                                  \
    case 4: CALL(4); break;                                                                  \
    case 5: CALL(5); break;                                                                  \
    case 6: CALL(6); break;                                                                  \
    case 7: CALL(7); break;                                                                  \
    default: CALL(8); break;                                                                 \
    }

hipError_t launch_assoc(const RunView &R, hipStream_t s)
{
    constexpr int RR = 4;
    const dim3 grid(blocks(R.M, 256 * RR), (unsigned)R.KC);
#define RVEA_ASSOC(MV) k_assoc<MV, RR><<<grid, 256, 0, s>>>(R)
    RVEA_M_DISPATCH(R.m, RVEA_ASSOC);
#undef RVEA_ASSOC
    return hipGetLastError();
}

hipError_t launch_rerank(const RunView &R, hipStream_t s)
{
#define RVEA_RERANK(MV) k_rerank<MV><<<blocks(R.M, 256), 256, 0, s>>>(R)
    RVEA_M_DISPATCH(R.m, RVEA_RERANK);
#undef RVEA_RERANK
    return hipGetLastError();
}

hipError_t launch_select_back(const RunView &R, hipStream_t s)
{
    k_surv<<<blocks(R.M, 256), 256, 0, s>>>(R);
    k_newpop<<<blocks(R.K, 256), 256, 0, s>>>(R);
    k_commit<<<blocks(R.K, 256), 256, 0, s>>>(R);
    return hipGetLastError();
}

int assoc_rows_per_block() { return 256 * 4; }

}  // namespace rvea
