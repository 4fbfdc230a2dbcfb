// k_select.hip -- reference-vector guided selection (Alg. 1; Eqs. 2, 4, 5).
//
// The paper forms the n x r angle tensor, masks it per column and takes
// column-wise APD argmins.  Here the 2N x K cosine matrix is never stored:
// (z*, the column minima over the rows that take part (Alg. 1), is reduced
// where the rows are produced: parents in k_prep, children in k_offspring
// or k_rollout.)
//   k_assoc   single-precision pass over (row, vector) pairs: V tiles of 32
//             vectors sit in LDS and are broadcast to every lane; each lane
//             holds RR rows of f' = F - z* and keeps, per vector chunk, the
//             running maximum of f'.v and a bit mask of the tiles whose
//             maximum came within 2*eps of it (eps bounds the float error of
//             one dot product); nothing per pair is written
//   k_rerank  double precision over the candidate tiles only: cosine
//             f'.v / (|f'| |v|) written as an fma chain, argmax with lowest
//             index on ties (Eq. 2), theta = acos, APD of Eq. 4 with the
//             vector's gamma (Eq. 5); per vector the minimum of (APD, row)
//             by one 64-bit atomic min on a packed word (the APD's bit
//             pattern above the row index), so the survivor (Alg. 1's
//             per-vector argmin, lowest row on ties) needs no second pass
//   k_newpop  slot j <- its survivor's gene row and objectives, written into
//             the other buffer of the population pair (no copy-back); also
//             the next generation's row stamps, block counts and resets
// Every cross-workgroup combination is an order-free min, so the result
// does not depend on scheduling.
#include <algorithm>

#include "rvea_dev.h"
#include "rvea_internal.h"

namespace rvea {

// 2*eps for a row of norm nrm: |f'.v (float) - f'.v (exact)| <= 6u |f'| for
// unit v with u = 2^-24 (rounding of f', of v and three operations); the
// margin used is 16u per side.
__device__ __forceinline__ float two_eps(float nrm) { return 0x1p-19f * nrm; }

// Gamma pass (rows are the unit vectors themselves): the single-precision
// score is minus the squared distance |v_i - v_j|^2 = 2 - 2 cos, whose error
// scales with the distance, so that nearly parallel vectors (far below the
// resolution of a binary32 cosine near 1) stay separable.  With v rounded to
// binary32 (2^-24 per component), the per-component differences off by at
// most 3 * 2^-24 and an fma chain of m <= 8 squares, a score at squared
// distance S is off by at most 2^-24 (17 sqrt(S) + 8 S) + 2^-42; 2 eps doubles
// it and adds a factor 2 margin.
__device__ __forceinline__ float two_eps_dist(float S)
{
    return 0x1p-22f * (17.0f * sqrtf(S) + 8.0f * S) + 0x1p-40f;
}

// -|a - v|^2 over MD components
template <int MD>
__device__ __forceinline__ float negdist(const float *a, const float4 *v)
{
    float t = a[0] - v[0].x;
    float s = t * t;
    if (MD > 1) { t = a[1] - v[0].y; s = fmaf(t, t, s); }
    if (MD > 2) { t = a[2] - v[0].z; s = fmaf(t, t, s); }
    if (MD > 3) { t = a[3] - v[0].w; s = fmaf(t, t, s); }
    if (MD > 4) { t = a[4] - v[1].x; s = fmaf(t, t, s); }
    if (MD > 5) { t = a[5] - v[1].y; s = fmaf(t, t, s); }
    if (MD > 6) { t = a[6] - v[1].z; s = fmaf(t, t, s); }
    if (MD > 7) { t = a[7] - v[1].w; s = fmaf(t, t, s); }
    return -s;
}

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

// GAMMA = false: rows are the merged objective rows f' = F - z*.
// GAMMA = true:  rows are the reference vectors themselves (Eq. 5), with the
// pair (j, j) excluded.
template <int MD, int RR, bool GAMMA>
__device__ __forceinline__ void assoc_body(const RunView &R, int64_t bx, int c, int gate)
{
    // gamma pass, uniform exits: gate 1 always runs; gate 0 runs when the
    // vectors changed; gate 2 also needs the index to have asked for it
    if (GAMMA && gate != 1 && (*R.vchanged == 0 || (gate == 2 && R.gtot[1] == 0))) return;
    constexpr int NV4 = MD <= 4 ? 1 : 2;  // float4 per vector
    __shared__ float4 sv[1024 * NV4];
    const int64_t j0 = (int64_t)c * R.CS;
    const int64_t left = R.K - j0;
    const int nvec = (int)(left < R.CS ? left : R.CS);
    const int ntile = (nvec + kTile - 1) / kTile;
    const float4 pad = make_float4(-1e30f, -1e30f, -1e30f, -1e30f);
    const float4 *Vg = reinterpret_cast<const float4 *>(R.V32);
    for (int idx = threadIdx.x; idx < ntile * kTile * NV4; idx += 256) {
        const int v = idx / NV4;
        if (v < nvec)
            sv[idx] = Vg[(j0 + v) * NV4 + (idx % NV4)];
        else
            sv[idx] = pad;
    }
    const int64_t nrows = GAMMA ? R.K : R.M;

    float z[MD];
    const uint32_t *zb = zbuf(R, *R.t_done + 1);
    const float *Fm = fm_of(R, *R.t_done);
#pragma unroll
    for (int k = 0; k < MD; ++k) z[k] = GAMMA ? 0.f : ord_dec(zb[k]);
    float f[RR][MD], e2[RR], cm[RR];
    uint32_t mk[RR];
    int64_t rows[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int64_t i = bx * (256 * RR) + r * 256 + threadIdx.x;
        rows[r] = i;
        // the row's values load beside its take-part flag, not after it
        float fr[MD];
#pragma unroll
        for (int k = 0; k < MD; ++k)
            fr[k] = i < nrows ? (GAMMA ? R.V32[i * (NV4 * 4) + k] : Fm[i * MD + k]) : 0.f;
        const bool ok = i < nrows && (GAMMA || R.mvalid[i]);
        float n2 = 0.f;
#pragma unroll
        for (int k = 0; k < MD; ++k) {
            f[r][k] = ok ? (GAMMA ? fr[k] : fr[k] - z[k]) : 0.f;
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
        const int64_t jt = j0 + (int64_t)tl * kTile;
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
                float sa = GAMMA ? negdist<MD>(f[r], va) : dotf<MD>(f[r], va);
                float sb = GAMMA ? negdist<MD>(f[r], vb) : dotf<MD>(f[r], vb);
                if (GAMMA) {
                    sa = rows[r] == jt + jj ? -INFINITY : sa;
                    sb = rows[r] == jt + jj + 1 ? -INFINITY : sb;
                }
                tm[r] = fmaxf(tm[r], fmaxf(sa, sb));
            }
        }
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            const uint32_t bit = 1u << tl;
            // gamma: the margin of the current best squared distance (none
            // before the first score; it only shrinks as the best improves)
            const float e = !GAMMA ? e2[r] : (cm[r] == -INFINITY ? 0.f : two_eps_dist(-cm[r]));
            // branch-free: a new maximum by more than 2 eps restarts the mask
            const bool up = tm[r] > cm[r] + e, near = tm[r] >= cm[r] - e;
            mk[r] = up ? bit : (near ? (mk[r] | bit) : mk[r]);
            cm[r] = near ? fmaxf(cm[r], tm[r]) : cm[r];
        }
    }
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int64_t i = rows[r];
        if (i < nrows) {
            R.pmax[(int64_t)c * R.M + i] = cm[r];
            R.pmask[(int64_t)c * R.M + i] = mk[r];
        }
    }
}

// maximum / sum over an aligned group of N adjacent lanes (N = 4, 8 or 16,
// every lane active), by the pairings of partner32
template <int N>
__device__ __forceinline__ float group_max(float v)
{
    v = fmaxf(v, __int_as_float(partner32<0>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(partner32<1>(__float_as_int(v))));
    if constexpr (N >= 8) v = fmaxf(v, __int_as_float(partner32<2>(__float_as_int(v))));
    if constexpr (N >= 16) v = fmaxf(v, __int_as_float(partner32<3>(__float_as_int(v))));
    return v;
}
template <int N>
__device__ __forceinline__ int group_sum(int v)
{
    v += partner32<0>(v);
    v += partner32<1>(v);
    if constexpr (N >= 8) v += partner32<2>(v);
    if constexpr (N >= 16) v += partner32<3>(v);
    return v;
}

// one level of the best-cosine reduction (largest value, lowest index on
// ties; the item's gamma travels with it; duplicates are or-ed)
template <int L, bool GAMMA>
__device__ __forceinline__ void best_level(double &best, int64_t &bj, double &gam, int &dup)
{
    const double ob = partner32<L>(best);
    const int64_t oj = partner32<L>(bj);
    double og = 0.0;
    if (!GAMMA) og = partner32<L>(gam);
    dup |= partner32<L>(dup);
    if (ob > best || (ob == best && oj < bj)) {
        best = ob;
        bj = oj;
        gam = og;
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

// Re-rank: one 64-lane wave per 16 rows, in five phases.
//   1. four lanes per row split the row's vector chunks: maximum of the chunk
//      maxima (threshold gmax - 2 eps), then the tiles of the chunks above
//      the threshold become work items (row, first vector of the tile);
//   2. the wave walks the flattened (item, vector) space, one vector per
//      lane: binary64 cosine f.v / (|f| |v|) as an fma chain, then the best
//      value of each item with the lowest index over its 32 lanes;
//   3. one lane per row: the best of its items;
//   4. a row with more than kItems candidate tiles (crowded vectors that
//      binary32 cannot separate), beyond the wave's kWaveItems, or left
//      without a usable candidate is scanned in full by the whole wave
//      (counted);
//   5. one lane per row: angle, APD and the per-vector atomic minimum
//      (selection), or gamma (GAMMA: rows are the vectors, i != j, exactly
//      parallel vectors skipped).
constexpr int kItems = 64;   // candidate tiles per row
constexpr int kCache = 4;    // candidate chunks per lane kept in registers
constexpr int kBatchRows = 8;  // rows per wave of the batched launch
constexpr int kCand = 64;      // candidate vectors per wave after the binary32 prefilter

// kRows rows per wave (4, 8 or 16): fewer rows give more waves to hide the
// phases' memory latency on small populations, more rows less per-row
// overhead on large ones.
template <int MD, bool GAMMA, int kRows>
__device__ __forceinline__ void rerank_body(const RunView &R, int64_t bx, int gate)
{
    constexpr int kLanes = 64 / kRows;  // lanes per row in phase 1
    constexpr int kWaveItems = 12 * kRows < kItems ? kItems : 12 * kRows;  // tiles per wave
    // gamma pass, uniform exits: gate 1 always runs; gate 0 runs when the
    // vectors changed; gate 2 also needs the index to have asked for it
    if (GAMMA && gate != 1 && (*R.vchanged == 0 || (gate == 2 && R.gtot[1] == 0))) return;
    __shared__ double s_f[kRows][MD];
    __shared__ double s_nrm[kRows];
    __shared__ int s_state[kRows];  // 0 inactive, 1 items, 2 zero row, 3 full scan
    __shared__ int s_cnt[kRows], s_off[kRows];
    __shared__ int s_item[kWaveItems];  // row << 27 | first vector of the tile
    __shared__ double s_best[kWaveItems];
    __shared__ double s_gam[kWaveItems];  // gamma of the item's best vector (selection)
    __shared__ int s_bj[kWaveItems];
    __shared__ unsigned char s_dup[kWaveItems];
    // selection rows: the row's binary32 f' and threshold, and the candidate
    // vectors that pass the binary32 prefilter (row << 27 | vector), their
    // count per row and their binary64 cosines
    __shared__ float s_f32[kRows][MD];
    __shared__ float s_thr[kRows];
    __shared__ int s_rc[kRows];
    __shared__ int s_cand[kCand];
    __shared__ double s_cos[kCand];

    const int t = threadIdx.x;
    const int r = t / kLanes, sub = t % kLanes;
    const int64_t base = bx * kRows;
    const int64_t i = base + r;
    const int64_t nrows = GAMMA ? R.K : R.M;

    // ---- phase 1
    int state = 0, cnt = 0;
    float thr = 0.f;
    const bool act = i < nrows && (GAMMA || R.mvalid[i]);
    // this lane's chunk maxima and tile masks, the first kCache chunks read
    // together (one round trip; they do not depend on the row's objectives)
    float cmax[kCache];
    uint32_t cmask[kCache];
#pragma unroll
    for (int u = 0; u < kCache; ++u) {
        const int c = sub + u * kLanes;
        cmax[u] = -INFINITY;
        cmask[u] = 0u;
        if (i < nrows && c < R.KC) {  // not waiting for the take-part flag
            cmax[u] = R.pmax[(int64_t)c * R.M + i];
            cmask[u] = R.pmask[(int64_t)c * R.M + i];
        }
    }
    // the row's objectives (vector), also loaded beside the flag
    double rv[MD];
    float rf[MD];
#pragma unroll
    for (int k = 0; k < MD; ++k) {
        rv[k] = 0.0;
        rf[k] = 0.f;
        if (i < nrows) {
            if (GAMMA) {
                rv[k] = R.V[i * MD + k];
                rf[k] = R.V32[i * (MD <= 4 ? 4 : 8) + k];
            } else {
                rf[k] = fm_of(R, *R.t_done)[i * MD + k];
            }
        }
    }
    if (act) {
        double f[MD], nrm;
        float f32[MD];
        float n2f = 0.f;
#pragma unroll
        for (int k = 0; k < MD; ++k) {
            float fk;
            if (GAMMA) {
                f[k] = rv[k];
                fk = rf[k];
            } else {
                const float zk = ord_dec(zbuf(R, *R.t_done + 1)[k]);
                const float Fk = rf[k];
                f[k] = (double)Fk - (double)zk;
                fk = Fk - zk;
            }
            f32[k] = fk;
            n2f = fmaf(fk, fk, n2f);
        }
        if (GAMMA) {
            nrm = R.vn[i];
        } else {
            double n2 = f[0] * f[0];
#pragma unroll
            for (int k = 1; k < MD; ++k) n2 = fma(f[k], f[k], n2);
            nrm = sqrt(n2);
        }
        if (sub == 0) {
#pragma unroll
            for (int k = 0; k < MD; ++k) {
                s_f[r][k] = f[k];
                if (!GAMMA) s_f32[r][k] = f32[k];
            }
            s_nrm[r] = nrm;
        }
        state = (!GAMMA && nrm == 0.0) ? 2 : 1;
        float gm = fmaxf(fmaxf(cmax[0], cmax[1]), fmaxf(cmax[2], cmax[3]));
        for (int c = sub + kCache * kLanes; c < R.KC; c += kLanes)
            gm = fmaxf(gm, R.pmax[(int64_t)c * R.M + i]);
        thr = gm;
        if (!GAMMA) thr = gm - two_eps(sqrtf(n2f));
    }
    // a row's lanes are adjacent and aligned: combine within the group
    thr = group_max<kLanes>(thr);
    if (GAMMA && act && thr > -INFINITY) thr -= two_eps_dist(-thr);  // scores are -|v_i - v_j|^2
    // candidate tiles of this lane's chunks: those in registers, then any
    // further chunks (more than kCache per lane) read again
    bool more = false;
    if (act && state == 1) {
#pragma unroll
        for (int u = 0; u < kCache; ++u)
            if (cmax[u] >= thr) cnt += __popc(cmask[u]);
        for (int c = sub + kCache * kLanes; c < R.KC; c += kLanes) {
            if (R.pmax[(int64_t)c * R.M + i] >= thr) {
                more = true;
                cnt += __popc(R.pmask[(int64_t)c * R.M + i]);
            }
        }
    }
    const int tot = group_sum<kLanes>(cnt);
    if (act && state == 1 && (tot < 1 || tot > kItems)) state = 3;
    // exclusive prefix of the tile counts over the row's four lanes
    int pre = cnt;  // inclusive scan over the row's lanes, then exclusive
#pragma unroll
    for (int o = 1; o < kLanes; o <<= 1) {
        const int y = __shfl_up(pre, o, 64);
        if (sub >= o) pre += y;
    }
    pre -= cnt;
    if (sub == 0) {
        s_state[r] = act ? state : 0;
        s_cnt[r] = (act && state == 1) ? tot : 0;
        if (!GAMMA) {
            s_thr[r] = thr;
            s_rc[r] = 0;
        }
    }
    __syncthreads();
    if (t == 0) {  // rows' item offsets, in row order; a row beyond the wave's capacity scans in full
        int used = 0;
        for (int q = 0; q < kRows; ++q) {
            if (s_cnt[q] > 0 && used + s_cnt[q] > kWaveItems) {
                s_state[q] = 3;
                s_cnt[q] = 0;
            }
            s_off[q] = used;
            used += s_cnt[q];
        }
    }
    __syncthreads();
    const int total = s_off[kRows - 1] + s_cnt[kRows - 1];
    if (act && s_state[r] == 1) {
        int q = s_off[r] + pre;
        auto put = [&](int c, uint32_t mk) {
            while (mk) {
                const int tl = __ffs(mk) - 1;
                mk &= mk - 1;
                s_item[q++] = (r << 27) | (int)((int64_t)c * R.CS + (int64_t)tl * kTile);
            }
        };
#pragma unroll
        for (int u = 0; u < kCache; ++u)
            if (cmax[u] >= thr) put(sub + u * kLanes, cmask[u]);
        if (more) {
            for (int c = sub + kCache * kLanes; c < R.KC; c += kLanes)
                if (R.pmax[(int64_t)c * R.M + i] >= thr) put(c, R.pmask[(int64_t)c * R.M + i]);
        }
    }
    __syncthreads();

    __shared__ double s_rb[kRows], s_rg[kRows];
    __shared__ int s_rj[kRows], s_full[kRows];
    const int rounds = (total * kTile + 63) / 64;

    // ---- phase 2, selection rows: the candidate tiles' vectors are scored
    // in binary32 exactly as the association scored them (same f', same
    // binary32 vectors, same operations), and only those at or above the
    // row's threshold are kept: the binary64 maximum is among them (its
    // binary32 score is within 2 eps of the binary32 maximum, like the tiles
    // it lies in), and so is every vector tied with it.  Candidates are
    // appended in row order, so each row's are contiguous.  More than kCand
    // in the wave (vectors crowded below binary32 resolution), or more than
    // three candidate tiles per row on average (crowding again, decided before
    // any scoring): the tiles are taken whole instead, as for the gamma pass.
    bool tiles = GAMMA || total > 3 * kRows;
    if (!tiles) {
        constexpr int NV4 = MD <= 4 ? 1 : 2;
        const float4 *V4 = reinterpret_cast<const float4 *>(R.V32);
        int ncand = 0;  // uniform
        for (int k = 0; k < rounds; ++k) {
            const int e = t + 64 * k;
            const int item = e >> 5;
            bool keep = false;
            int code = 0, row = 0;
            if (item < total) {
                row = s_item[item] >> 27;
                const int64_t j = (int64_t)(s_item[item] & ((1 << 27) - 1)) + (e & 31);
                if (j < R.K) {
                    float4 v[NV4];
#pragma unroll
                    for (int q = 0; q < NV4; ++q) v[q] = V4[j * NV4 + q];
                    float fr[MD];
#pragma unroll
                    for (int kk = 0; kk < MD; ++kk) fr[kk] = s_f32[row][kk];
                    keep = dotf<MD>(fr, v) >= s_thr[row];
                    code = (row << 27) | (int)j;
                }
            }
            const unsigned long long b = __ballot(keep);
            const int pos = ncand + (int)__builtin_amdgcn_mbcnt_hi(
                                        (uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
            if (keep) {
                if (pos < kCand) s_cand[pos] = code;
                atomicAdd(&s_rc[row], 1);
            }
            ncand += __popcll(b);
        }
        tiles = ncand > kCand;  // uniform
        __syncthreads();
        if (!tiles) {
            // binary64 cosines of the candidates, one lane each
            for (int q = t; q < ncand; q += 64) {
                const int code = s_cand[q];
                const int row = code >> 27;
                const int64_t j = code & ((1 << 27) - 1);
                double f[MD];
#pragma unroll
                for (int kk = 0; kk < MD; ++kk) f[kk] = s_f[row][kk];
                s_cos[q] = dotd<MD>(f, R.V + j * MD) / (s_nrm[row] * R.vn[j]);
            }
            __syncthreads();
            // ---- phase 3, selection rows: one lane per row, the best of its
            // candidates (largest cosine, lowest index on ties)
            if (t < kRows) {
                const int st = s_state[t];
                double best = -INFINITY;
                int64_t bj = R.K;
                bool full = st == 3;
                if (st == 1) {
                    int o = 0;
                    for (int q = 0; q < t; ++q) o += s_rc[q];
                    for (int q = o; q < o + s_rc[t]; ++q) {
                        const double b2 = s_cos[q];
                        const int64_t j = s_cand[q] & ((1 << 27) - 1);
                        if (b2 > best || (b2 == best && j < bj)) {
                            best = b2;
                            bj = j;
                        }
                    }
                    if (bj >= R.K) full = true;
                }
                s_full[t] = full ? 1 : 0;
                s_rb[t] = best;
                s_rg[t] = bj < R.K ? R.gamma[bj] : 0.0;
                s_rj[t] = (int)bj;
            }
            __syncthreads();
        }
    }

    // ---- phase 2 (gamma rows, or crowded selection rows): flattened
    // (item, vector) space, 32 lanes per item, binary64 throughout
    for (int k = 0; tiles && k < rounds; ++k) {
        const int e = t + 64 * k;
        const int item = e >> 5;
        double best = -INFINITY, gam = 0.0;
        int64_t bj = R.K;
        int dup = 0;
        if (item < total) {
            const int row = s_item[item] >> 27;
            const int64_t j = (int64_t)(s_item[item] & ((1 << 27) - 1)) + (e & 31);
            const int64_t irow = base + row;
            if (j < R.K && (!GAMMA || j != irow)) {
                double f[MD];
#pragma unroll
                for (int kk = 0; kk < MD; ++kk) f[kk] = s_f[row][kk];
                // the vector's gamma comes in the same round trip as V and |v|
                if (!GAMMA) gam = R.gamma[j];
                const double cv = dotd<MD>(f, R.V + j * MD) / (s_nrm[row] * R.vn[j]);
                if (GAMMA && cv >= 1.0) {
                    dup = 1;
                } else {
                    best = cv;
                    bj = j;
                }
            }
        }
        best_level<0, GAMMA>(best, bj, gam, dup);
        best_level<1, GAMMA>(best, bj, gam, dup);
        best_level<2, GAMMA>(best, bj, gam, dup);
        best_level<3, GAMMA>(best, bj, gam, dup);
        best_level<4, GAMMA>(best, bj, gam, dup);
        if ((t & 31) == 0 && item < total) {
            s_best[item] = best;
            s_gam[item] = gam;
            s_bj[item] = (int)bj;
            s_dup[item] = dup;
        }
    }
    __syncthreads();

    // ---- phase 3: one lane per row merges its items
    if (tiles && t < kRows) {
        const int st = s_state[t];
        double best = -INFINITY, gam = 0.0;
        int64_t bj = R.K;
        bool full = st == 3;
        if (st == 1) {
            const int o = s_off[t], n = s_cnt[t];
            for (int q = o; q < o + n; ++q) {
                if (s_dup[q]) full = true;
                const double b = s_best[q];
                const int64_t j = s_bj[q];
                if (j < R.K && (b > best || (b == best && j < bj))) {
                    best = b;
                    bj = j;
                    gam = s_gam[q];
                }
            }
            if (bj >= R.K) full = true;
        }
        s_full[t] = full ? 1 : 0;
        s_rb[t] = best;
        s_rg[t] = gam;
        s_rj[t] = (int)bj;
    }
    __syncthreads();

    // ---- phase 4: rows left without a usable candidate set are scanned in
    // full by the whole wave: every vector in binary64, the maximum with the
    // lowest index (the plain definition), GAMMA skipping i = j and exactly
    // parallel vectors
    for (int rr = 0; rr < kRows; ++rr) {
        if (!s_full[rr]) continue;  // uniform
        const int64_t row_i = base + rr;
        double f[MD];
#pragma unroll
        for (int k = 0; k < MD; ++k) f[k] = s_f[rr][k];
        const double nrm = s_nrm[rr];
        double best = -INFINITY;
        int64_t bj = R.K;
        for (int64_t j = t; j < R.K; j += 64) {
            if (GAMMA && j == row_i) continue;
            const double cv = dotd<MD>(f, R.V + j * MD) / (nrm * R.vn[j]);
            if (GAMMA && cv >= 1.0) continue;
            if (cv > best) {
                best = cv;
                bj = j;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int64_t oj = __shfl_xor(bj, o, 64);
            if (ob > best || (ob == best && oj < bj)) {
                best = ob;
                bj = oj;
            }
        }
        if (t == 0) {
            atomicAdd(&R.counters[1], 1ull);
            s_rb[rr] = best;
            s_rj[rr] = (int)bj;
            if (!GAMMA) s_rg[rr] = bj < R.K ? R.gamma[bj] : R.gamma[0];
        }
    }
    __syncthreads();

    // ---- phase 5: one lane per row writes the result
    if (t >= kRows) return;
    const int64_t row_i = base + t;
    const int st = s_state[t];
    if (st == 0) {
        if (!GAMMA && row_i < R.M) {
            R.assoc[row_i] = -1;
            R.apd[row_i] = INFINITY;
        }
        return;
    }
    if (!GAMMA && st == 2) {
        R.assoc[row_i] = 0;
        R.apd[row_i] = 0.0;
        atomicMin(&R.key[0], (unsigned long long)row_i);  // APD 0
        return;
    }
    double best = s_rb[t];
    int64_t bj = s_rj[t];
    if (GAMMA) {  // no other vector: the angle to the nearest neighbour is taken as pi/2
        R.gamma[row_i] = bj < R.K ? acos(best < -1.0 ? -1.0 : best) : 1.5707963267948966;
        return;
    }
    // no finite cosine (cannot happen for a finite, nonzero row): vector 0
    const double gj = bj < R.K ? s_rg[t] : R.gamma[0];
    if (bj >= R.K) bj = 0;
    const double nrm = s_nrm[t];
    const double cc = best > 1.0 ? 1.0 : (best < -1.0 ? -1.0 : best);
    const double th = acos(cc);
    const double a = (1.0 + *R.pen * th / gj) * nrm;
    R.assoc[row_i] = (int32_t)bj;
    R.apd[row_i] = a;
    // (APD, row) in one word: the APD's bit pattern (monotone for doubles
    // >= 0) above the row index, its lowest kb bits dropped; the minimum
    // names the survivor directly, the lowest row among equal APDs
    const unsigned long long ab = (unsigned long long)__double_as_longlong(a);
    atomicMin(&R.key[bj], ((ab >> R.kb) << R.kb) | (unsigned long long)row_i);
}

// The new population g (Alg. 1) written into the other buffer of
// each pair: slot j <- its survivor's gene row and objectives, or empty; the
// survivor is the row index held in the vector's key.  The same pass stamps
// the rows generation g+1 will read, counts valid slots per block (the next
// preparation's offsets), reduces the survivors' extremes when an
// adaptation follows, and clears generation g+1's ideal point and free-row
// counter.
// The last workgroup to finish counts the generation (t_done = g): every
// workgroup has read t_done before it reports.
__device__ __forceinline__ void newpop_body(const RunView &R, int64_t bx)
{
    __shared__ uint32_t smin[kMaxM], smax[kMaxM];
    __shared__ int wc[4];
    const int64_t j = bx * 256 + threadIdx.x;
    // the vector's key does not depend on the generation counter: both load
    // together, then the survivor's row and objectives together
    const unsigned long long kj = j < R.K ? R.key[j] : ~0ull;
    const int64_t g = *R.t_done + 1;
    if (threadIdx.x < kMaxM) {
        smin[threadIdx.x] = 0xffffffffu;
        smax[threadIdx.x] = 0u;
    }
    if (bx == 0 && threadIdx.x < R.m) zbuf(R, g + 1)[threadIdx.x] = 0xffffffffu;
    if (bx == 0 && threadIdx.x == 0) *R.freecnt = 0;
    const int32_t *row0 = slot_row_of(R, g - 1);
    const float *F0 = fm_of(R, g - 1);
    int32_t *row1 = slot_row_of(R, g);
    uint8_t *val1 = valid_of(R, g);
    float *F1 = fm_of(R, g);
    const int64_t si = (int64_t)(kj & ((1ull << R.kb) - 1));
    const int v = (j < R.K && kj != ~0ull && si < R.M) ? 1 : 0;  // else no row for vector j
    const int32_t s = v ? (int32_t)si : 0;
    float fs[kMaxM];
    int32_t row = 0;
    if (v) {
        row = s < R.K ? row0[s] : R.off_row[s - R.K];
#pragma unroll
        for (int k = 0; k < kMaxM; ++k)
            if (k < R.m) fs[k] = F0[(int64_t)s * R.m + k];
    }
    __syncthreads();
    if (j < R.K) {
        if (!v) {
            R.surv[j] = -1;
            val1[j] = 0;
            row1[j] = row0[j];
        } else {
            R.surv[j] = s;
            val1[j] = 1;
            row1[j] = row;
            R.stamp[row] = (int32_t)(g + 1);
        }
    }
    // the survivors' extremes feed only an adaptation right after this
    // generation (g a multiple of the period): other generations skip the
    // reductions (uniform branch)
    const bool ext = g % R.period == 0;
#pragma unroll
    for (int k = 0; k < kMaxM; ++k) {
        if (k >= R.m) break;
        uint32_t e = 0xffffffffu;
        if (j < R.K) {
            const float x = v ? fs[k] : __int_as_float(0x7fc00000);
            F1[j * R.m + k] = x;
            if (v) e = ord_enc(x);
        }
        if (ext) {
            const uint32_t lo = wave_min(e);
            const uint32_t hi = wave_max(e == 0xffffffffu ? 0u : e);
            if ((threadIdx.x & 63) == 0) {
                if (lo != 0xffffffffu) atomicMin(&smin[k], lo);
                atomicMax(&smax[k], hi);
            }
        }
    }
    const unsigned long long b = __ballot(v);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (ext && threadIdx.x < R.m) {
        if (smin[threadIdx.x] != 0xffffffffu) atomicMin(&R.rbits[threadIdx.x], smin[threadIdx.x]);
        atomicMax(&R.rbits[R.m + threadIdx.x], smax[threadIdx.x]);
    }
    if (threadIdx.x == 0) {
        R.bcount[bx] = wc[0] + wc[1] + wc[2] + wc[3];
        // no fence: the last workgroup only writes t_done, and every
        // workgroup's read of it completed (its value was used by all waves
        // before the barrier above) before its own count was added
        const uint32_t nb = (uint32_t)((R.K + 255) / 256);
        if (atomicAdd(R.ndone, 1u) == nb - 1) {
            *R.t_done = g;
            *R.ndone = 0;
        }
    }
}

// ------------------------------------------------------- single-run kernels
template <int MD, int RR, bool GAMMA>
__global__ __launch_bounds__(256) void k_assoc(RunView R, int gate)
{
    assoc_body<MD, RR, GAMMA>(R, blockIdx.x, blockIdx.y, gate);
}
template <int MD, bool GAMMA, int ROWS>
__global__ __launch_bounds__(64) void k_rerank(RunView R, int gate)
{
    rerank_body<MD, GAMMA, ROWS>(R, blockIdx.x, gate);
}
__global__ __launch_bounds__(256) void k_newpop(RunView R) { newpop_body(R, blockIdx.x); }

// ----------------------------------------------------- batched (many runs)
// blockIdx.x is decoded into (run, local block) through the span table; for
// the association, local = chunk * row_blocks + row_block.
template <int MD, int RR, bool GAMMA>
__global__ __launch_bounds__(256) void kb_assoc(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    const int64_t local = blockIdx.x - sp[s].start;
    const int64_t nbx = sp[s].nbx;
    const RunView &R = runs[sp[s].run];
    // an indexed run's gamma pass also needs its index build to have asked
    assoc_body<MD, RR, GAMMA>(R, local % nbx, (int)(local / nbx), R.gG > 0 ? 2 : 0);
}
template <int MD, bool GAMMA>
__global__ __launch_bounds__(64) void kb_rerank(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    const RunView &R = runs[sp[s].run];
    rerank_body<MD, GAMMA, kBatchRows>(R, blockIdx.x - sp[s].start, R.gG > 0 ? 2 : 0);
}
// the batched gamma passes, U blocks per workgroup (U = kSkipBlocks when
// the launch has blocks enough to fill the device U times over: most
// generations skip them; else 1, so that a few runs' pass keeps its
// parallelism in the generations that run it)
template <int MD, int RR, int U>
__global__ __launch_bounds__(256) void kb_gamma_assoc(const RunView *runs, const Span *sp, int n,
                                                      int64_t total)
{
    span_blocks<U>(runs, sp, n, total, gamma_open, [](const RunView &R, int64_t local, int nbx) {
        assoc_body<MD, RR, true>(R, local % nbx, (int)(local / nbx), 1);
    });
}
// (with U > 1 the re-rank body is called, not inlined: inlined U times it
// would keep several times the registers live)
template <int MD>
__device__ __attribute__((noinline)) void gamma_rerank_call(const RunView &R, int64_t local)
{
    rerank_body<MD, true, kBatchRows>(R, local, 1);
}
template <int MD, int U>
__global__ __launch_bounds__(64) void kb_gamma_rerank(const RunView *runs, const Span *sp, int n,
                                                      int64_t total)
{
    span_blocks<U>(runs, sp, n, total, gamma_open, [](const RunView &R, int64_t local, int) {
        if constexpr (U == 1)
            rerank_body<MD, true, kBatchRows>(R, local, 1);
        else
            gamma_rerank_call<MD>(R, local);
    });
}
__global__ __launch_bounds__(256) void kb_newpop(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    newpop_body(runs[sp[s].run], blockIdx.x - sp[s].start);
}

// ------------------------------------------------------------- launchers
static unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

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

// association launch with R.rr rows per lane (1, 2 or 4) and R.KC chunks
template <bool GAMMA>
static void assoc_launch(const RunView &R, hipStream_t s, int gate)
{
    const int64_t rows = GAMMA ? R.K : R.M;
#define RVEA_ASSOC(MV)                                                                       \
    switch (R.rr) {                                                                          \
    case 1:                                                                                  \
        k_assoc<MV, 1, GAMMA><<<dim3(blocks(rows, 256), (unsigned)R.KC), 256, 0, s>>>(R, gate); \
        break;                                                                               \
    case 2:                                                                                  \
        k_assoc<MV, 2, GAMMA><<<dim3(blocks(rows, 512), (unsigned)R.KC), 256, 0, s>>>(R, gate); \
        break;                                                                               \
    default:                                                                                 \
        k_assoc<MV, 4, GAMMA><<<dim3(blocks(rows, 1024), (unsigned)R.KC), 256, 0, s>>>(R, gate); \
        break;                                                                               \
    }
    RVEA_M_DISPATCH(R.m, RVEA_ASSOC);
#undef RVEA_ASSOC
}

hipError_t launch_assoc(const RunView &R, hipStream_t s)
{
    if (R.gG > 0) return launch_assoc_grid(R, s);  // indexed: the re-rank is folded in
    assoc_launch<false>(R, s, 1);
    return hipGetLastError();
}

// re-rank launch with R.rk rows per wave (4, 8 or 16)
template <bool GAMMA>
static void rerank_launch(const RunView &R, hipStream_t s, int gate)
{
    const int64_t rows = GAMMA ? R.K : R.M;
#define RVEA_RERANK(MV)                                                                      \
    switch (R.rk) {                                                                          \
    case 4: k_rerank<MV, GAMMA, 4><<<blocks(rows, 4), 64, 0, s>>>(R, gate); break;           \
    case 8: k_rerank<MV, GAMMA, 8><<<blocks(rows, 8), 64, 0, s>>>(R, gate); break;           \
    default: k_rerank<MV, GAMMA, 16><<<blocks(rows, 16), 64, 0, s>>>(R, gate); break;        \
    }
    RVEA_M_DISPATCH(R.m, RVEA_RERANK);
#undef RVEA_RERANK
}

hipError_t launch_rerank(const RunView &R, hipStream_t s)
{
    if (R.gG > 0) return hipSuccess;
    rerank_launch<false>(R, s, 1);
    return hipGetLastError();
}

// gamma of Eq. 5 through the same two passes, rows = vectors, with the
// gamma pass's own chunking and rows per lane
hipError_t launch_gamma(const RunView &R, hipStream_t s, int force)
{
    RunView G = R;
    G.KC = R.gKC;
    G.CS = R.gCS;
    G.rr = R.grr;
    assoc_launch<true>(G, s, force);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    rerank_launch<true>(G, s, force);
    return hipGetLastError();
}

hipError_t launch_select_back(const RunView &R, hipStream_t s)
{
    k_newpop<<<blocks(R.K, 256), 256, 0, s>>>(R);
    return hipGetLastError();
}

int assoc_rows_per_block() { return 256 * 4; }
int rerank_rows_per_wave() { return kBatchRows; }

int default_rerank_rows(int64_t rows)
{
    // enough waves to hide latency: about 8 per SIMD of the 1,024 at 16 rows
    return rows >= 131072 ? 16 : (rows >= 12288 ? 8 : 4);
}

hipError_t launch_batch_select(int phase, int cls, const RunView *runs, const Span *sp, int n,
                               int64_t blocks, hipStream_t s)
{
    constexpr int RR = 4;
    const dim3 g((unsigned)blocks);
    switch (phase) {
    case BP_NEWPOP: kb_newpop<<<g, 256, 0, s>>>(runs, sp, n); break;
    case BP_ASSOC:
#define RVEA_BA(MV) kb_assoc<MV, RR, false><<<g, 256, 0, s>>>(runs, sp, n)
        RVEA_M_DISPATCH(cls, RVEA_BA);
#undef RVEA_BA
        break;
    case BP_RERANK:
#define RVEA_BR(MV) kb_rerank<MV, false><<<g, 64, 0, s>>>(runs, sp, n)
        RVEA_M_DISPATCH(cls, RVEA_BR);
#undef RVEA_BR
        break;
    case BP_GAMMA_ASSOC:
    case BP_GAMMA_RERANK: {
        const bool wide = blocks >= (int64_t)kSkipBlocks * kFillBlocks;
        const dim3 gw((unsigned)(wide ? (blocks + kSkipBlocks - 1) / kSkipBlocks : blocks));
        if (phase == BP_GAMMA_ASSOC) {
#define RVEA_BGA(MV)                                                                   \
    (wide ? kb_gamma_assoc<MV, RR, kSkipBlocks><<<gw, 256, 0, s>>>(runs, sp, n, blocks) \
          : kb_gamma_assoc<MV, RR, 1><<<gw, 256, 0, s>>>(runs, sp, n, blocks))
            RVEA_M_DISPATCH(cls, RVEA_BGA);
#undef RVEA_BGA
        } else {
#define RVEA_BGR(MV)                                                                \
    (wide ? kb_gamma_rerank<MV, kSkipBlocks><<<gw, 64, 0, s>>>(runs, sp, n, blocks) \
          : kb_gamma_rerank<MV, 1><<<gw, 64, 0, s>>>(runs, sp, n, blocks))
            RVEA_M_DISPATCH(cls, RVEA_BGR);
#undef RVEA_BGR
        }
        break;
    }
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace rvea
