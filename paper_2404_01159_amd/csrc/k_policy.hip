// k_policy.hip -- the policy-rollout problem (m = 2, d = 6,728): Gaussian
// initialization of the policy weights and evaluation of a population of
// 32 -> 64 -> 64 -> 8 tanh policies by rollouts on a linear system.
//
// Genes of one individual (row-major matrices, [out][in]):
//   W1 64x32 at 0, b1 64 at 2048, W2 64x64 at 2112 (no bias), W3 8x64 at 6208,
//   b3 8 at 6720.
// For each of E = 16 start states x0[e], T steps of
//   u = tanh(W3 tanh(W2 tanh(W1 x + b1)) + b3),   x <- A x + B u,
// with f1 = sum_t |x_t|^2 (t = 1..T) and f2 = sum_t |u_t|^2 (t = 0..T-1), both
// averaged over the E rollouts.  Weight matrices and layer inputs are bfloat16
// (round to nearest even), products accumulate in binary32 on the matrix
// cores; biases and the state stay binary32.  The dynamics also run on the
// matrix cores: each binary32 operand a is split into bfloat16 parts
// a_hi = bf16(a), a_lo = bf16(a - a_hi), and A x is accumulated as
// A_hi x_hi + A_lo x_hi + A_hi x_lo (relative error about 2^-17 per product,
// against 2^-24 for binary32 products at four times the matrix-core time).
//
// One wavefront evaluates one individual with its 16 rollouts as the N = 16
// columns of every product: each layer is W . H^T, so the layer's output (the
// MFMA accumulator: lane l holds rows 4(l/16)..+3 of column l%16) is already
// the next product's B operand once two output tiles are packed to
// bfloat16, provided the weights are loaded with the matching permutation of
// the contraction index.  Nothing crosses lanes inside the 200-step loop.
#include <hip/hip_runtime.h>

#include "rvea_dev.h"
#include "rvea_internal.h"

namespace rvea {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));

constexpr int kW1 = 0, kB1 = 2048, kW2 = 2112, kW3 = 6208, kB3 = 6720;
static_assert(kB3 + 8 == kPolicyD, "policy gene layout");

// eight binary32 values to bfloat16 (v_cvt_pk_bf16_f32, round to nearest even)
__device__ __forceinline__ bf16x8 to_bf16(f32x4 lo, f32x4 hi)
{
    const f32x8 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_convertvector(v, bf16x8);
}

// the four low / high bfloat16 lanes of a pack, widened (exactly) to binary32
__device__ __forceinline__ f32x4 lo4(bf16x8 v)
{
    return f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
}
__device__ __forceinline__ f32x4 hi4(bf16x8 v)
{
    return f32x4{(float)v[4], (float)v[5], (float)v[6], (float)v[7]};
}

__device__ __forceinline__ f32x4 ld4(const float *p)
{
    const float4 v = *reinterpret_cast<const float4 *>(p);
    return f32x4{v.x, v.y, v.z, v.w};
}

// tanh(x) = 1 - 2 / (exp(2x) + 1) with the hardware exp2 and reciprocal
// (saturates to +-1, tanh(0) = 0 exactly)
__device__ __forceinline__ float tanh_f(float x)
{
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // 2 log2(e)
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

__device__ __forceinline__ f32x4 tanh4(f32x4 v)
{
    return f32x4{tanh_f(v[0]), tanh_f(v[1]), tanh_f(v[2]), tanh_f(v[3])};
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Rollout evaluation of n individuals, one wavefront each, four per block:
// the offspring of the current generation (offspring = 1: genes in rows
// off_row[q], objectives into the merged rows K + q; a generation without
// valid parents wrote no offspring and is skipped) or the initial population
// (offspring = 0: slot q of population 0).
//
// Registers hold the weight matrices, b3 and the state; the dynamics
// operands (shared by the block) and b1 (per wavefront) sit in LDS and are
// re-read every step, which keeps the wavefront within 128 registers, i.e.
// four wavefronts per SIMD: the 4,096 individuals of a generation are then
// resident at once on 256 CUs.
constexpr int kRollWaves = 4;
struct RolloutLds {
    bf16x8 ab[8][64];  // dynamics operands: (A tile 0, A tile 1, B tile 0, B tile 1) x (hi, lo)
    f32x4 b1[kRollWaves][4][4];       // b1 rows 16m+4g..+3 per (m, g)
};

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_rollout(RunView R, int64_t n, int offspring)
{
    const int check_nv = offspring;
    const int32_t *rows = offspring ? R.off_row : slot_row_of(R, 0);
    float *F = offspring ? fm_of(R, *R.t_done) + R.K * R.m : fm_of(R, 0);
    __shared__ RolloutLds sh;
    const int wv = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * kRollWaves + wv;
    const bool active = q < n && !(check_nv && *R.nvalid == 0);
    const int l = threadIdx.x & 63;
    const int c = l & 15;  // MFMA row of the A operand / column (rollout) of B and D
    const int g = l >> 4;  // lane group: k-slots 8g..8g+7 of A and B, rows 4g..4g+3 of D
    const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};

    // Dynamics operands, split into bfloat16 high and low parts.  Output
    // tile `to` holds state rows 16to..16to+15.  The state part contracts
    // over the 32 state entries in the layer-1 slot order (slot e of group g
    // is entry 4g+e or 16+4g+(e-4)); the input part over the 8 entries of u,
    // which lane groups 0, 1 hold as slots 0..3 (entry 4g+e), every other
    // slot zero.
    const float *A = R.lq, *B = R.lq + 1024, *x0 = R.lq + 1280;
    for (int idx = threadIdx.x; idx < 8 * 64; idx += 256) {
        const int k = idx >> 6, ll = idx & 63, cc = ll & 15, gg = ll >> 4;
        const int to = (k >> 1) & 1;
        f32x4 v0 = z4, v1 = z4;
        if (k < 4) {
            v0 = ld4(A + (16 * to + cc) * 32 + 4 * gg);
            v1 = ld4(A + (16 * to + cc) * 32 + 16 + 4 * gg);
        } else if (gg < 2) {
            v0 = ld4(B + (16 * to + cc) * 8 + 4 * gg);
        }
        const bf16x8 hi = to_bf16(v0, v1);
        sh.ab[k][ll] = (k & 1) ? to_bf16(v0 - lo4(hi), v1 - hi4(hi)) : hi;
    }

    // Weight operands.  Contraction slot e of lane group g stands for input
    // 4g+e (e < 4) or 16+4g+(e-4) (e >= 4) of a 32-wide chunk: the inputs
    // that lane group holds in two consecutive output tiles of the layer
    // before.
    const float *w = R.X + (int64_t)(active ? rows[q] : 0) * R.ld;
    bf16x8 w1[4], w2[4][2], w3[2];
    f32x4 b3 = z4;
    if (active) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const float *p = w + kW1 + (16 * m + c) * 32 + 4 * g;
            w1[m] = to_bf16(ld4(p), ld4(p + 16));
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                const float *p2 = w + kW2 + (16 * m + c) * 64 + 32 * kc + 4 * g;
                w2[m][kc] = to_bf16(ld4(p2), ld4(p2 + 16));
            }
            if (c == 0) sh.b1[wv][m][g] = ld4(w + kB1 + 16 * m + 4 * g);
        }
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
            const float *p3 = w + kW3 + c * 64 + 32 * kc + 4 * g;
            w3[kc] = c < 8 ? to_bf16(ld4(p3), ld4(p3 + 16)) : to_bf16(z4, z4);
        }
        if (g < 2) b3 = ld4(w + kB3 + 4 * g);
    }
    __syncthreads();
    if (!active) return;  // uniform per wavefront

    // state of rollout c: xs[T][r] = x[16T+4g+r]
    f32x4 xs[2];
    xs[0] = ld4(x0 + c * 32 + 4 * g);
    xs[1] = ld4(x0 + c * 32 + 16 + 4 * g);

    double f1 = 0.0, f2 = 0.0;
    const int T = R.lq_T;
    for (int t = 0; t < T; ++t) {
        // LDS operands are re-read each step rather than held in registers
        asm volatile("" ::: "memory");
        // layer 1: 64 x 32 . 32 x 16
        const bf16x8 xb = to_bf16(xs[0], xs[1]);
        f32x4 h[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            h[m] = tanh4(__builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[m], xb, sh.b1[wv][m][g], 0,
                                                                  0, 0));
        // layer 2: 64 x 64 . 64 x 16
        const bf16x8 hb0 = to_bf16(h[0], h[1]), hb1 = to_bf16(h[2], h[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[m][0], hb0, z4, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[m][1], hb1, a, 0, 0, 0);
            h[m] = tanh4(a);
        }
        // layer 3: 8 (padded to 16) x 64 . 64 x 16
        const bf16x8 gb0 = to_bf16(h[0], h[1]), gb1 = to_bf16(h[2], h[3]);
        f32x4 u = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3[0], gb0, b3, 0, 0, 0);
        u = tanh4(__builtin_amdgcn_mfma_f32_16x16x32_bf16(w3[1], gb1, u, 0, 0, 0));
        float su = u[0] * u[0];
        su = fmaf(u[1], u[1], su);
        su = fmaf(u[2], u[2], su);
        su = fmaf(u[3], u[3], su);
        f2 += (double)su;
        // dynamics: x <- A x + B u as three bfloat16 products per operand pair
        const bf16x8 xlo = to_bf16(xs[0] - lo4(xb), xs[1] - hi4(xb));
        const bf16x8 uhi = to_bf16(u, z4);
        const bf16x8 ulo = to_bf16(u - lo4(uhi), z4);
        f32x4 xn[2];
#pragma unroll
        for (int to = 0; to < 2; ++to) {
            const bf16x8 ah = sh.ab[2 * to][l], al = sh.ab[2 * to + 1][l];
            const bf16x8 bh = sh.ab[4 + 2 * to][l], bl = sh.ab[5 + 2 * to][l];
            f32x4 a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xb, z4, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, xb, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, xlo, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, uhi, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, uhi, a, 0, 0, 0);
            xn[to] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, ulo, a, 0, 0, 0);
        }
        xs[0] = xn[0];
        xs[1] = xn[1];
        float sx = xs[0][0] * xs[0][0];
#pragma unroll
        for (int r = 1; r < 4; ++r) sx = fmaf(xs[0][r], xs[0][r], sx);
#pragma unroll
        for (int r = 0; r < 4; ++r) sx = fmaf(xs[1][r], xs[1][r], sx);
        f1 += (double)sx;
    }
    f1 = wave_sum(f1);
    f2 = wave_sum(f2);
    const float fv[2] = {(float)(f1 / (double)R.lq_E), (float)(f2 / (double)R.lq_E)};
    if (l == 0) {
        F[2 * q] = fv[0];
        F[2 * q + 1] = fv[1];
    }
    // offspring: rows that take part and the ideal point of this generation
    if (check_nv) child_ideal(R, *R.t_done + 1, l == 0, R.K + q, fv);
}

// Gaussian initialization of rows 0..N-1: genes 4p..4p+3 of individual i
// from the Philox words of counter (p, i, 0, TAG_INIT), two Box-Muller pairs
// (u1 = (top 24 bits + 1) / 2^24 in (0,1], u2 = top 24 bits / 2^24):
// sigma * sqrt(-2 ln u1) * (cos, sin)(2 pi u2), clipped to the bounds, in
// binary64 and rounded once.  One thread per four genes.
__global__ __launch_bounds__(256) void k_init_gauss(RunView R)
{
    const int Q = (R.d + 3) / 4;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= R.N * (int64_t)Q) return;
    const int64_t i = idx / Q;
    const int p = (int)(idx - i * Q);
    const W4 wd = draw(R, (uint32_t)p, (uint32_t)i, 0u, TAG_INIT);
    double z[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double u1 = (double)((wd.w[2 * h] >> 8) + 1u) * 0x1p-24;
        const double u2 = (double)(wd.w[2 * h + 1] >> 8) * 0x1p-24;
        const double rr = sqrt(-2.0 * log(u1));
        const double a = (2.0 * M_PI) * u2;
        double s, co;
        sincos(a, &s, &co);
        z[2 * h] = rr * co;
        z[2 * h + 1] = rr * s;
    }
    float *row = R.X + i * (int64_t)R.ld + 4 * p;
    float x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = (float)dclip(R.lq_sigma * z[k], R.lb, R.ub);
    *reinterpret_cast<float4 *>(row) = make_float4(x[0], x[1], x[2], x[3]);  // 4p+4 <= ld
    if (p == 0) {
        R.valids[i] = 1;  // population 0
        R.slot_rows[i] = (int32_t)i;
    }
}

hipError_t launch_init_gauss(const RunView &R, hipStream_t s)
{
    const int64_t units = R.N * (int64_t)((R.d + 3) / 4);
    k_init_gauss<<<dim3((unsigned)((units + 255) / 256)), 256, 0, s>>>(R);
    return hipGetLastError();
}

hipError_t launch_rollout(const RunView &R, hipStream_t s, bool offspring)
{
    const int64_t n = R.N;
    const dim3 grid((unsigned)((n + kRollWaves - 1) / kRollWaves));
    if (offspring)
        k_rollout<<<grid, 256, 0, s>>>(R, n, 1);
    else
        k_rollout<<<grid, 256, 0, s>>>(R, n, 0);
    return hipGetLastError();
}

}  // namespace rvea
