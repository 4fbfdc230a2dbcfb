// rvea_problems.h -- device evaluation of the library's test problems
// (Eq. 1 instances).  Single precision, as the offspring's objectives are
// stored; the per-gene distance terms are summed in double.
//
// Problem shape (ids as in rvea.h): the first m-1 variables, sorted, give the
// uniform-spacings simplex point w; the other k = d-m+1 variables z give a
// distance term g >= 0 that vanishes at z = 1/2; f = (1+g) w (linear front)
// or (1+g) w/|w| (sphere front).
#pragma once

#include "rvea_dev.h"

namespace rvea {

// 2 sin^2(pi x) = 1 - cos(2 pi x), with the hardware cosine (its argument in
// revolutions): measured absolute error below 1.3e-7 for |x| <= 2 against
// binary64, and the term enters the objectives as (1 + g), so their relative
// error from it stays below 2e-7
__device__ __forceinline__ float two_sin2pi(float x) { return 1.0f - __builtin_amdgcn_cosf(x); }

// distance term of one variable (before averaging)
__device__ __forceinline__ float dist_term(int problem, float z)
{
    const float t = z - 0.5f;
    if (problem == 2) return t * t;
    return 10.0f * (t * t) + two_sin2pi(4.0f * t);
}

// objectives from the m-1 position variables and the summed distance terms
__device__ __forceinline__ void finish_objectives(int problem, int m, int d, const float *pos,
                                                  double gsum, float *f)
{
    float y[kMaxM];
    for (int i = 0; i < m - 1; ++i) y[i] = pos[i];
    for (int i = 1; i < m - 1; ++i) {  // insertion sort, m-1 <= 7
        const float v = y[i];
        int j = i - 1;
        while (j >= 0 && y[j] > v) {
            y[j + 1] = y[j];
            --j;
        }
        y[j + 1] = v;
    }
    float w[kMaxM];
    w[0] = y[0];
    for (int i = 1; i < m - 1; ++i) w[i] = y[i] - y[i - 1];
    w[m - 1] = 1.0f - y[m - 2];
    const double k = (double)(d - m + 1);
    const float g = (problem == 2) ? (float)(4.0 * gsum / k) : (float)(gsum / k);
    const float s = 1.0f + g;
    if (problem == 1) {
        for (int i = 0; i < m; ++i) f[i] = s * w[i];
    } else {
        float n2 = w[0] * w[0];
        for (int i = 1; i < m; ++i) n2 = fmaf(w[i], w[i], n2);
        const float nrm = sqrtf(n2);
        for (int i = 0; i < m; ++i) f[i] = s * (w[i] / nrm);
    }
}

}  // namespace rvea
