// rvea_index.h -- the cell of a reference vector (or a row direction) in
// the association index: a G x G grid over the scaled simplex for three
// objectives, a line of G cells for two.  Shared by the index build
// (k_grid.hip) and the adaptation, which counts each adapted vector into
// its cell as it writes it (k_vectors.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace rvea {

// cell of a direction x >= 0 (x != 0); q pulled onto the simplex if rounding
// left it just outside.  -1 if the coordinates are not finite.
__device__ __forceinline__ int cell_of(double x0, double x1, double x2, const double *r, int G)
{
    const double y0 = x0 / r[0], y1 = x1 / r[1], y2 = x2 / r[2];
    const double s = y0 + y1 + y2;
    double q1 = y0 / s, q2 = y1 / s;
    if (!(q1 >= 0.0 && q2 >= 0.0 && q1 <= 2.0 && q2 <= 2.0)) return -1;
    const double t = q1 + q2;
    if (t > 1.0) {
        q1 /= t;
        q2 /= t;
    }
    int ci = (int)floor(q1 * G), cj = (int)floor(q2 * G);
    ci = ci < 0 ? 0 : (ci > G - 1 ? G - 1 : ci);
    cj = cj < 0 ? 0 : (cj > G - 1 ? G - 1 : cj);
    return ci * G + cj;
}

// share u of a direction x on the scaled simplex and its cell; -1 unless
// both components are >= 0 and finite with a positive sum
__device__ __forceinline__ int line_cell_of(double x0, double x1, const double *r, int G,
                                            double &u)
{
    const double a = x0 / r[0], b = x1 / r[1];
    const double s = a + b;
    u = b / s;
    if (!(a >= 0.0 && b >= 0.0 && s > 0.0 && s <= 1.79e308 && u >= 0.0 && u <= 1.0))
        return -1;
    const int c = (int)(u * G);
    return c < G ? c : G - 1;
}

}  // namespace rvea
